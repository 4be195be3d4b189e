"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Tolerances: factors and single applications / SpMVs
relative 1e-12 (max-abs error over max-abs value, per factor); FP64 solves
to rtol 1e-8 within relative 1e-10 of the oracle's solution and +-1
iteration; FP32-factor and multi-RHS solves converge to 1e-8."""
import numpy as np
import pytest
import torch

from paper_1703_01325_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1703_01325_amd import api as A
    return A


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


class Case:
    def __init__(self, O, sysm, k, transpose=False):
        self.s = sysm
        self.k = k
        self.O = O.OracleILU(sysm.nb, sysm.bs, sysm.Ap, sysm.Aj, k).factor(sysm.Ax)
        self.Ax = cuda(sysm.Ax)
        self.rhs = O.spmv(sysm.nb, sysm.bs, sysm.Ap, sysm.Aj, sysm.Ax, sysm.xstar)

    def gpu(self, api, transpose=False, precision="fp64", mode=2, tile_rows=None):
        M = api.BlockILU(self.s.nb, self.s.bs, self.s.Ap, self.s.Aj, self.k, transpose=transpose)
        M.tune(mode=mode, tile_rows=tile_rows)
        bad = M.factor(self.Ax, precision=precision)
        assert bad == -1
        return M


def small_cases():
    out = [("cube10_b3", lambda: synth.small_10cube(), 0),
           ("cube10_b3", lambda: synth.small_10cube(), 1)]
    for bs in (1, 2, 4, 5, 6, 7, 8):
        out.append((f"grid_b{bs}", (lambda b: (lambda: synth.reservoir(7, 6, 5, b, seed=30 + b)))(bs), 1))
    out.append(("ragged_b3_k2", lambda: synth.reservoir(13, 3, 11, 3, seed=44), 2))
    return out


SMALL = small_cases()


def factor_parts(O, s, F):
    rows = np.repeat(np.arange(s.nb), np.diff(O.Pp))
    bb = s.bs * s.bs
    Fm = np.asarray(F).reshape(-1, bb)
    return Fm[O.Pj < rows], Fm[O.Pj > rows]


@pytest.mark.parametrize("name,make,k", SMALL, ids=[f"{c[0]}_k{c[2]}" for c in SMALL])
def test_factor_parity(api, oracle_mod, name, make, k):
    c = Case(oracle_mod, make(), k)
    M = c.gpu(api)
    F, D = M.factors()
    F, D = F.cpu().numpy(), D.cpu().numpy()
    gL, gU = factor_parts(c.O, c.s, F)
    oL, oU = factor_parts(c.O, c.s, c.O.F)
    if oL.size:
        assert rel(gL, oL) <= 1e-12
        assert rel(gU, oU) <= 1e-12
    assert rel(D, c.O.Dinv) <= 1e-12


def test_factor_long_rows(api, oracle_mod):
    """Full fill (k = nb) of a random pattern with b = 8: the first level's
    row fits the LDS budget of the LDS factorisation kernel, the longer rows
    after it take the merge-walking kernel; factors and an application are
    checked against the oracle."""
    from types import SimpleNamespace
    nb, bs, k = 48, 8, 48
    Ap, Aj = synth.random_block_pattern(nb, 0.15, seed=91)
    Ax = synth.random_block_values(Ap, Aj, bs, seed=92)
    O = oracle_mod.OracleILU(nb, bs, Ap, Aj, k).factor(Ax)
    M = api.BlockILU(nb, bs, Ap, Aj, k)
    assert M.factor(cuda(Ax)) == -1
    F, D = M.factors()
    s = SimpleNamespace(nb=nb, bs=bs)
    gL, gU = factor_parts(O, s, F.cpu().numpy())
    oL, oU = factor_parts(O, s, O.F)
    assert rel(gL, oL) <= 1e-12 and rel(gU, oU) <= 1e-12
    assert rel(D.cpu().numpy(), O.Dinv) <= 1e-12
    r = np.random.default_rng(93).standard_normal(nb * bs)
    assert rel(M.apply(cuda(r)).cpu().numpy(), O.apply(r)) <= 1e-12
    M.check()


FACTOR_CASES = SMALL + [("ragged_b1_k3", lambda: synth.reservoir(13, 3, 11, 1, seed=45), 3),
                        ("res7x6x5_b4_k2", lambda: synth.reservoir(7, 6, 5, 4, seed=47), 2),
                        ("res7x6x5_b8_k2", lambda: synth.reservoir(7, 6, 5, 8, seed=48), 2),
                        ("layered60x220x85", lambda: synth.layered_60x220x85(), 0),
                        ("layered60x220x85", lambda: synth.layered_60x220x85(), 1),
                        ("mid64", lambda: synth.mid_64cube(), 2),
                        # rows of up to 31, 41 and 92 KiB: two, two and one
                        # wavefront per workgroup of the persistent launch;
                        # up to 119 KiB: the A_pj blocks staged a run of
                        # pivots at a time
                        ("poisson16x10x10_b4_k3", lambda: synth.poisson7(10, 4, nx=16), 3),
                        ("poisson24x10x10_b8_k2", lambda: synth.poisson7(10, 8, nx=24), 2),
                        ("poisson24x8x8_b8_k3", lambda: synth.poisson7(8, 8, nx=24), 3),
                        ("poisson32x10x10_b8_k3", lambda: synth.poisson7(10, 8, nx=32), 3)]


@pytest.mark.parametrize("name,make,k", FACTOR_CASES, ids=[f"{c[0]}_k{c[2]}" for c in FACTOR_CASES])
def test_factor_waves_match_levels(api, name, make, k):
    """The persistent factorisation (a wavefront per row, rows waiting for
    their pivot rows' finished blocks) and one launch per L level run the
    same arithmetic: the same bits, also after a refactorisation with other
    values (P and D^{-1} restart at kNotReady each time)."""
    s = make()
    print(f"[factor] {name} k={k}", flush=True)
    Ax = cuda(s.Ax)
    Ax2 = cuda(s.Ax * (1.0 + 0.25 * np.cos(np.arange(s.Ax.size))))
    A = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, k)
    B = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, k)
    try:
        A.tune(factor="levels")
        for mode in ("waves", "waves16", "waves4"):
            B.tune(factor=mode)
            for vals in (Ax, Ax2):
                assert A.factor(vals) == -1
                assert B.factor(vals) == -1
                FA, DA = A.factors()
                FB, DB = B.factors()
                assert torch.equal(FA, FB) and torch.equal(DA, DB), mode
    finally:
        A.close()
        B.close()


def test_factor_waves_timeout_reported(api):
    """The persistent factorisation with its bounded waits cut to one poll
    (forced from the host; every wavefront still finishes its rows and the
    launch drains) reports the expired wait as BILU_ERR_TIMEOUT; with the
    default limit back, the next factorisation gives the bits of one launch
    per level."""
    from paper_1703_01325_amd import _native as N
    s = synth.layered_60x220x85()
    print("[factor timeout] 60x220x85 k=0 spin_limit=1", flush=True)
    Ax = cuda(s.Ax)
    A = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 0)
    B = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 0)
    try:
        B.tune(factor="waves", spin_limit=1)
        with pytest.raises(N.BiluError) as err:
            B.factor(Ax)
        assert err.value.code == N.ERR_TIMEOUT
        B.tune(spin_limit=0)
        A.tune(factor="levels")
        assert A.factor(Ax) == -1
        assert B.factor(Ax) == -1
        FA, DA = A.factors()
        FB, DB = B.factors()
        assert torch.equal(FA, FB) and torch.equal(DA, DB)
        with pytest.raises(N.BiluError):
            B.tune(spin_limit=-1)
    finally:
        A.close()
        B.close()


MODES = [(0, None), (1, None), (2, None), (2, 1), (2, 13), (2, 64)]


@pytest.mark.parametrize("mode,tile_rows", MODES,
                         ids=["per_level", "level_chunks", "tiled", "tiled1", "tiled13", "tiled64"])
@pytest.mark.parametrize("name,make,k", SMALL, ids=[f"{c[0]}_k{c[2]}" for c in SMALL])
def test_apply_and_spmv_parity(api, oracle_mod, name, make, k, mode, tile_rows):
    c = Case(oracle_mod, make(), k)
    M = c.gpu(api, transpose=True, mode=mode, tile_rows=tile_rows)
    rng = np.random.default_rng(7)
    r = rng.standard_normal(c.s.n)
    z = M.apply(cuda(r)).cpu().numpy()
    assert rel(z, c.O.apply(r)) <= 1e-12
    zt = M.apply(cuda(r), transpose=True).cpu().numpy()
    assert rel(zt, c.O.apply(r, transpose=True)) <= 1e-12
    y = M.spmv(c.Ax, cuda(r)).cpu().numpy()
    assert rel(y, oracle_mod.spmv(c.s.nb, c.s.bs, c.s.Ap, c.s.Aj, c.s.Ax, r)) <= 1e-12
    yt = M.spmv(c.Ax, cuda(r), transpose=True).cpu().numpy()
    assert rel(yt, oracle_mod.spmv(c.s.nb, c.s.bs, c.s.Ap, c.s.Aj, c.s.Ax, r, True)) <= 1e-12
    M.check()


def test_apply_deterministic_across_modes(api, oracle_mod):
    """Every schedule computes each row with the same arithmetic in the same
    order, so all modes and repeated runs agree bit for bit."""
    c = Case(oracle_mod, synth.small_10cube(), 1)
    M = c.gpu(api, transpose=True)
    r = cuda(np.random.default_rng(1).standard_normal(c.s.n))
    z1 = M.apply(r)
    z1t = M.apply(r, transpose=True)
    for mode, tile in MODES:
        M.tune(mode=mode, tile_rows=tile)
        for _ in range(2):
            assert torch.equal(M.apply(r), z1)
            assert torch.equal(M.apply(r, transpose=True), z1t)
    M.check()


@pytest.mark.parametrize("R", [2, 8, 13, 32])
def test_multi_rhs_columns(api, oracle_mod, R):
    c = Case(oracle_mod, synth.reservoir(6, 5, 7, 3, seed=12), 1)
    M = c.gpu(api, transpose=True)
    B = np.random.default_rng(R).standard_normal((c.s.n, R))
    Z = M.apply(cuda(B)).cpu().numpy()
    Y = M.spmv(c.Ax, cuda(B)).cpu().numpy()
    ZT = M.apply(cuda(B), transpose=True).cpu().numpy()
    for j in range(R):
        assert rel(Z[:, j], c.O.apply(B[:, j])) <= 1e-12
        assert rel(ZT[:, j], c.O.apply(B[:, j], transpose=True)) <= 1e-12
        assert rel(Y[:, j], oracle_mod.spmv(c.s.nb, c.s.bs, c.s.Ap, c.s.Aj, c.s.Ax, B[:, j])) <= 1e-12


PAIR_CASES = [("res6x5x7_b3_k1", lambda: synth.reservoir(6, 5, 7, 3, seed=12), 1, "fp64"),
              ("res6x5x7_b3_k1_fp32", lambda: synth.reservoir(6, 5, 7, 3, seed=12), 1, "fp32"),
              ("res7x6x5_b2_k2", lambda: synth.reservoir(7, 6, 5, 2, seed=32), 2, "fp64"),
              ("res13x3x11_b1_k3", lambda: synth.reservoir(13, 3, 11, 1, seed=45), 3, "fp64"),
              ("res9x8x7_b5_k0", lambda: synth.reservoir(9, 8, 7, 5, seed=46), 0, "fp64")]


@pytest.mark.parametrize("name,make,k,prec", PAIR_CASES, ids=[c[0] for c in PAIR_CASES])
def test_rhs_pairs_identical(api, name, make, k, prec):
    """Two right-hand sides per wavefront (single tiles, R even) give, for
    every column, the bits of one column per wavefront and of a one-column
    application, in both sweeps of M^{-1} and of M^{-T}."""
    s = make()
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, k, transpose=True)
    try:
        M.tune(mode=2, tile_group=1)
        assert M.factor(cuda(s.Ax), precision=prec) == -1
        for R in (2, 8):
            B = cuda(np.random.default_rng(100 + R).standard_normal((s.n, R)))
            for tr in (False, True):
                M.tune(rhs_pairs=True)
                Zp = M.apply(B, transpose=tr)
                M.tune(rhs_pairs=False)
                Z1 = M.apply(B, transpose=tr)
                assert torch.equal(Zp, Z1), (R, tr)
                for j in (0, R - 1):
                    zj = M.apply(B[:, j].contiguous(), transpose=tr)
                    assert torch.equal(Zp[:, j], zj), (R, tr, j)
    finally:
        M.close()


def test_rhs_pairs_mid64_ilu1(api, oracle_mod):
    """The multi-right-hand-side workload of the benchmark (64^3, b = 3,
    ILU(1)) with 8 columns: pairs against single columns, bit for bit, and
    two columns against the oracle."""
    s = synth.mid_64cube()
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 1)
    try:
        assert M.factor(cuda(s.Ax)) == -1
        B = synth.multi_rhs(s.n, 8, seed=41)
        M.tune(rhs_pairs=True)
        Zp = M.apply(cuda(B))
        M.tune(rhs_pairs=False)
        Z1 = M.apply(cuda(B))
        assert torch.equal(Zp, Z1)
        O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, 1).factor(s.Ax)
        for j in (0, 7):
            assert rel(Zp[:, j].cpu().numpy(), O.apply(B[:, j].copy())) <= 1e-12
    finally:
        M.close()


SPLIT_CASES = [("cube10_b3_k1", lambda: synth.small_10cube(), 1, None),
               ("cube10_b3_k1_fp32", lambda: synth.small_10cube(), 1, "fp32"),
               ("cube10_b3_k0_groups", lambda: synth.small_10cube(), 0, 3),
               ("res7x6x5_b2_k2", lambda: synth.reservoir(7, 6, 5, 2, seed=32), 2, None),
               ("res13x3x11_b1_k3", lambda: synth.reservoir(13, 3, 11, 1, seed=45), 3, None),
               ("res9x8x7_b5_k1", lambda: synth.reservoir(9, 8, 7, 5, seed=46), 1, None)]


@pytest.mark.parametrize("name,make,k,group", SPLIT_CASES, ids=[c[0] for c in SPLIT_CASES])
def test_split_dinv_identical(api, oracle_mod, name, make, k, group):
    """D^{-1} y formed by blocks ahead of an unfused U' sweep gives the bits
    of the fused sweep (same products in the same order; with FP32 factors
    both multiply by the FP32-rounded D^{-1}), in applications and in a
    whole BiCGSTAB solve, and matches the oracle."""
    s = make()
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, k)
    fp32 = group == "fp32"
    try:
        M.tune(mode=2, tile_group=None if fp32 else group)
        assert M.factor(cuda(s.Ax), precision="fp32" if fp32 else "fp64") == -1
        r = cuda(np.random.default_rng(7).standard_normal(s.n))
        M.tune(split_dinv=True)
        zs = M.apply(r)
        M.tune(split_dinv=False)
        zf = M.apply(r)
        assert torch.equal(zs, zf)
        if not fp32:
            O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, k).factor(s.Ax)
            assert rel(zs.cpu().numpy(), O.apply(r.cpu().numpy())) <= 1e-12
        b = cuda(oracle_mod.spmv(s.nb, s.bs, s.Ap, s.Aj, s.Ax, s.xstar))
        M.tune(split_dinv=True)
        xs, st1, _ = M.solve(cuda(s.Ax), b, rtol=1e-8)
        M.tune(split_dinv=False)
        xf, st2, _ = M.solve(cuda(s.Ax), b, rtol=1e-8)
        assert st1 == 0 and st2 == 0 and torch.equal(xs, xf)
    finally:
        M.close()


@pytest.mark.parametrize("k", [0, 1])
def test_solve_parity_small(api, oracle_mod, k):
    c = Case(oracle_mod, synth.small_10cube(), k)
    M = c.gpu(api)
    x, st, info = M.solve(c.Ax, cuda(c.rhs), rtol=1e-8)
    xo, ito, rro, sto = c.O.solve(c.s.Ax, c.rhs, rtol=1e-8)
    assert st == 0 and sto == 0
    (s1, it1, rr1, _), = info
    assert abs(it1 - ito) <= 1 and rr1 <= 1e-8
    x = x.cpu().numpy()
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-10


def test_solve_transpose_parity(api, oracle_mod):
    c = Case(oracle_mod, synth.small_10cube(), 1)
    M = c.gpu(api, transpose=True)
    g = np.random.default_rng(3).standard_normal(c.s.n)
    lam, st, info = M.solve(c.Ax, cuda(g), rtol=1e-10, transpose=True)
    lo, ito, rro, sto = c.O.solve(c.s.Ax, g, rtol=1e-10, transpose=True)
    assert st == 0 and sto == 0 and abs(info[0][1] - ito) <= 1
    assert np.linalg.norm(lam.cpu().numpy() - lo) / np.linalg.norm(lo) <= 1e-10


def test_multi_rhs_solve(api, oracle_mod):
    c = Case(oracle_mod, synth.small_10cube(), 1)
    M = c.gpu(api)
    B = synth.multi_rhs(c.s.n, 8, seed=41)
    X, st, info = M.solve(c.Ax, cuda(B), rtol=1e-8)
    assert st == 0
    X = X.cpu().numpy()
    for j in range(8):
        xo, ito, rro, sto = c.O.solve(c.s.Ax, B[:, j], rtol=1e-8)
        assert info[j][0] == 0 and info[j][2] <= 1e-8 and abs(info[j][1] - ito) <= 1
        assert np.linalg.norm(X[:, j] - xo) / np.linalg.norm(xo) <= 1e-10


def test_fp32_factors(api, oracle_mod):
    c = Case(oracle_mod, synth.small_10cube(), 1)
    M = c.gpu(api, precision="fp32")
    F32, D32 = M.factors_f32()
    F32, D32 = F32.cpu().numpy(), D32.cpu().numpy()
    # the FP32 bytes are the round-to-nearest-even of the FP64 factors
    assert np.array_equal(F32, oracle_mod.round_f32(M.factors()[0].cpu().numpy()))
    r = np.random.default_rng(5).standard_normal(c.s.n)
    z = M.apply(cuda(r)).cpu().numpy()
    zo = oracle_mod.apply(c.s.nb, c.s.bs, c.O.Pp, c.O.Pj, F32, D32, r)
    assert rel(z, zo) <= 1e-12
    x, st, info = M.solve(c.Ax, cuda(c.rhs), rtol=1e-8)
    assert st == 0 and info[0][2] <= 1e-8


def test_singular_pivot(api, oracle_mod):
    s = synth.reservoir(5, 4, 3, 3, seed=8)
    Ax = s.Ax.copy()
    rows = np.repeat(np.arange(s.nb), np.diff(s.Ap))
    d = np.nonzero(s.Aj == rows)[0][7]
    Ax[d * 9] = np.nan          # non-finite pivot block in block row 7
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 0)
    assert M.factor(cuda(Ax)) == 7
    with pytest.raises(oracle_mod.OracleError) as ei:
        oracle_mod.factor(s.nb, s.bs, s.Ap, s.Aj, Ax, s.Ap, s.Aj)
    assert ei.value.row == 7


def test_grad_A(api, oracle_mod):
    s = synth.reservoir(5, 4, 3, 4, seed=21)
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 1)
    rng = np.random.default_rng(0)
    lam, x = rng.standard_normal(s.n), rng.standard_normal(s.n)
    dA = M.grad_A(cuda(lam), cuda(x)).cpu().numpy()
    assert rel(dA, oracle_mod.grad_A(s.nb, s.bs, s.Ap, s.Aj, lam, x)) <= 1e-15


# ---------------------------------------------------------------------------
# full-size workloads, in the launch configuration the benchmark times
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k", [0, 1])
def test_layered_full_size_apply_spmv(api, oracle_mod, k):
    s = synth.layered_60x220x85()
    c = Case(oracle_mod, s, k)
    M = c.gpu(api, mode=2)
    F, D = M.factors()
    gL, gU = factor_parts(c.O, s, F.cpu().numpy())
    oL, oU = factor_parts(c.O, s, c.O.F)
    assert rel(gL, oL) <= 1e-12 and rel(gU, oU) <= 1e-12
    assert rel(D.cpu().numpy(), c.O.Dinv) <= 1e-12
    r = np.random.default_rng(11).standard_normal(s.n)
    assert rel(M.apply(cuda(r)).cpu().numpy(), c.O.apply(r)) <= 1e-12
    assert rel(M.spmv(c.Ax, cuda(r)).cpu().numpy(), oracle_mod.spmv(s.nb, s.bs, s.Ap, s.Aj, s.Ax, r)) <= 1e-12
    M.check()


def test_mid_full_size_solve(api, oracle_mod):
    s = synth.mid_64cube()
    c = Case(oracle_mod, s, 1)
    M = c.gpu(api, mode=2)
    x, st, info = M.solve(c.Ax, cuda(c.rhs), rtol=1e-8)
    xo, ito, rro, sto = c.O.solve(s.Ax, c.rhs, rtol=1e-8)
    assert st == 0 and sto == 0 and abs(info[0][1] - ito) <= 1 and info[0][2] <= 1e-8
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-10


# ---------------------------------------------------------------------------
# GMRES(m)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k,restart", [(0, 30), (1, 5)])
def test_gmres_parity_small(api, oracle_mod, k, restart):
    c = Case(oracle_mod, synth.small_10cube(), k)
    M = c.gpu(api, transpose=True)
    x, st, info = M.solve(c.Ax, cuda(c.rhs), method="gmres", restart=restart, rtol=1e-8)
    xo, ito, rro, sto = c.O.solve(c.s.Ax, c.rhs, method=1, restart=restart, rtol=1e-8)
    assert st == 0 and sto == 0
    assert abs(info[0][1] - ito) <= 1 and info[0][2] <= 1e-8
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-10
    g = np.random.default_rng(9).standard_normal(c.s.n)
    lam, st, info = M.solve(c.Ax, cuda(g), method="gmres", restart=restart, rtol=1e-10, transpose=True)
    lo, ito, rro, sto = c.O.solve(c.s.Ax, g, method=1, restart=restart, rtol=1e-10, transpose=True)
    assert st == 0 and sto == 0 and abs(info[0][1] - ito) <= 1
    assert np.linalg.norm(lam.cpu().numpy() - lo) / np.linalg.norm(lo) <= 1e-10


def test_gmres_mid_full_size(api, oracle_mod):
    s = synth.mid_64cube()
    c = Case(oracle_mod, s, 1)
    M = c.gpu(api)
    x, st, info = M.solve(c.Ax, cuda(c.rhs), method="gmres", restart=30, rtol=1e-8)
    xo, ito, rro, sto = c.O.solve(s.Ax, c.rhs, method=1, restart=30, rtol=1e-8)
    assert st == 0 and sto == 0 and abs(info[0][1] - ito) <= 1 and info[0][2] <= 1e-8
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-10


# ---------------------------------------------------------------------------
# adjoint through torch.autograd
# ---------------------------------------------------------------------------
def _loss_parts(s):
    sel = torch.from_numpy(s.extras["sel"]).cuda()
    d = torch.from_numpy(s.extras["d"]).cuda()
    return sel, d


def test_autograd_small_vs_oracle_and_fd(api, oracle_mod):
    from paper_1703_01325_amd import autograd as AG
    s = synth.reservoir(6, 5, 4, 4, seed=55, sigma=2.0)
    synth.add_adjoint_extras(s, frac=0.05, n_fd=10)
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 1, transpose=True)
    Ax = cuda(s.Ax).requires_grad_(True)
    assert M.factor(Ax.detach()) == -1
    rhs = oracle_mod.spmv(s.nb, s.bs, s.Ap, s.Aj, s.Ax, s.xstar)
    b = cuda(rhs).requires_grad_(True)
    sel, d = _loss_parts(s)
    x = AG.solve(Ax, b, M)
    loss = 0.5 * ((x[sel] - d) ** 2).sum()
    loss.backward()
    # oracle gradient: lambda = A^{-T} C^T (C x - d), dA = -lambda x^T
    O = oracle_mod.OracleILU(s.nb, s.bs, s.Ap, s.Aj, 1).factor(s.Ax)
    xo, *_ = O.solve(s.Ax, rhs, rtol=1e-13, maxit=5000)
    g = np.zeros(s.n)
    g[s.extras["sel"]] = xo[s.extras["sel"]] - s.extras["d"]
    lo, *_ = O.solve(s.Ax, g, rtol=1e-13, maxit=5000, transpose=True)
    dAo = oracle_mod.grad_A(s.nb, s.bs, s.Ap, s.Aj, lo, xo)
    assert rel(b.grad.cpu().numpy(), lo) <= 1e-10
    assert rel(Ax.grad.cpu().numpy(), dAo) <= 1e-10
    # central finite differences of the loss (GPU solves, fixed preconditioner)
    h = 1e-6
    bb = s.bs * s.bs

    def L(Axv, bv):
        xv, st, _ = M.solve(Axv, bv, rtol=1e-13, maxit=5000)
        assert st == 0
        return float(0.5 * ((xv[sel] - d) ** 2).sum())

    Ad, bd = Ax.detach(), b.detach()
    for blk, (r, cc) in zip(s.extras["fd_blocks"], s.extras["fd_rc"]):
        idx = int(blk * bb + cc * s.bs + r)
        Ap_, Am_ = Ad.clone(), Ad.clone()
        Ap_[idx] += h
        Am_[idx] -= h
        fd = (L(Ap_, bd) - L(Am_, bd)) / (2 * h)
        assert abs(fd - float(Ax.grad[idx])) <= 1e-6 * max(1.0, abs(fd)) + 1e-9
    for q in s.extras["fd_b"]:
        bp, bm = bd.clone(), bd.clone()
        bp[int(q)] += h
        bm[int(q)] -= h
        fd = (L(Ad, bp) - L(Ad, bm)) / (2 * h)
        assert abs(fd - float(b.grad[int(q)])) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_autograd_thermal_full_size_fd(api):
    """64^3, b = 4, ILU(1): gradient against central differences on 20
    entries of A and 20 of b, and the adjoint residual."""
    from paper_1703_01325_amd import autograd as AG
    s = synth.thermal_64cube()
    M = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, 1, transpose=True)
    Ax = cuda(s.Ax).requires_grad_(True)
    assert M.factor(Ax.detach()) == -1
    b = M.spmv(Ax.detach(), cuda(s.xstar)).requires_grad_(True)
    sel, d = _loss_parts(s)
    x = AG.solve(Ax, b, M)
    loss = 0.5 * ((x[sel] - d) ** 2).sum()
    loss.backward()
    g = torch.zeros_like(x.detach())
    g[sel] = x.detach()[sel] - d
    res = M.spmv(Ax.detach(), b.grad, transpose=True) - g
    assert float(res.norm() / g.norm()) <= 1e-11
    h = 1e-6
    bb = s.bs * s.bs

    def L(Axv, bv):
        xv, st, _ = M.solve(Axv, bv, rtol=1e-13, maxit=5000)
        assert st == 0
        return float(0.5 * ((xv[sel] - d) ** 2).sum())

    Ad, bd = Ax.detach(), b.detach()
    for blk, (r, cc) in zip(s.extras["fd_blocks"], s.extras["fd_rc"]):
        idx = int(blk * bb + cc * s.bs + r)
        Ap_, Am_ = Ad.clone(), Ad.clone()
        Ap_[idx] += h
        Am_[idx] -= h
        fd = (L(Ap_, bd) - L(Am_, bd)) / (2 * h)
        assert abs(fd - float(Ax.grad[idx])) <= 1e-6 * max(1.0, abs(fd)) + 1e-9
    for q in s.extras["fd_b"]:
        bp, bm = bd.clone(), bd.clone()
        bp[int(q)] += h
        bm[int(q)] -= h
        fd = (L(Ad, bp) - L(Ad, bm)) / (2 * h)
        assert abs(fd - float(b.grad[int(q)])) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


@pytest.mark.parametrize("bs", [1, 2, 3])
def test_spmv_short_and_long_rows(api, oracle_mod, bs):
    """SpMV over several columns with rows from 1 to about 40 blocks and a
    ragged last wavefront: the wavefronts whose rows fit the LDS copy of
    their blocks and those that read A directly give the same bits as one
    column per pass, and each column matches the oracle."""
    nb = 300
    Ap, Aj = synth.graded_block_pattern(nb, 0.002, 0.1, seed=71 + bs)
    Ax = synth.random_block_values(Ap, Aj, bs, seed=72 + bs)
    M = api.BlockILU(nb, bs, Ap, Aj, 0)
    R = 11
    X = synth.multi_rhs(nb * bs, R, seed=73)
    M.tune(rhs_tile=1)
    y1 = M.spmv(cuda(Ax), cuda(X))
    for rt in (4, 8):
        M.tune(rhs_tile=rt)
        assert torch.equal(M.spmv(cuda(Ax), cuda(X)), y1)
    yc = y1.cpu().numpy()
    for j in range(R):
        assert rel(yc[:, j], oracle_mod.spmv(nb, bs, Ap, Aj, Ax, X[:, j].copy())) <= 1e-13


@pytest.mark.parametrize("bs", [1, 2, 3, 4])
def test_spmv_streamed_a(api, oracle_mod, bs):
    """One column with A staged through LDS (nontemporal whole-wavefront
    loads, rows in contiguous ranges per XCD) gives the bits of the direct
    kernel, on rows from 1 to about 40 blocks (long rows read A directly) and
    a ragged last wavefront, and matches the oracle; block sizes above 3 have
    no staged form and are unaffected."""
    nb = 1000 + 37 * bs
    Ap, Aj = synth.graded_block_pattern(nb, 0.002, 0.04, seed=81 + bs)
    Ax = synth.random_block_values(Ap, Aj, bs, seed=82 + bs)
    M = api.BlockILU(nb, bs, Ap, Aj, 0)
    x = np.random.default_rng(83).standard_normal(nb * bs)
    M.tune(spmv_stream=False)
    y0 = M.spmv(cuda(Ax), cuda(x))
    M.tune(spmv_stream=True)
    y1 = M.spmv(cuda(Ax), cuda(x))
    assert torch.equal(y0, y1)
    assert rel(y1.cpu().numpy(), oracle_mod.spmv(nb, bs, Ap, Aj, Ax, x)) <= 1e-13
    M.close()


@pytest.mark.parametrize("bs", [1, 3, 8])
@pytest.mark.parametrize("R", [2, 3, 5, 8, 16, 17, 32])
def test_spmv_column_lanes(api, oracle_mod, bs, R):
    """The default several-column SpMV (lanes over columns) gives, column by
    column, the bits of the one-column-per-pass kernel, for A and A^T, with
    column counts below, at and above each lane width."""
    nb = 157
    Ap, Aj = synth.graded_block_pattern(nb, 0.005, 0.08, seed=81 + bs)
    Ax = synth.random_block_values(Ap, Aj, bs, seed=82 + bs)
    M = api.BlockILU(nb, bs, Ap, Aj, 0, transpose=True)
    X = synth.multi_rhs(nb * bs, R, seed=83 + R)
    A, Xd = cuda(Ax), cuda(X)
    M.tune(rhs_tile=1)
    y1 = M.spmv(A, Xd)
    t1 = M.spmv(A, Xd, transpose=True)
    M.tune(rhs_tile=0)
    assert torch.equal(M.spmv(A, Xd), y1)
    assert torch.equal(M.spmv(A, Xd, transpose=True), t1)
    yc = y1.cpu().numpy()
    for j in (0, R - 1):
        assert rel(yc[:, j], oracle_mod.spmv(nb, bs, Ap, Aj, Ax, X[:, j].copy())) <= 1e-13


@pytest.mark.parametrize("rt", [1, 4, 8])
def test_rhs_tile_parity(api, oracle_mod, rt):
    """Columns per pass change only how the columns are grouped: every
    column's arithmetic is the same, so results are bit-identical."""
    c = Case(oracle_mod, synth.reservoir(9, 7, 5, 3, seed=61), 1)
    M = c.gpu(api)
    R = 13
    B = synth.multi_rhs(c.s.n, R, seed=41)
    zt = M.apply(cuda(B))                 # row tiles, one wavefront per (tile, column)
    M.tune(mode=1, rhs_tile=8)
    z8 = M.apply(cuda(B))
    y8 = M.spmv(c.Ax, cuda(B))
    M.tune(rhs_tile=rt)
    z = M.apply(cuda(B))
    y = M.spmv(c.Ax, cuda(B))
    assert torch.equal(z, z8) and torch.equal(y, y8) and torch.equal(zt, z8)
    zc = z.cpu().numpy()
    for j in (0, 5, 12):
        assert rel(zc[:, j], c.O.apply(B[:, j])) <= 1e-12
    M.check()


def test_autotune(api, oracle_mod):
    c = Case(oracle_mod, synth.small_10cube(), 1)
    M = c.gpu(api)
    r = cuda(np.random.default_rng(4).standard_normal(c.s.n))
    z0 = M.apply(r)
    res = M.autotune(1)
    assert res["candidates"] >= 2 and res["sweep_mode"] in (1, 2)
    assert 0 < res["apply_us"] <= res["default_us"]
    assert torch.equal(M.apply(r), z0)
    B = cuda(synth.multi_rhs(c.s.n, 8, seed=41))
    Z0 = M.apply(B)
    res8 = M.autotune(8)
    assert res8["rhs_tile"] in (1, 4, 8) and 0 < res8["apply_us"] <= res8["default_us"]
    assert torch.equal(M.apply(B), Z0)
    x, st, info = M.solve(c.Ax, cuda(c.rhs), rtol=1e-8)
    assert st == 0
    M.check()


@pytest.mark.parametrize("name,make,k", [SMALL[0], SMALL[1], SMALL[-1], SMALL[5]],
                         ids=["cube10_k0", "cube10_k1", "ragged_k2", "b5_k1"])
def test_fused_sweep_spmv_identical(api, oracle_mod, name, make, k):
    """The solvers run each U' sweep together with the SpMV of its output;
    the SpMV rows are formed with the same operations in the same order, so
    solves with and without the fused launch agree bit for bit."""
    c = Case(oracle_mod, make(), k)
    M = c.gpu(api)
    b = cuda(c.rhs)
    M.tune(fuse_spmv=False)
    x0, st0, info0 = M.solve(c.Ax, b, rtol=1e-10)
    M.tune(fuse_spmv=True, tile_group=1)      # the fused order takes single tiles
    M.timing(True)
    x1, st1, info1 = M.solve(c.Ax, b, rtol=1e-10)
    t = M.timing_read()
    M.timing(False)
    assert t["sweep_U_spmv"][0] > 0           # the fused launch ran
    assert st0 == st1 == 0 and info0 == info1 and torch.equal(x0, x1)
    g0, _, _ = M.solve(c.Ax, b, method="gmres", restart=20, rtol=1e-10)
    M.tune(fuse_spmv=False)
    g1, _, _ = M.solve(c.Ax, b, method="gmres", restart=20, rtol=1e-10)
    assert torch.equal(g0, g1)
    M.check()
    M.tune(fuse_spmv=False)


# ---------------------------------------------------------------------------
# tile groups: several tiles per workgroup, rows handed over through LDS
# ---------------------------------------------------------------------------
GROUPED = [
    ("cube10_k0_t25", lambda: synth.small_10cube(), 0, 25),          # 4 tiles per plane
    ("cube10_k0_t50", lambda: synth.small_10cube(), 0, 50),          # 2 tiles per plane
    ("cube10_k0_t100", lambda: synth.small_10cube(), 0, 100),        # whole planes
    ("cube10_k0_t30", lambda: synth.small_10cube(), 0, 30),          # tiles across planes
    ("grid_b1_k0", lambda: synth.reservoir(8, 6, 10, 1, seed=81), 0, 24),
    ("grid_b5_k0", lambda: synth.reservoir(8, 6, 10, 5, seed=82), 0, 16),
    ("grid_b8_k0", lambda: synth.reservoir(8, 6, 10, 8, seed=83), 0, 48),
    ("cube10_k1_t25", lambda: synth.small_10cube(), 1, 25),          # falls back where needed
]


@pytest.mark.parametrize("group", [2, 3, 4])
@pytest.mark.parametrize("name,make,k,tile", GROUPED, ids=[g[0] for g in GROUPED])
def test_grouped_tiles_parity(api, oracle_mod, name, make, k, tile, group):
    """Grouped row tiles compute every row with the arithmetic of the single
    tiles, so applications agree bit for bit with the ungrouped layout (one
    and several right-hand sides, transposed too; single tiles keeping only
    a ring of chunks in LDS where dependencies allow) and with the oracle to
    1e-12."""
    c = Case(oracle_mod, make(), k)
    M = c.gpu(api, transpose=True, tile_rows=tile)
    rng = np.random.default_rng(17)
    r = cuda(rng.standard_normal(c.s.n))
    B = cuda(rng.standard_normal((c.s.n, 3)))
    M.tune(tile_group=1)
    ring = list(M.info().lds_ring)
    z1, zt1, Z1 = M.apply(r), M.apply(r, transpose=True), M.apply(B)
    if k == 0 and tile in (48, 50, 100):
        assert min(ring) > 0                  # single tiles keep a ring of chunks in LDS
    M.tune(tile_group=group)
    used = M.info().tile_group
    assert 1 <= used <= group
    if k == 0 and tile in (25, 50, 16, 24, 48):
        assert used == group                  # tiles stacked over consecutive planes
    for _ in range(2):
        z, zt, Z = M.apply(r), M.apply(r, transpose=True), M.apply(B)
        assert torch.equal(z, z1) and torch.equal(zt, zt1) and torch.equal(Z, Z1)
    assert rel(z.cpu().numpy(), c.O.apply(r.cpu().numpy())) <= 1e-12
    assert rel(zt.cpu().numpy(), c.O.apply(r.cpu().numpy(), transpose=True)) <= 1e-12
    M.check()


HELPED = GROUPED + [("ragged_b3_k2", lambda: synth.reservoir(13, 3, 11, 3, seed=44), 2, None),
                    ("grid_b4_k1", lambda: synth.reservoir(9, 8, 7, 4, seed=63), 1, None)]


@pytest.mark.parametrize("group", [1, 2, 3, 4])
@pytest.mark.parametrize("name,make,k,tile", HELPED, ids=[g[0] for g in HELPED])
def test_helper_tiles_parity(api, oracle_mod, name, make, k, tile, group):
    """With a helper wavefront per tile, a tile reads the values of other
    tiles from the helper's LDS ring instead of global memory: the same
    values in the same arithmetic, so applications (both directions, FP64
    and FP32 factors) equal those without helpers bit for bit, on
    consecutive calls."""
    c = Case(oracle_mod, make(), k)
    rng = np.random.default_rng(23)
    r = cuda(rng.standard_normal(c.s.n))
    for precision in ("fp64", "fp32"):
        M = c.gpu(api, transpose=True, precision=precision, tile_rows=tile)
        M.tune(tile_group=group, helper=False)
        z1, zt1 = M.apply(r), M.apply(r, transpose=True)
        M.tune(helper=True)
        for _ in range(3):
            assert torch.equal(M.apply(r), z1)
            assert torch.equal(M.apply(r, transpose=True), zt1)
        M.check()
        M.close()
    assert rel(z1.cpu().numpy(), c.O.apply(r.cpu().numpy())) <= 1e-5


def test_helper_tiles_solve(api, oracle_mod):
    """A BiCGSTAB solve with helper wavefronts matches the oracle's."""
    c = Case(oracle_mod, synth.small_10cube(), 1)
    M = c.gpu(api, tile_rows=25)
    M.tune(helper=True)
    x, st, info = M.solve(c.Ax, cuda(c.rhs), rtol=1e-8)
    xo, ito, rro, sto = c.O.solve(c.s.Ax, c.rhs, rtol=1e-8)
    assert st == 0 and sto == 0 and abs(info[0][1] - ito) <= 1 and info[0][2] <= 1e-8
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-10
    M.check()


def test_grouped_tiles_fp32_and_solve(api, oracle_mod):
    """FP32 factors on grouped tiles (same rows as ungrouped, bit for bit),
    and a solve with grouped tiles matches the oracle's."""
    c = Case(oracle_mod, synth.small_10cube(), 0)
    M = c.gpu(api, precision="fp32", tile_rows=25)
    r = cuda(np.random.default_rng(5).standard_normal(c.s.n))
    M.tune(tile_group=1)
    z1 = M.apply(r)
    M.tune(tile_group=4)
    assert M.info().tile_group == 4
    assert torch.equal(M.apply(r), z1)
    M2 = c.gpu(api, tile_rows=25)
    M2.tune(tile_group=4)
    x, st, info = M2.solve(c.Ax, cuda(c.rhs), rtol=1e-8)
    xo, ito, rro, sto = c.O.solve(c.s.Ax, c.rhs, rtol=1e-8)
    assert st == 0 and sto == 0 and abs(info[0][1] - ito) <= 1 and info[0][2] <= 1e-8
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-10
    M2.check()


# ---------------------------------------------------------------------------
# tiles made of blocks of grid lines
# ---------------------------------------------------------------------------
BLOCKS = [("cube10_k0", lambda: synth.small_10cube(), 0, (3, 2)),
          ("cube10_k0_b7x3", lambda: synth.small_10cube(), 0, (7, 3)),
          ("cube10_k1_b5x1", lambda: synth.small_10cube(), 1, (5, 1)),
          ("grid_b4_k0", lambda: synth.reservoir(9, 8, 7, 4, seed=61), 0, (4, 4)),
          ("grid_b2_k0", lambda: synth.reservoir(11, 5, 6, 2, seed=62), 0, (2, 3))]


@pytest.mark.parametrize("name,make,k,blk", BLOCKS, ids=[b[0] for b in BLOCKS])
def test_line_block_tiles_parity(api, oracle_mod, name, make, k, blk):
    """Line-block tiles compute every row with the same operations in the
    same order as row-range tiles: applications (both directions) match the
    oracle and the row-range result bit for bit, also in FP32."""
    c = Case(oracle_mod, make(), k)
    M = c.gpu(api, transpose=True)
    r = cuda(np.random.default_rng(71).standard_normal(c.s.n))
    z0, zt0 = M.apply(r), M.apply(r, transpose=True)
    M.tune(tile_block=blk)
    info = M.info()
    assert list(info.tile_block) == [blk[0] + 256 * blk[1]] * 4
    for _ in range(2):
        z, zt = M.apply(r), M.apply(r, transpose=True)
        assert torch.equal(z, z0) and torch.equal(zt, zt0)
    assert rel(z.cpu().numpy(), c.O.apply(r.cpu().numpy())) <= 1e-12
    x, st, inf = M.solve(c.Ax, cuda(c.rhs), rtol=1e-8)
    xo, ito, rro, sto = c.O.solve(c.s.Ax, c.rhs, rtol=1e-8)
    assert st == 0 and abs(inf[0][1] - ito) <= 1
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-10
    M.check()
    M.factor(c.Ax, precision="fp32")
    F32, D32 = M.factors_f32()
    z32 = M.apply(r).cpu().numpy()
    zo32 = oracle_mod.apply(c.s.nb, c.s.bs, c.O.Pp, c.O.Pj, F32.cpu().numpy(), D32.cpu().numpy(), r.cpu().numpy())
    assert rel(z32, zo32) <= 1e-12


# ---------------------------------------------------------------------------
# line sweeps (blocks of grid lines, one diagonal per step)
# ---------------------------------------------------------------------------
LINES = [("cube10_b3_7x3", lambda: synth.small_10cube(), (7, 3)),
         ("cube10_b3_1x1", lambda: synth.small_10cube(), (1, 1)),
         ("cube10_b3_4x5", lambda: synth.small_10cube(), (4, 5)),
         ("ragged_b3_3x2", lambda: synth.reservoir(13, 7, 9, 3, seed=81), (3, 2)),
         ("ragged_b2_5x4", lambda: synth.reservoir(11, 5, 6, 2, seed=82), (5, 4)),
         ("grid_b4_4x4", lambda: synth.reservoir(9, 8, 7, 4, seed=83), (4, 4)),
         ("grid_b1_8x8", lambda: synth.reservoir(17, 9, 10, 1, seed=84), (8, 8)),
         ("grid_b8_2x4", lambda: synth.reservoir(6, 5, 9, 8, seed=85), (2, 4))]


@pytest.mark.parametrize("name,make,blk", LINES, ids=[c[0] for c in LINES])
def test_line_sweep_parity(api, oracle_mod, name, make, blk):
    """The L and U' line sweeps form every row with the same operations in the
    same order as the tiled sweeps: applications match the tiled result bit
    for bit and the oracle within 1e-12, in FP64 and on the FP32 bytes; a
    BiCGSTAB solve matches the oracle's, and bilu_apply_noalloc agrees."""
    from paper_1703_01325_amd import _native as N
    c = Case(oracle_mod, make(), 0)
    M = c.gpu(api)
    r = cuda(np.random.default_rng(91).standard_normal(c.s.n))
    z0 = M.apply(r)
    M.tune(line_sweep=blk)
    assert M.factor(c.Ax) == -1
    assert list(M.info().line_sweep) == [blk[0] + 256 * blk[1]] * 2
    for _ in range(3):
        assert torch.equal(M.apply(r), z0)
    z = torch.empty_like(r)
    N.bilu_apply_noalloc(M._ctx, r.data_ptr(), z.data_ptr(), 1, torch.cuda.current_stream().cuda_stream)
    assert torch.equal(z, z0)
    assert rel(z0.cpu().numpy(), c.O.apply(r.cpu().numpy())) <= 1e-12
    x, st, inf = M.solve(c.Ax, cuda(c.rhs), rtol=1e-8)
    xo, ito, rro, sto = c.O.solve(c.s.Ax, c.rhs, rtol=1e-8)
    assert st == 0 and abs(inf[0][1] - ito) <= 1
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-10
    M.check()
    M.factor(c.Ax, precision="fp32")
    F32, D32 = M.factors_f32()
    z32 = M.apply(r).cpu().numpy()
    zo32 = oracle_mod.apply(c.s.nb, c.s.bs, c.O.Pp, c.O.Pj, F32.cpu().numpy(), D32.cpu().numpy(), r.cpu().numpy())
    assert rel(z32, zo32) <= 1e-12
    M.check()
