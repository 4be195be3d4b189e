"""GPU parity of batches of independent systems (uneven sizes and block
sizes) against the oracle run on each member alone.  Tolerances as for one
system: factors, applications and SpMVs relative 1e-12 per member; solves
to rtol 1e-8 within relative 1e-10 of the member's oracle solution and +-1
iteration."""
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


def small_members():
    """Members of the uneven-batch recipe on small grids, plus systems with
    the block sizes the recipe does not draw, so every block size runs."""
    out = [synth.uneven_batch_member(s, side_lo=3, side_hi=9) for s in range(12)]
    out += [synth.reservoir(5, 4, 3, b, seed=70 + b) for b in (1, 5, 7)]
    out.append(synth.reservoir(1, 1, 1, 3, seed=80))       # a single block row
    return out


def build(api, oracle_mod, members, k=0, precision="fp64"):
    B = api.BlockILUBatch([(m.nb, m.bs, m.Ap, m.Aj) for m in members], k)
    Ax = [cuda(m.Ax) for m in members]
    assert B.factor(Ax, precision=precision) is None
    O = [oracle_mod.OracleILU(m.nb, m.bs, m.Ap, m.Aj, k).factor(m.Ax) for m in members]
    return B, Ax, O


def split(B, v):
    return [v[B.offsets[s]:B.offsets[s + 1]] for s in range(B.nsys)]


@pytest.mark.parametrize("k", [0, 1])
def test_batch_factor_apply_spmv(api, oracle_mod, k):
    members = small_members()
    B, Ax, O = build(api, oracle_mod, members, k)
    assert B.offsets[-1] == sum(m.n for m in members)
    for s, m in enumerate(members):
        F, D = B.member(s).factors()
        assert rel(D.cpu().numpy(), O[s].Dinv) <= 1e-12
        rows = np.repeat(np.arange(m.nb), np.diff(O[s].Pp))
        Fg = F.cpu().numpy().reshape(-1, m.bs * m.bs)
        Fo = np.asarray(O[s].F).reshape(-1, m.bs * m.bs)
        for part in (O[s].Pj < rows, O[s].Pj > rows):
            if part.any():
                assert rel(Fg[part], Fo[part]) <= 1e-12, s
    rng = np.random.default_rng(11)
    r = rng.standard_normal(B.n)
    z = split(B, B.apply(cuda(r)).cpu().numpy())
    y = split(B, B.spmv(cuda(r)).cpu().numpy())
    rs = split(B, r)
    for s, m in enumerate(members):
        assert rel(z[s], O[s].apply(rs[s])) <= 1e-12, s
        assert rel(y[s], oracle_mod.spmv(m.nb, m.bs, m.Ap, m.Aj, m.Ax, rs[s])) <= 1e-12, s


def test_batch_apply_repeatable(api, oracle_mod):
    """The level-merged queue gives every row the same arithmetic whatever
    the interleaving, so repeated applications agree bit for bit."""
    B, Ax, O = build(api, oracle_mod, small_members(), 1)
    r = cuda(np.random.default_rng(2).standard_normal(B.n))
    z1 = B.apply(r)
    for _ in range(3):
        assert torch.equal(B.apply(r), z1)


def test_batch_autotune_keeps_results(api, oracle_mod):
    """The batch autotune only re-tiles the members: applications, SpMVs
    and solves give the same bits before and after, and the tuned pair is
    no slower than the one in force when timed the same way."""
    members = small_members()
    B, Ax, O = build(api, oracle_mod, members, 1)
    r = cuda(np.random.default_rng(4).standard_normal(B.n))
    rhs = cuda(np.concatenate([oracle_mod.spmv(m.nb, m.bs, m.Ap, m.Aj, m.Ax, m.xstar) for m in members]))
    z1, y1 = B.apply(r), B.spmv(r)
    x1, st1, info1 = B.solve(rhs, rtol=1e-8)
    t = B.autotune()
    assert t["candidates"] >= 1 and t["tile_scale"] in (0.25, 0.5, 1.0, 2.0, 4.0)
    assert t["pair_us"] <= t["default_us"]
    for _ in range(2):
        assert torch.equal(B.apply(r), z1) and torch.equal(B.spmv(r), y1)
    x2, st2, info2 = B.solve(rhs, rtol=1e-8)
    assert st1 == st2 == 0 and info1 == info2 and torch.equal(x1, x2)
    zs = split(B, z1.cpu().numpy())
    rs = split(B, r.cpu().numpy())
    for s in range(len(members)):
        assert rel(zs[s], O[s].apply(rs[s])) <= 1e-12, s


def test_batch_solve(api, oracle_mod):
    members = small_members()
    B, Ax, O = build(api, oracle_mod, members, 0)
    rhs = np.concatenate([oracle_mod.spmv(m.nb, m.bs, m.Ap, m.Aj, m.Ax, m.xstar) for m in members])
    x, st, info = B.solve(cuda(rhs), rtol=1e-8)
    assert st == 0
    xs = split(B, x.cpu().numpy())
    rs = split(B, rhs)
    for s, m in enumerate(members):
        xo, ito, rro, sto = O[s].solve(m.Ax, rs[s], rtol=1e-8)
        stg, itg, rrg = info[s][:3]
        assert sto == 0 and stg == 0 and rrg <= 1e-8, (s, info[s])
        assert abs(itg - ito) <= 1, (s, itg, ito)
        assert np.linalg.norm(xs[s] - xo) / np.linalg.norm(xo) <= 1e-10, s


def test_batch_solve_zero_member(api, oracle_mod):
    """A member with b = 0 is done before the first step (x = 0) while the
    others iterate."""
    members = small_members()[:5]
    B, Ax, O = build(api, oracle_mod, members, 0)
    parts = [oracle_mod.spmv(m.nb, m.bs, m.Ap, m.Aj, m.Ax, m.xstar) for m in members]
    parts[2] = np.zeros_like(parts[2])
    x, st, info = B.solve(cuda(np.concatenate(parts)), rtol=1e-8)
    assert st == 0
    xs = split(B, x.cpu().numpy())
    assert info[2][1] == 0 and not np.any(xs[2])
    for s in (0, 1, 3, 4):
        assert info[s][0] == 0 and info[s][2] <= 1e-8


def test_batch_fp32_factors(api, oracle_mod):
    members = small_members()
    B, Ax, O = build(api, oracle_mod, members, 0, precision="fp32")
    rhs = np.concatenate([oracle_mod.spmv(m.nb, m.bs, m.Ap, m.Aj, m.Ax, m.xstar) for m in members])
    x, st, info = B.solve(cuda(rhs), rtol=1e-8)
    assert st == 0
    assert all(i[0] == 0 and i[2] <= 1e-8 for i in info)


def test_uneven_batch_full_size(api, oracle_mod):
    """The 256-member uneven batch (sides U{8..40}, b from {2,3,4,6,8},
    ILU(0)) solved together; the largest member, the smallest and two more
    are checked against the oracle, and every member must reach 1e-8."""
    members = [synth.uneven_batch_member(s) for s in range(256)]
    B = api.BlockILUBatch([(m.nb, m.bs, m.Ap, m.Aj) for m in members], 0)
    Ax = [cuda(m.Ax) for m in members]
    assert B.factor(Ax) is None
    rhs_parts = [None] * len(members)
    sizes = np.array([m.n for m in members])
    check = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 17, 200})
    rng = np.random.default_rng(9)
    for s, m in enumerate(members):
        rhs_parts[s] = rng.uniform(-1.0, 1.0, m.n)
    rhs = np.concatenate(rhs_parts)
    r = cuda(rhs)
    z = split(B, B.apply(r).cpu().numpy())
    y = split(B, B.spmv(r).cpu().numpy())
    x, st, info = B.solve(r, rtol=1e-8)
    assert st == 0
    assert all(i[0] == 0 and i[2] <= 1e-8 for i in info)
    xs = split(B, x.cpu().numpy())
    for s in check:
        m = members[s]
        O = oracle_mod.OracleILU(m.nb, m.bs, m.Ap, m.Aj, 0).factor(m.Ax)
        assert rel(z[s], O.apply(rhs_parts[s])) <= 1e-12, s
        assert rel(y[s], oracle_mod.spmv(m.nb, m.bs, m.Ap, m.Aj, m.Ax, rhs_parts[s])) <= 1e-12, s
        xo, ito, rro, sto = O.solve(m.Ax, rhs_parts[s], rtol=1e-8)
        assert sto == 0 and abs(info[s][1] - ito) <= 1, (s, info[s], ito)
        assert np.linalg.norm(xs[s] - xo) / np.linalg.norm(xo) <= 1e-10, s
