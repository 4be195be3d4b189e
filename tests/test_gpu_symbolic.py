"""GPU symbolic phase (Algorithm 3 with Eq 1-2) and GPU level sets (Eq 4):
integer work, so bit-exact with the oracle -- the pattern P, the level of
fill of every entry, and for all four sweeps the level of every row,
level_ptr and level_rows (rows ascending inside a level).  A context
analysed with BILU_DEVICE_SYMBOLIC must equal a host-analysed one in every
host view and in the numbers its kernels produce."""
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


def cuda_i32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


def check_vs_oracle(api, O, name, nb, Ap, Aj, k, sweeps=(0, 1, 2, 3)):
    print(f"[symbolic] {name} nb={nb} k={k}", flush=True)
    Pp, Pj, lev = api.symbolic_device(cuda_i32(Ap), cuda_i32(Aj), k)
    oPp, oPj, olev = O.symbolic(nb, Ap, Aj, k)
    np.testing.assert_array_equal(Pp.cpu().numpy(), oPp)
    np.testing.assert_array_equal(Pj.cpu().numpy(), oPj)
    np.testing.assert_array_equal(lev.cpu().numpy(), olev)
    for w in sweeps:
        lvl, lp, lr = api.levels_device(Pp, Pj, w)
        olvl, onl = O.levels(nb, oPp, oPj, w)
        olp, olr = O.level_sets(olvl, onl)
        np.testing.assert_array_equal(lvl.cpu().numpy(), olvl, err_msg=f"sweep {w}")
        np.testing.assert_array_equal(lp.cpu().numpy(), olp, err_msg=f"sweep {w}")
        np.testing.assert_array_equal(lr.cpu().numpy(), olr, err_msg=f"sweep {w}")


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_random_patterns(api, oracle_mod, seed, k):
    nb = 50 + 23 * seed
    Ap, Aj = synth.random_block_pattern(nb, 0.02 + 0.01 * (seed % 4), seed, symmetric=(seed % 2 == 0))
    check_vs_oracle(api, oracle_mod, f"random{seed}", nb, Ap, Aj, k)


@pytest.mark.parametrize("grid,k", [((13, 11, 9), 0), ((13, 11, 9), 1), ((13, 11, 9), 2), ((9, 7, 8), 3),
                                    ((1, 1, 1), 0), ((1, 1, 1), 3), ((70, 1, 1), 2), ((2, 3, 1), 4)])
def test_grid_patterns(api, oracle_mod, grid, k):
    Ap, Aj = synth.stencil7_pattern(*grid)
    check_vs_oracle(api, oracle_mod, f"grid{grid}", int(np.prod(grid)), Ap, Aj, k)


def test_graded_pattern(api, oracle_mod):
    Ap, Aj = synth.graded_block_pattern(400, 0.002, 0.05, 7)
    for k in (0, 1, 2):
        check_vs_oracle(api, oracle_mod, "graded400", 400, Ap, Aj, k)


@pytest.mark.parametrize("k", [0, 1])
def test_layered_full_size(api, oracle_mod, k):
    # the 60 x 220 x 85 grid of the reservoir workload
    Ap, Aj = synth.stencil7_pattern(60, 220, 85)
    check_vs_oracle(api, oracle_mod, "layered60x220x85", 60 * 220 * 85, Ap, Aj, k, sweeps=(0, 1))


def test_cube64_ilu2(api, oracle_mod):
    Ap, Aj = synth.stencil7_pattern(64, 64, 64)
    check_vs_oracle(api, oracle_mod, "cube64", 64 ** 3, Ap, Aj, 2)


def test_poisson_120_ilu3(api, oracle_mod):
    # Table 1's largest fill: 7-point Poisson on 120^3 (b = 1), k = 3
    Ap, Aj = synth.stencil7_pattern(120, 120, 120)
    check_vs_oracle(api, oracle_mod, "poisson120", 120 ** 3, Ap, Aj, 3, sweeps=(0, 1))


def test_context_with_device_symbolic(api):
    s = synth.mid_64cube()
    for k in (0, 2):
        print(f"[symbolic] context k={k}", flush=True)
        A = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, k, transpose=True)
        B = api.BlockILU(s.nb, s.bs, s.Ap, s.Aj, k, transpose=True, device_symbolic=True)
        try:
            for a, b in zip(A.pattern(), B.pattern()):
                np.testing.assert_array_equal(a, b)
            for w in range(4):
                for a, b in zip(A.levels(w), B.levels(w)):
                    np.testing.assert_array_equal(a, b)
            ia, ib = A.info(), B.info()
            assert list(ia.nlev) == list(ib.nlev) and ia.tile_rows == ib.tile_rows
            Ax = torch.from_numpy(s.Ax).cuda()
            A.factor(Ax)
            B.factor(Ax)
            r = torch.from_numpy(np.random.default_rng(5).standard_normal(s.n)).cuda()
            assert torch.equal(A.apply(r), B.apply(r))
            assert torch.equal(A.apply(r, transpose=True), B.apply(r, transpose=True))
        finally:
            A.close()
            B.close()


def test_errors(api):
    from paper_1703_01325_amd import _native as N
    Ap, Aj = synth.stencil7_pattern(4, 3, 2)
    with pytest.raises(N.BiluError) as e:
        api.symbolic_device(cuda_i32(Ap), cuda_i32(Aj), -1)
    assert e.value.code == N.ERR_ARG
    bad = np.array(Aj, np.int32)
    bad[Ap[5]], bad[Ap[5] + 1] = bad[Ap[5] + 1], bad[Ap[5]]          # unsorted row 5
    with pytest.raises(N.BiluError) as e:
        api.symbolic_device(cuda_i32(Ap), cuda_i32(bad), 1)
    assert e.value.code == N.ERR_PATTERN
    # row 0 without its diagonal block
    Ap2 = np.array([0, 1, 2], np.int32)
    Aj2 = np.array([1, 1], np.int32)
    with pytest.raises(N.BiluError) as e:
        api.symbolic_device(cuda_i32(Ap2), cuda_i32(Aj2), 0)
    assert e.value.code == N.ERR_MISSING_DIAG
    # capacity below the entry count: Pp and the count are still produced
    dAp, dAj = cuda_i32(Ap), cuda_i32(Aj)
    Pp = torch.empty(Ap.size, dtype=torch.int32, device="cuda")
    Pj = torch.empty(4, dtype=torch.int32, device="cuda")
    lev = torch.empty(4, dtype=torch.int32, device="cuda")
    with pytest.raises(N.BiluError) as e:
        N.bilu_symbolic_device(Ap.size - 1, dAp.data_ptr(), dAj.data_ptr(), 1, Pp.data_ptr(), Pj.data_ptr(),
                               lev.data_ptr(), 4, api._stream())
    assert e.value.code == N.ERR_ARG
    # a row whose search reaches more block columns than the device table holds
    nb = 1200
    Apd = np.arange(0, nb * nb + 1, nb, dtype=np.int32)
    Ajd = np.tile(np.arange(nb, dtype=np.int32), nb)
    with pytest.raises(N.BiluError) as e:
        api.symbolic_device(cuda_i32(Apd), cuda_i32(Ajd), 0)
    assert e.value.code == N.ERR_ALLOC
