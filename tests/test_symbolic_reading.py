"""The per-row reading of Eq 1-2 that the device symbolic phase uses, on the
CPU against the oracle's row-by-row recurrence (Algorithm 3).

The GPU kernel (bilu_symbolic_device) does not run Eq 1-2's recurrence over
finished rows; it searches each row on its own: (i, j) is kept with level l
when the shortest path i -> ... -> j in the graph of A whose inner vertices
all lie below min(i, j) has l + 1 edges (the fill-path theorem, Hysom and
Pothen 2001).  The search below is that statement written out in Python,
independent of the library: k + 1 rounds of a Bellman-Ford search in the
(min, max) semiring.  If the reading were wrong (a strict / non-strict bound
on the inner vertices, paths through vertices above i, a level off by one),
one of these patterns would show it."""
import numpy as np
import pytest

from paper_1703_01325_amd import synth


def fill_path_levels(nb, Ap, Aj, k):
    Pp, Pj, Pl = [0], [], []
    for i in range(nb):
        M = {int(j): -1 for j in Aj[Ap[i]:Ap[i + 1]]}     # largest inner vertex so far
        lev = {j: 0 for j in M}
        front = [v for v in M if v < i]
        for L in range(2, k + 2):
            cand = {}
            for u in front:
                mu = max(M[u], u)
                for v in Aj[Ap[u]:Ap[u + 1]]:
                    v = int(v)
                    if mu < cand.get(v, nb):
                        cand[v] = mu
            front = []
            for v, m in cand.items():
                if m < M.get(v, nb):
                    M[v] = m
                    if v < i:
                        front.append(v)
                    if v not in lev and m < min(i, v):
                        lev[v] = L - 1
        cols = sorted(lev)
        Pj += cols
        Pl += [lev[c] for c in cols]
        Pp.append(len(Pj))
    return np.array(Pp, np.int32), np.array(Pj, np.int32), np.array(Pl, np.int32)


def cases():
    out = []
    for seed in range(12):
        nb = 40 + 9 * seed
        Ap, Aj = synth.random_block_pattern(nb, 0.03 + 0.01 * (seed % 4), seed, symmetric=(seed % 3 == 0))
        out.append((f"random{seed}", nb, Ap, Aj))
    Ap, Aj = synth.stencil7_pattern(6, 5, 7)
    out.append(("grid6x5x7", 210, Ap, Aj))
    Ap, Aj = synth.graded_block_pattern(120, 0.01, 0.2, 3)
    out.append(("graded120", 120, Ap, Aj))
    return out


@pytest.mark.parametrize("name,nb,Ap,Aj", cases(), ids=[c[0] for c in cases()])
def test_fill_paths_give_eq12_levels(oracle_mod, name, nb, Ap, Aj):
    for k in range(0, 5):
        want = oracle_mod.symbolic(nb, Ap, Aj, k)
        got = fill_path_levels(nb, np.asarray(Ap), np.asarray(Aj), k)
        for a, b in zip(want, got):
            np.testing.assert_array_equal(a, b)


def test_fill_path_bound_is_strict(oracle_mod):
    # 0 <- 2 -> 1 -> 0 style chain: row 2 reaches column 0 through vertex 1
    # only if inner vertices may equal or exceed min(i, j); the oracle keeps
    # (2, 0) only where A stores it.  A wrong (non-strict) bound would add it.
    Ap = np.array([0, 1, 3, 5], np.int32)
    Aj = np.array([0, 0, 1, 1, 2], np.int32)    # rows: {0}, {0,1}, {1,2}
    want = oracle_mod.symbolic(3, Ap, Aj, 3)
    got = fill_path_levels(3, Ap, Aj, 3)
    for a, b in zip(want, got):
        np.testing.assert_array_equal(a, b)
    # (2, 0) is fill of level 1 through the inner vertex 1 < min(2, 0)? No:
    # 1 > 0, so the entry must be absent
    assert 0 not in got[1][got[0][2]:got[0][3]].tolist()


def test_device_symbolic_has_no_host_fallback():
    """Without a GPU, asking bilu_analyze for the device symbolic phase fails
    with an error instead of quietly running the host analysis."""
    import torch
    from paper_1703_01325_amd import _native as N
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    Ap, Aj = synth.stencil7_pattern(4, 4, 4)
    with pytest.raises(N.BiluError) as e:
        N.bilu_analyze(64, 3, Ap, Aj, 1, N.DEVICE_SYMBOLIC)
    assert e.value.code in (N.ERR_ALLOC, N.ERR_HIP)
