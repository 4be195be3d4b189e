"""Host side of the library, on the CPU: the C ABI loads and exports every
symbol include/bilu.h declares, and the symbolic phase and level sets are
bit-exact with the oracle.  No GPU call is made here."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1703_01325_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def N():
    from paper_1703_01325_amd import _native
    return _native


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "bilu.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bilu_[A-Za-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(N):
    decl = declared_symbols()
    assert len(decl) >= 15
    assert sorted(N.EXPORTS) == decl
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (bilu_[A-Za-z0-9_]+)$", out, flags=re.M))
    for name in decl:
        assert name in exported, name
        assert getattr(N.lib, name) is not None


def lib_vs_oracle(N, O, nb, bs, Ap, Aj, k, transpose=True):
    ctx = N.bilu_analyze(nb, bs, Ap, Aj, k, N.WANT_TRANSPOSE if transpose else 0)
    try:
        N.bilu_validate(ctx)
        Pp, Pj, lev = N.bilu_get_pattern(ctx)
        oPp, oPj, olev = O.symbolic(nb, Ap, Aj, k)
        assert np.array_equal(Pp, oPp) and np.array_equal(Pj, oPj) and np.array_equal(lev, olev)
        for w in range(4 if transpose else 2):
            lp, lr = N.bilu_get_levels(ctx, w)
            olp, olr = O.level_sets(*O.levels(nb, oPp, oPj, w))
            assert np.array_equal(lp, olp) and np.array_equal(lr, olr), w
        info = N.bilu_get_info(ctx)
        rows = np.repeat(np.arange(nb), np.diff(Pp))
        assert info.nnzb_L == int((Pj < rows).sum()) and info.nnzb_U == int((Pj > rows).sum())
        assert info.nnzb_P == Pj.size and info.nnzb_A == Aj.size
    finally:
        N.bilu_destroy(ctx)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("k", [0, 1, 2, 4])
def test_random_patterns_bit_exact(N, oracle_mod, seed, k):
    nb = 60
    Ap, Aj = synth.random_block_pattern(nb, 0.05, seed, symmetric=(seed % 2 == 0))
    lib_vs_oracle(N, oracle_mod, nb, 1 + seed % 8, Ap, Aj, k)


@pytest.mark.parametrize("grid,k", [((10, 10, 10), 0), ((10, 10, 10), 1), ((7, 5, 4), 2),
                                    ((3, 9, 2), 3), ((1, 1, 1), 0), ((12, 1, 1), 1)])
def test_grid_patterns_bit_exact(N, oracle_mod, grid, k):
    Ap, Aj = synth.stencil7_pattern(*grid)
    nb = int(np.prod(grid))
    lib_vs_oracle(N, oracle_mod, nb, 3, Ap, Aj, k)


@pytest.mark.slow
@pytest.mark.parametrize("k", [1, 2])
def test_mid_grid_bit_exact(N, oracle_mod, k):
    Ap, Aj = synth.stencil7_pattern(64, 64, 64)
    lib_vs_oracle(N, oracle_mod, 64 ** 3, 3, Ap, Aj, k, transpose=False)


def test_large_k_full_fill(N, oracle_mod):
    nb = 40
    Ap, Aj = synth.random_block_pattern(nb, 0.06, 99)
    lib_vs_oracle(N, oracle_mod, nb, 2, Ap, Aj, nb)


def test_pattern_errors(N):
    Ap = np.array([0, 2, 4], np.int32)
    cases = [
        (np.array([1, 0, 0, 1], np.int32), Ap, N.ERR_PATTERN),         # unsorted
        (np.array([0, 0, 0, 1], np.int32), Ap, N.ERR_PATTERN),         # duplicate
        (np.array([0, 2, 0, 1], np.int32), Ap, N.ERR_PATTERN),         # out of range
        (np.array([1, 0], np.int32), np.array([0, 1, 2], np.int32), N.ERR_MISSING_DIAG),
    ]
    for Aj, ap, code in cases:
        with pytest.raises(N.BiluError) as ei:
            N.bilu_analyze(2, 3, ap, Aj, 0)
        assert ei.value.code == code
    for bs in (0, 33):
        with pytest.raises(N.BiluError) as ei:
            N.bilu_analyze(2, bs, Ap, np.array([0, 1, 0, 1], np.int32), 0)
        assert ei.value.code == N.ERR_ARG
    with pytest.raises(N.BiluError):
        N.bilu_analyze(2, 3, Ap, np.array([0, 1, 0, 1], np.int32), -1)


def test_gpu_calls_need_factor_first(N):
    Ap, Aj = synth.stencil7_pattern(3, 3, 1)
    ctx = N.bilu_analyze(9, 2, Ap, Aj, 0)
    try:
        # state errors are detected on the host before anything touches a GPU
        with pytest.raises(N.BiluError) as ei:
            N.bilu_apply(ctx, 1, 2, 1, 0)
        assert ei.value.code == N.ERR_STATE
        with pytest.raises(N.BiluError) as ei:
            N.bilu_factor_diag(ctx, 0, 0)
        assert ei.value.code == N.ERR_STATE
        with pytest.raises(N.BiluError) as ei:
            N.bilu_get_levels(ctx, N.SWEEP_UT)
        assert ei.value.code == N.ERR_STATE
    finally:
        N.bilu_destroy(ctx)


@pytest.mark.parametrize("tile_rows", [1, 2, 7, 64, 333, 5000])
def test_tiled_layouts_validate(N, tile_rows):
    for grid, k in (((10, 10, 10), 1), ((7, 5, 4), 2)):
        Ap, Aj = synth.stencil7_pattern(*grid)
        nb = int(np.prod(grid))
        ctx = N.bilu_analyze(nb, 3, Ap, Aj, k, N.WANT_TRANSPOSE)
        try:
            N.bilu_tune(ctx, N.TUNE_TILE_ROWS, tile_rows)
            N.bilu_validate(ctx)
        finally:
            N.bilu_destroy(ctx)
    Ap, Aj = synth.random_block_pattern(90, 0.05, 3)
    ctx = N.bilu_analyze(90, 5, Ap, Aj, 2, N.WANT_TRANSPOSE)
    try:
        N.bilu_tune(ctx, N.TUNE_TILE_ROWS, tile_rows)
        N.bilu_validate(ctx)
    finally:
        N.bilu_destroy(ctx)


@pytest.mark.parametrize("group", [0, 2, 3, 4])
@pytest.mark.parametrize("tile_rows", [0, 5, 16, 24, 40, 333])
def test_grouped_tiled_layouts_validate(N, tile_rows, group):
    """Tile groups pass the host self-check (codes into the group's LDS,
    waits covering every row read from an earlier member, ticket order of
    the groups) for every sweep, ragged tile counts included; on an ILU(0)
    grid whose planes hold whole tiles the requested group is used."""
    for grid, k in (((8, 6, 10), 0), ((8, 6, 10), 1), ((7, 5, 4), 2), ((5, 9, 11), 0)):
        Ap, Aj = synth.stencil7_pattern(*grid)
        nb = int(np.prod(grid))
        ctx = N.bilu_analyze(nb, 3, Ap, Aj, k, N.WANT_TRANSPOSE)
        try:
            N.bilu_tune(ctx, N.TUNE_TILE_GROUP, group)
            N.bilu_tune(ctx, N.TUNE_TILE_ROWS, tile_rows)
            N.bilu_validate(ctx)
            info = N.bilu_get_info(ctx)
            assert 1 <= info.tile_group <= 4
            if group and k == 0 and grid == (8, 6, 10) and tile_rows in (16, 24):
                # 48-row planes of 3 or 2 tiles: stacks of `group` planes
                assert info.tile_group == group
        finally:
            N.bilu_destroy(ctx)


def test_lds_ring_layouts_validate(N):
    """Single-tile layouts keep only the last few chunks of a tile in LDS when
    every in-tile dependency is that close: the host self-check decodes each
    ring slot to the row it holds when read and checks it against the
    pattern; the ring is used where planes are short, never for tile groups,
    and is always smaller than the tile."""
    seen = 0
    for grid, k in (((8, 6, 10), 0), ((8, 6, 10), 1), ((7, 5, 4), 2), ((20, 20, 20), 0), ((13, 7, 9), 1)):
        Ap, Aj = synth.stencil7_pattern(*grid)
        nb = int(np.prod(grid))
        ctx = N.bilu_analyze(nb, 3, Ap, Aj, k, N.WANT_TRANSPOSE)
        try:
            for group in (1, 0):
                N.bilu_tune(ctx, N.TUNE_TILE_GROUP, group)
                N.bilu_validate(ctx)
                info = N.bilu_get_info(ctx)
                for w in range(4):
                    ring = info.lds_ring[w]
                    assert ring == 0 or (info.tile_group == 1 and ring * info.rows_per_chunk < info.tile_rows)
                    seen += ring > 0
        finally:
            N.bilu_destroy(ctx)
    assert seen >= 8


@pytest.mark.parametrize("blk", [(1, 1), (7, 3), (3, 7), (4, 5), (2, 2), (40, 40)])
def test_line_block_layouts_validate(N, blk):
    """Tiles made of blocks of grid lines pass the host self-check (ring codes
    decoded to the row they hold when read, every other tile earlier in the
    ticket order) for all four sweeps.  ILU(0) grids use them; patterns whose
    blocks cannot be ordered (ILU(1) with blocks over several planes), or
    without grid lines (a random pattern), fall back to row-range tiles."""
    cases = (((8, 6, 10), 0, True), ((13, 7, 9), 0, True), ((9, 11, 4), 1, blk[1] == 1),
             ((5, 4, 3), 2, blk[1] == 1))
    for grid, k, expect in cases:
        Ap, Aj = synth.stencil7_pattern(*grid)
        nb = int(np.prod(grid))
        ctx = N.bilu_analyze(nb, 3, Ap, Aj, k, N.WANT_TRANSPOSE)
        try:
            N.bilu_tune(ctx, N.TUNE_TILE_BLOCK, blk[0] + 256 * blk[1])
            N.bilu_validate(ctx)
            info = N.bilu_get_info(ctx)
            used = [info.tile_block[w] for w in range(4)]
            if expect:
                assert used == [blk[0] + 256 * blk[1]] * 4, (grid, k, used)
            assert all(u in (0, blk[0] + 256 * blk[1]) for u in used)
            assert all(info.lds_ring[w] >= 1 for w in range(4) if used[w])
            N.bilu_tune(ctx, N.TUNE_TILE_BLOCK, 0)
            N.bilu_validate(ctx)
            assert list(N.bilu_get_info(ctx).tile_block) == [0, 0, 0, 0]
        finally:
            N.bilu_destroy(ctx)
    Ap, Aj = synth.random_block_pattern(90, 0.05, 3)
    ctx = N.bilu_analyze(90, 5, Ap, Aj, 1, N.WANT_TRANSPOSE)
    try:
        N.bilu_tune(ctx, N.TUNE_TILE_BLOCK, blk[0] + 256 * blk[1])
        N.bilu_validate(ctx)
        assert list(N.bilu_get_info(ctx).tile_block) == [0, 0, 0, 0]
    finally:
        N.bilu_destroy(ctx)


def test_tune_arguments(N):
    """Out-of-range launch knobs are refused; accepted ones keep valid
    layouts (host self-check), and a requested tile size is reported."""
    Ap, Aj = synth.stencil7_pattern(6, 5, 4)
    ctx = N.bilu_analyze(120, 3, Ap, Aj, 0, 0)
    try:
        for param, bad in ((N.TUNE_SWEEP_MODE, 3), (N.TUNE_TILE_ROWS, -1), (N.TUNE_TILE_GROUP, 5),
                           (N.TUNE_TILE_GROUP, -1), (N.TUNE_RHS_TILE, 3), (N.TUNE_FUSE_SPMV, 2), (99, 0)):
            with pytest.raises(N.BiluError) as ei:
                N.bilu_tune(ctx, param, bad)
            assert ei.value.code == N.ERR_ARG
        N.bilu_tune(ctx, N.TUNE_TILE_GROUP, 2)
        N.bilu_tune(ctx, N.TUNE_TILE_ROWS, 30)       # one plane of 6x5 cells per tile
        N.bilu_validate(ctx)
        info = N.bilu_get_info(ctx)
        assert info.tile_rows == 30 and info.tile_group == 2
        N.bilu_tune(ctx, N.TUNE_TILE_GROUP, 1)
        N.bilu_validate(ctx)
        assert N.bilu_get_info(ctx).tile_group == 1
    finally:
        N.bilu_destroy(ctx)


def test_batch_create_host(N):
    """Batch creation is host analysis only: offsets are the members' unknown
    counts laid end to end, members keep their own bit-exact analysis, and a
    bad member is named."""
    members = [synth.uneven_batch_member(s, side_lo=3, side_hi=6) for s in range(6)]
    b = N.bilu_batch_create([(m.nb, m.bs, m.Ap, m.Aj) for m in members], 1)
    try:
        import ctypes as ct
        off_p, n = N.bilu_batch_offsets(b)
        off = np.ctypeslib.as_array(ct.cast(off_p, ct.POINTER(ct.c_int64)), shape=(len(members) + 1,))
        assert list(off) == list(np.concatenate([[0], np.cumsum([m.n for m in members])]))
        assert n == off[-1]
        for s, m in enumerate(members):
            ctx = N.bilu_batch_member(b, s)
            info = N.bilu_get_info(ctx)
            assert (info.nb, info.bs, info.k) == (m.nb, m.bs, 1)
            N.bilu_validate(ctx)
        with pytest.raises(N.BiluError):
            N.bilu_batch_member(b, len(members))
    finally:
        N.bilu_batch_destroy(b)
    bad = list(members[:3])
    Ap = bad[1].Ap.copy()
    Aj = bad[1].Aj.copy()
    Aj[[0, 1]] = Aj[[1, 0]]                      # unsorted row 0 of member 1
    with pytest.raises(N.BiluError) as ei:
        N.bilu_batch_create([(m.nb, m.bs, m.Ap, m.Aj) for m in bad[:1]] + [(bad[1].nb, bad[1].bs, Ap, Aj)], 0)
    assert ei.value.code == N.ERR_PATTERN and "system 1" in str(ei.value)
    with pytest.raises(N.BiluError) as ei:
        N.bilu_batch_create([(0, 3, np.zeros(1, np.int32), np.zeros(0, np.int32))], 0)
    assert ei.value.code == N.ERR_ARG


@pytest.mark.parametrize("blk", [(1, 1), (7, 3), (3, 7), (4, 5), (21, 1), (2, 2)])
def test_line_sweep_layouts_validate(N, blk):
    """Line-sweep layouts pass their host self-check (every row once at the
    chunk and lane the kernel computes it, each factor slot the neighbour the
    kernel reads, neighbours one step earlier in the block or in an earlier
    block) on 7-point ILU(0) grids, ragged ones included; other patterns keep
    the tiled sweeps."""
    v = blk[0] + 256 * blk[1]
    for grid, bs, k, expect in (((8, 6, 10), 3, 0, True), ((13, 7, 9), 3, 0, True), ((5, 11, 4), 2, 0, True),
                                ((9, 11, 4), 3, 1, False), ((6, 5, 4), 8, 0, blk[0] * blk[1] <= 8)):
        Ap, Aj = synth.stencil7_pattern(*grid)
        nb = int(np.prod(grid))
        ctx = N.bilu_analyze(nb, bs, Ap, Aj, k, N.WANT_TRANSPOSE)
        try:
            N.bilu_tune(ctx, N.TUNE_LINE_SWEEP, v)
            N.bilu_validate(ctx)
            used = list(N.bilu_get_info(ctx).line_sweep)
            assert used == ([v, v] if expect else [0, 0]), (grid, bs, k, used)
            N.bilu_tune(ctx, N.TUNE_LINE_SWEEP, 0)
            assert list(N.bilu_get_info(ctx).line_sweep) == [0, 0]
        finally:
            N.bilu_destroy(ctx)
    Ap, Aj = synth.random_block_pattern(90, 0.05, 3)
    ctx = N.bilu_analyze(90, 3, Ap, Aj, 0, 0)
    try:
        N.bilu_tune(ctx, N.TUNE_LINE_SWEEP, v)
        N.bilu_validate(ctx)
        assert list(N.bilu_get_info(ctx).line_sweep) == [0, 0]
    finally:
        N.bilu_destroy(ctx)
