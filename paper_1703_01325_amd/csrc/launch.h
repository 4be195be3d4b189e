// Launchers of the sweep and SpMV kernels, one set per block size B.  Their
// kernel templates are instantiated in sweep_b.hip, compiled once per B
// (1..8), and the batch sweep in batch_sweep.hip, so the many
// instantiations build in parallel translation units.  Each returns false
// when no kernel exists for the requested combination.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sweep_kernels.h"

namespace bilu {
namespace launch {

// Level-chunk sweep (k_sweep): prec is a bilu_precision, rt the columns per
// pass (1, 4 or 8).
template <int B>
bool sweep(int prec, int rt, int blocks, hipStream_t s, const dev::SweepArgs& a);

// Tiled sweep: one wavefront per tile (a.group == 1) or one workgroup of
// a.group wavefronts per tile group; kmax 3, 6 or 9 (3 only for B >= 5).
template <int B>
bool tiled(int kmax, int prec, bool fuse, bool multi, int blocks, size_t lds, hipStream_t s,
           const dev::TiledArgs& a);

// Tile groups of a.group >= 1 tiles, each member with a helper wavefront
// that hands it the values of other tiles through LDS (one right-hand side).
template <int B>
bool helped(int kmax, int prec, bool fuse, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a);

// U' sweep fused with the SpMV of its output (single tiles, one column).
template <int B>
bool fused(int kmax, int prec, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a,
           const dev::FusedSpmvArgs& m);

// Line sweep (k_sweep_lines) of L (fuse = false) or U' (fuse = true).
// Single tiles with two right-hand sides per wavefront (a.R even, a.group 1).
template <int B>
bool pairs(int kmax, int prec, bool fuse, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a);

template <int B>
bool lines(int prec, bool fuse, int blocks, hipStream_t s, const dev::LineArgs& a);

// y = A x (trans = false) or A^T x, rt columns per pass (1, 4 or 8), or
// rt = 0: lanes over the R columns (2 <= R <= 32); nothing runs when gate
// is given and *gate == 0.  stream_a (one column, A x, b <= 3): A staged
// through LDS with nontemporal loads, rows in contiguous ranges per XCD.
template <int B>
bool spmv(int rt, bool trans, int nb, const int32_t* rp, const int32_t* cj, const int64_t* src, const double* Ax,
          const double* x, double* y, int R, hipStream_t s, const int* gate = nullptr, bool stream_a = false);

// Batch sweep over the members' tiled layouts (every block size in one
// kernel); fuse: the second sweep of an application (D^{-1} fused).
bool batch_sweep(bool fp32, bool fuse, int blocks, size_t lds, hipStream_t s, const dev::BatchSweepArgs& a);

}  // namespace launch
}  // namespace bilu
