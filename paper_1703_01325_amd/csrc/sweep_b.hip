// Sweep and SpMV launchers for one block size, BILU_B (set by the build,
// 1..8): every kernel template of sweep_kernels.h that this block size uses
// is instantiated here and nowhere else.
#include <hip/hip_runtime.h>

#include "bilu.h"
#include "launch.h"

#ifndef BILU_B
#error "BILU_B (the block size of this translation unit) must be defined"
#endif

namespace bilu {
namespace launch {

namespace {

template <int B, typename T, int RT>
void sweep_k(int blocks, hipStream_t s, const dev::SweepArgs& a)
{
    hipLaunchKernelGGL((dev::k_sweep<B, T, RT>), dim3(blocks), dim3(dev::kThreads), 0, s, a);
}

template <int B, typename T, bool FUSE, bool MULTI>
bool tiled_k(int kmax, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a)
{
    if (a.group > 1) {
        if (a.group > kGroupMax) return false;
        const dim3 threads(64 * a.group);
        if constexpr (B >= 5) {
            if (kmax != 3) return false;
            hipLaunchKernelGGL((dev::k_sweep_grouped<B, T, FUSE, 3, MULTI, false>), dim3(blocks), threads, lds, s, a);
            return true;
        } else {
            switch (kmax) {
            case 3: hipLaunchKernelGGL((dev::k_sweep_grouped<B, T, FUSE, 3, MULTI, false>), dim3(blocks), threads, lds, s, a); return true;
            case 6: hipLaunchKernelGGL((dev::k_sweep_grouped<B, T, FUSE, 6, MULTI, false>), dim3(blocks), threads, lds, s, a); return true;
            case 9: hipLaunchKernelGGL((dev::k_sweep_grouped<B, T, FUSE, 9, MULTI, false>), dim3(blocks), threads, lds, s, a); return true;
            }
            return false;
        }
    }
    if constexpr (B >= 5) {
        if (kmax != 3) return false;
        hipLaunchKernelGGL((dev::k_sweep_tiled<B, T, FUSE, 3, MULTI>), dim3(blocks), dim3(64), lds, s, a);
        return true;
    } else {
        switch (kmax) {
        case 3: hipLaunchKernelGGL((dev::k_sweep_tiled<B, T, FUSE, 3, MULTI>), dim3(blocks), dim3(64), lds, s, a); return true;
        case 6: hipLaunchKernelGGL((dev::k_sweep_tiled<B, T, FUSE, 6, MULTI>), dim3(blocks), dim3(64), lds, s, a); return true;
        case 9: hipLaunchKernelGGL((dev::k_sweep_tiled<B, T, FUSE, 9, MULTI>), dim3(blocks), dim3(64), lds, s, a); return true;
        }
        return false;
    }
}

// Tile groups (a.group >= 1) with a helper wavefront per member; one
// right-hand side.
template <int B, typename T, bool FUSE>
bool helped_k(int kmax, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a)
{
    if (a.group < 1 || a.group > kHelpGroupMax) return false;
    const dim3 threads(128 * a.group);
    if constexpr (B >= 5) {
        if (kmax != 3) return false;
        hipLaunchKernelGGL((dev::k_sweep_grouped<B, T, FUSE, 3, false, true>), dim3(blocks), threads, lds, s, a);
        return true;
    } else {
        switch (kmax) {
        case 3: hipLaunchKernelGGL((dev::k_sweep_grouped<B, T, FUSE, 3, false, true>), dim3(blocks), threads, lds, s, a); return true;
        case 6: hipLaunchKernelGGL((dev::k_sweep_grouped<B, T, FUSE, 6, false, true>), dim3(blocks), threads, lds, s, a); return true;
        case 9: hipLaunchKernelGGL((dev::k_sweep_grouped<B, T, FUSE, 9, false, true>), dim3(blocks), threads, lds, s, a); return true;
        }
        return false;
    }
}

template <int B, typename T>
bool tiled_t(int kmax, bool fuse, bool multi, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a)
{
    if (fuse) return multi ? tiled_k<B, T, true, true>(kmax, blocks, lds, s, a) : tiled_k<B, T, true, false>(kmax, blocks, lds, s, a);
    return multi ? tiled_k<B, T, false, true>(kmax, blocks, lds, s, a) : tiled_k<B, T, false, false>(kmax, blocks, lds, s, a);
}

// Single tiles, two right-hand sides per wavefront (a.R even).
template <int B, typename T>
bool pairs_k(int kmax, bool fuse, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a)
{
    if (a.group > 1 || a.R < 2 || a.R % 2 != 0) return false;
#define BILU_PAIRS(K)                                                                                         \
    do {                                                                                                      \
        if (fuse)                                                                                             \
            hipLaunchKernelGGL((dev::k_sweep_tiled_pairs<B, T, true, K>), dim3(blocks), dim3(64), lds, s, a);  \
        else                                                                                                  \
            hipLaunchKernelGGL((dev::k_sweep_tiled_pairs<B, T, false, K>), dim3(blocks), dim3(64), lds, s, a); \
    } while (0)
    if constexpr (B >= 5) {
        if (kmax != 3) return false;
        BILU_PAIRS(3);
        return true;
    } else {
        switch (kmax) {
        case 3: BILU_PAIRS(3); return true;
        case 6: BILU_PAIRS(6); return true;
        case 9: BILU_PAIRS(9); return true;
        }
        return false;
    }
#undef BILU_PAIRS
}

template <int B, typename T>
bool fused_k(int kmax, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a, const dev::FusedSpmvArgs& m)
{
    if constexpr (B >= 5) {
        if (kmax != 3) return false;
        hipLaunchKernelGGL((dev::k_sweep_tiled_spmv<B, T, 3>), dim3(blocks), dim3(64), lds, s, a, m);
        return true;
    } else {
        switch (kmax) {
        case 3: hipLaunchKernelGGL((dev::k_sweep_tiled_spmv<B, T, 3>), dim3(blocks), dim3(64), lds, s, a, m); return true;
        case 6: hipLaunchKernelGGL((dev::k_sweep_tiled_spmv<B, T, 6>), dim3(blocks), dim3(64), lds, s, a, m); return true;
        case 9: hipLaunchKernelGGL((dev::k_sweep_tiled_spmv<B, T, 9>), dim3(blocks), dim3(64), lds, s, a, m); return true;
        }
        return false;
    }
}

template <int B, int RT, bool TR>
void spmv_k(int nb, const int32_t* rp, const int32_t* cj, const int64_t* src, const double* Ax, const double* x,
            double* y, int R, hipStream_t s, const int* gate, bool stream_a)
{
    constexpr int RPC = 64 / B;
    const int64_t waves = (static_cast<int64_t>(nb) + RPC - 1) / RPC;
    int blocks = static_cast<int>((waves + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock);
    stream_a = stream_a && RT == 1 && !TR && dev::SpmvStage<B>::doubles > 0;
    if (stream_a) blocks = (blocks + 7) / 8 * 8;
    const size_t dyn = stream_a ? sizeof(double) * dev::kWavesPerBlock * dev::SpmvStage<B>::doubles : 0;
    hipLaunchKernelGGL((dev::k_spmv<B, RT, TR>), dim3(blocks), dim3(dev::kThreads), dyn, s, nb, rp, cj, src, Ax, x,
                       y, R, gate, stream_a ? 1 : 0);
}

template <int B, int CW, bool TR>
void spmv_cols_k(int nb, const int32_t* rp, const int32_t* cj, const int64_t* src, const double* Ax,
                 const double* x, double* y, int R, hipStream_t s, const int* gate)
{
    constexpr int RPW = 64 / CW;
    const int64_t waves = (static_cast<int64_t>(nb) + RPW - 1) / RPW;
    const int blocks = static_cast<int>((waves + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock);
    hipLaunchKernelGGL((dev::k_spmv_cols<B, CW, TR>), dim3(blocks), dim3(dev::kThreads), 0, s, nb, rp, cj, src, Ax,
                       x, y, R, gate);
}

template <int B, int CW>
void spmv_cols_t(bool trans, int nb, const int32_t* rp, const int32_t* cj, const int64_t* src, const double* Ax,
                 const double* x, double* y, int R, hipStream_t s, const int* gate)
{
    if (trans) spmv_cols_k<B, CW, true>(nb, rp, cj, src, Ax, x, y, R, s, gate);
    else spmv_cols_k<B, CW, false>(nb, rp, cj, src, Ax, x, y, R, s, gate);
}

}  // namespace

template <int B>
bool sweep(int prec, int rt, int blocks, hipStream_t s, const dev::SweepArgs& a)
{
    const bool f32 = prec == BILU_FACTORS_FP32;
    switch (rt) {
    case 1: f32 ? sweep_k<B, float, 1>(blocks, s, a) : sweep_k<B, double, 1>(blocks, s, a); return true;
    case 4: f32 ? sweep_k<B, float, 4>(blocks, s, a) : sweep_k<B, double, 4>(blocks, s, a); return true;
    case 8: f32 ? sweep_k<B, float, 8>(blocks, s, a) : sweep_k<B, double, 8>(blocks, s, a); return true;
    }
    return false;
}

template <int B>
bool tiled(int kmax, int prec, bool fuse, bool multi, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a)
{
    if (prec == BILU_FACTORS_FP32) return tiled_t<B, float>(kmax, fuse, multi, blocks, lds, s, a);
    return tiled_t<B, double>(kmax, fuse, multi, blocks, lds, s, a);
}

template <int B>
bool pairs(int kmax, int prec, bool fuse, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a)
{
    if (prec == BILU_FACTORS_FP32) return pairs_k<B, float>(kmax, fuse, blocks, lds, s, a);
    return pairs_k<B, double>(kmax, fuse, blocks, lds, s, a);
}

template <int B>
bool helped(int kmax, int prec, bool fuse, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a)
{
    if (prec == BILU_FACTORS_FP32)
        return fuse ? helped_k<B, float, true>(kmax, blocks, lds, s, a) : helped_k<B, float, false>(kmax, blocks, lds, s, a);
    return fuse ? helped_k<B, double, true>(kmax, blocks, lds, s, a) : helped_k<B, double, false>(kmax, blocks, lds, s, a);
}

template <int B>
bool fused(int kmax, int prec, int blocks, size_t lds, hipStream_t s, const dev::TiledArgs& a,
           const dev::FusedSpmvArgs& m)
{
    if (prec == BILU_FACTORS_FP32) return fused_k<B, float>(kmax, blocks, lds, s, a, m);
    return fused_k<B, double>(kmax, blocks, lds, s, a, m);
}

template <int B>
bool lines(int prec, bool fuse, int blocks, hipStream_t s, const dev::LineArgs& a)
{
    const dim3 g(blocks), t(64);
    if (prec == BILU_FACTORS_FP32) {
        if (fuse) hipLaunchKernelGGL((dev::k_sweep_lines<B, float, true>), g, t, 0, s, a);
        else hipLaunchKernelGGL((dev::k_sweep_lines<B, float, false>), g, t, 0, s, a);
    } else {
        if (fuse) hipLaunchKernelGGL((dev::k_sweep_lines<B, double, true>), g, t, 0, s, a);
        else hipLaunchKernelGGL((dev::k_sweep_lines<B, double, false>), g, t, 0, s, a);
    }
    return true;
}

template <int B>
bool spmv(int rt, bool trans, int nb, const int32_t* rp, const int32_t* cj, const int64_t* src, const double* Ax,
          const double* x, double* y, int R, hipStream_t s, const int* gate, bool stream_a)
{
    if (rt == 0) {
        // lanes over columns
        if (R < 2 || R > 32) return false;
        if (R <= 2) spmv_cols_t<B, 2>(trans, nb, rp, cj, src, Ax, x, y, R, s, gate);
        else if (R <= 4) spmv_cols_t<B, 4>(trans, nb, rp, cj, src, Ax, x, y, R, s, gate);
        else if (R <= 8) spmv_cols_t<B, 8>(trans, nb, rp, cj, src, Ax, x, y, R, s, gate);
        else if (R <= 16) spmv_cols_t<B, 16>(trans, nb, rp, cj, src, Ax, x, y, R, s, gate);
        else spmv_cols_t<B, 32>(trans, nb, rp, cj, src, Ax, x, y, R, s, gate);
        return true;
    }
    switch (rt) {
    case 1: trans ? spmv_k<B, 1, true>(nb, rp, cj, src, Ax, x, y, R, s, gate, stream_a) : spmv_k<B, 1, false>(nb, rp, cj, src, Ax, x, y, R, s, gate, stream_a); return true;
    case 4: trans ? spmv_k<B, 4, true>(nb, rp, cj, src, Ax, x, y, R, s, gate, stream_a) : spmv_k<B, 4, false>(nb, rp, cj, src, Ax, x, y, R, s, gate, stream_a); return true;
    case 8: trans ? spmv_k<B, 8, true>(nb, rp, cj, src, Ax, x, y, R, s, gate, stream_a) : spmv_k<B, 8, false>(nb, rp, cj, src, Ax, x, y, R, s, gate, stream_a); return true;
    }
    return false;
}

template bool sweep<BILU_B>(int, int, int, hipStream_t, const dev::SweepArgs&);
template bool tiled<BILU_B>(int, int, bool, bool, int, size_t, hipStream_t, const dev::TiledArgs&);
template bool pairs<BILU_B>(int, int, bool, int, size_t, hipStream_t, const dev::TiledArgs&);
template bool helped<BILU_B>(int, int, bool, int, size_t, hipStream_t, const dev::TiledArgs&);
template bool fused<BILU_B>(int, int, int, size_t, hipStream_t, const dev::TiledArgs&, const dev::FusedSpmvArgs&);
template bool lines<BILU_B>(int, bool, int, hipStream_t, const dev::LineArgs&);
template bool spmv<BILU_B>(int, bool, int, const int32_t*, const int32_t*, const int64_t*, const double*,
                           const double*, double*, int, hipStream_t, const int*, bool);

}  // namespace launch
}  // namespace bilu
