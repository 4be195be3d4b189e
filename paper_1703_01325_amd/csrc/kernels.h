// HIP kernels for gfx950 (CDNA4, wave64) other than the sweeps and the
// SpMV: backfill, factorisation, split and layouts, Krylov vector and
// scalar steps.  Included once, by bilu_api.hip.
#pragma once

#include "sweep_kernels.h"

namespace bilu {
namespace dev {

// ---------------------------------------------------------------------------
// Backfill (Algorithm 5 steps 3-4): P takes A's block where A stores one
// and a zero block at every fill position.
// ---------------------------------------------------------------------------
__global__ void k_backfill(int64_t nP, int bb, const int32_t* __restrict__ PtoA,
                           const double* __restrict__ Ax, double* __restrict__ P)
{
    const int64_t total = nP * bb;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t e = g / bb;
        const int t = static_cast<int>(g - e * bb);
        const int32_t a = PtoA[e];
        P[g] = a >= 0 ? Ax[static_cast<int64_t>(a) * bb + t] : 0.0;
    }
}

// The same for a compile-time block size (the index arithmetic needs no
// 64-bit division by a run-time value).
template <int B>
__global__ void k_backfill_b(int64_t nP, const int32_t* __restrict__ PtoA, const double* __restrict__ Ax,
                             double* __restrict__ P)
{
    constexpr int BB = B * B;
    const int64_t total = nP * BB;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t e = g / BB;
        const int t = static_cast<int>(g - e * BB);
        const int32_t a = PtoA[e];
        P[g] = a >= 0 ? Ax[static_cast<int64_t>(a) * BB + t] : 0.0;
    }
}

// ---------------------------------------------------------------------------
// Block ILU(0) on P (Algorithm 4) for the block rows of one level of the L
// schedule: one 64-thread workgroup per block row, thread t = c*B + r owns
// element (r, c) of the block being formed.
//   for p < i in row i, ascending:  A_ip <- A_ip * inv(A_pp)
//       for j > p in row i with (p, j) in P:  A_ij <- A_ij - A_ip * A_pj
//   then inv(A_ii) by Gauss-Jordan with partial pivoting inside the block.
// The pairs (i, j), (p, j) of each pivot come from the host-built update
// lists (as in k_factor_rows_lds); this kernel serves the rows whose blocks
// do not fit the LDS budget and works on P in global memory.
// ---------------------------------------------------------------------------
template <int B>
__global__ __launch_bounds__(64) void k_factor_rows(const int32_t* __restrict__ rows, int nrows,
                                                    const int32_t* __restrict__ Pp,
                                                    const int32_t* __restrict__ Pj,
                                                    const int32_t* __restrict__ Pdiag,
                                                    const int32_t* __restrict__ upd_ptr,
                                                    const int32_t* __restrict__ upd_f,
                                                    const int32_t* __restrict__ upd_g,
                                                    double* __restrict__ P,
                                                    double* __restrict__ Dinv, int* bad_row)
{
    constexpr int BB = B * B;
    constexpr int W = 2 * B;
    constexpr int kPairs = 64 / BB > 0 ? 64 / BB : 1;
    __shared__ double sL[BB];
    __shared__ double sW[B * W];
    __shared__ int sPiv;
    __shared__ int sBad;
    if (static_cast<int>(blockIdx.x) >= nrows) return;
    const int i = rows[blockIdx.x];
    const int t = threadIdx.x;
    const int r = t % B;
    const int c = t / B;
    const int sub = t / BB;
    const int el = t - sub * BB;
    const int er = el % B;
    const int ec = el / B;
    const int e0 = Pp[i];
    const int d = Pdiag[i];
    if (t == 0) sBad = 0;
    for (int e = Pp[i]; e < d; ++e) {
        const int p = Pj[e];
        double tv = 0.0;
        if (t < BB) {
            const double* Aip = P + static_cast<int64_t>(e) * BB;
            const double* Dp = Dinv + static_cast<int64_t>(p) * BB;
#pragma unroll
            for (int u = 0; u < B; ++u) tv += Aip[u * B + r] * Dp[c * B + u];
        }
        __syncthreads();
        if (t < BB) {
            P[static_cast<int64_t>(e) * BB + t] = tv;
            sL[t] = tv;
        }
        __syncthreads();
        // the update pairs of pivot entry e (host-built lists, one target
        // block per column j), 64 / BB of them at a time; each element is
        // summed in the same order as one pair at a time
        if (sub < kPairs)
            for (int q = upd_ptr[e] + sub; q < upd_ptr[e + 1]; q += kPairs) {
                const double* Apj = P + static_cast<int64_t>(upd_g[q]) * BB;
                double sacc = 0.0;
#pragma unroll
                for (int u = 0; u < B; ++u) sacc += sL[u * B + er] * Apj[ec * B + u];
                P[static_cast<int64_t>(e0 + upd_f[q]) * BB + el] -= sacc;
            }
        __syncthreads();
    }
    // Gauss-Jordan on [U_ii | I], row-major in LDS.
    if (t < BB) {
        sW[r * W + c] = P[static_cast<int64_t>(d) * BB + t];
        sW[r * W + B + c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int col = 0; col < B; ++col) {
        if (t == 0) {
            int piv = col;
            double best = fabs(sW[col * W + col]);
            for (int rr = col + 1; rr < B; ++rr) {
                const double v = fabs(sW[rr * W + col]);
                if (v > best) {
                    best = v;
                    piv = rr;
                }
            }
            if (!(best > 0.0) || !isfinite(best)) sBad = 1;
            sPiv = piv;
        }
        __syncthreads();
        const int piv = sPiv;
        if (piv != col && t < W) {
            const double tmp = sW[col * W + t];
            sW[col * W + t] = sW[piv * W + t];
            sW[piv * W + t] = tmp;
        }
        __syncthreads();
        const double dd = sW[col * W + col];
        __syncthreads();
        if (t < W) sW[col * W + t] /= dd;
        __syncthreads();
        double fct[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int idx = t + 64 * s;
            fct[s] = idx < B * W ? sW[(idx / W) * W + col] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int idx = t + 64 * s;
            if (idx < B * W) {
                const int rr = idx / W;
                const int cc = idx - rr * W;
                if (rr != col) sW[idx] -= fct[s] * sW[col * W + cc];
            }
        }
        __syncthreads();
    }
    if (t < BB) Dinv[static_cast<int64_t>(i) * BB + t] = sW[r * W + B + c];
    if (t == 0 && sBad) atomicMin(bad_row, i);
}

// ---------------------------------------------------------------------------
// Block ILU(0) on P (Algorithm 4), the same arithmetic as k_factor_rows with
// the row held in LDS: one workgroup per block row of an L level gathers the
// row's blocks, the inverse pivot blocks D_p^{-1} of its pivots and every
// block A_pj the row's updates read (host-built lists: upd[e] holds, for the
// pivot entry e = (i, p), the pairs (f, g) of entries (i, j) and (p, j) with
// the same column j > p, f as a block index inside row i), then eliminates in
// LDS and writes the row and D_i^{-1} back.  Thread t = c*B + r owns element
// (r, c) of a block.
// LDS: [row blocks][pivot inverses][A_pj blocks] doubles, then the lists.
// ---------------------------------------------------------------------------
template <int B>
__global__ __launch_bounds__(64) void k_factor_rows_lds(const int4* __restrict__ rec, int nrows,
                                                        const int32_t* __restrict__ Pj,
                                                        const int32_t* __restrict__ upd_ptr,
                                                        const int32_t* __restrict__ upd_f,
                                                        const int32_t* __restrict__ upd_g, double* __restrict__ P,
                                                        double* __restrict__ Dinv, int* bad_row)
{
    constexpr int BB = B * B;
    constexpr int W = 2 * B;
    extern __shared__ double smem[];
    __shared__ double sW[B * W];
    __shared__ int sPiv;
    __shared__ int sBad;
    if (static_cast<int>(blockIdx.x) >= nrows) return;
    // the row's record: row, first entry, entries, pivots (blocks 0..dk-1 of
    // the row), first update pair, update pairs
    const int4 ra = rec[2 * blockIdx.x];
    const int4 rb = rec[2 * blockIdx.x + 1];
    const int i = ra.x;
    const int e0 = ra.y;
    const int nrow = ra.z;
    const int dk = ra.w;
    const int u0 = rb.x;
    const int npair = rb.y;
    const int t = threadIdx.x;
    const int r = t % B;
    const int c = t / B;
    constexpr int kPairs = 64 / BB > 0 ? 64 / BB : 1;
    const int sub = t / BB;
    const int el = t - sub * BB;
    const int er = el % B;
    const int ec = el / B;
    double* sRow = smem;
    double* sD = sRow + nrow * BB;
    double* sU = sD + dk * BB;
    int* sQ = reinterpret_cast<int*>(sU + npair * BB);    // [dk + 1] pair ranges
    int* sF = sQ + dk + 1;                                 // [npair] target block in the row
    int* sG = sF + npair;                                  // [npair] source entry (p, j)
    int* sPv = sG + npair;                                 // [dk] pivot rows
    if (t == 0) sBad = 0;
    // the row, and the lists
    for (int x = t; x < nrow * BB; x += 64) sRow[x] = P[static_cast<int64_t>(e0) * BB + x];
    for (int x = t; x <= dk; x += 64) sQ[x] = upd_ptr[e0 + x] - u0;
    for (int x = t; x < npair; x += 64) {
        sF[x] = upd_f[u0 + x];
        sG[x] = upd_g[u0 + x];
    }
    for (int x = t; x < dk; x += 64) sPv[x] = Pj[e0 + x];
    __syncthreads();
    // the finished blocks of earlier rows the row reads
    for (int x = t; x < dk * BB; x += 64) {
        const int k = x / BB;
        sD[x] = Dinv[static_cast<int64_t>(sPv[k]) * BB + (x - k * BB)];
    }
    for (int x = t; x < npair * BB; x += 64) {
        const int q = x / BB;
        sU[x] = P[static_cast<int64_t>(sG[q]) * BB + (x - q * BB)];
    }
    __syncthreads();
    for (int k = 0; k < dk; ++k) {
        double tv = 0.0;
        if (t < BB) {
#pragma unroll
            for (int u = 0; u < B; ++u) tv += sRow[k * BB + u * B + r] * sD[k * BB + c * B + u];
        }
        __syncthreads();
        if (t < BB) sRow[k * BB + t] = tv;
        __syncthreads();
        // the pairs of pivot k update distinct blocks of the row (one per
        // column j): 64 / BB pairs at a time, thread (sub, el) on element el
        // of pair sub, each element summed in the same order as one at a time
        if (sub < kPairs)
            for (int q = sQ[k] + sub; q < sQ[k + 1]; q += kPairs) {
                double acc = 0.0;
#pragma unroll
                for (int u = 0; u < B; ++u) acc += sRow[k * BB + u * B + er] * sU[q * BB + ec * B + u];
                sRow[sF[q] * BB + el] -= acc;
            }
        __syncthreads();
    }
    // Gauss-Jordan on [U_ii | I], row-major in LDS.
    if (t < BB) {
        sW[r * W + c] = sRow[dk * BB + t];
        sW[r * W + B + c] = (r == c) ? 1.0 : 0.0;
    }
    for (int x = t; x < nrow * BB; x += 64) P[static_cast<int64_t>(e0) * BB + x] = sRow[x];
    __syncthreads();
    for (int col = 0; col < B; ++col) {
        if (t == 0) {
            int piv = col;
            double best = fabs(sW[col * W + col]);
            for (int rr = col + 1; rr < B; ++rr) {
                const double v = fabs(sW[rr * W + col]);
                if (v > best) {
                    best = v;
                    piv = rr;
                }
            }
            if (!(best > 0.0) || !isfinite(best)) sBad = 1;
            sPiv = piv;
        }
        __syncthreads();
        const int piv = sPiv;
        if (piv != col && t < W) {
            const double tmp = sW[col * W + t];
            sW[col * W + t] = sW[piv * W + t];
            sW[piv * W + t] = tmp;
        }
        __syncthreads();
        const double dd = sW[col * W + col];
        __syncthreads();
        if (t < W) sW[col * W + t] /= dd;
        __syncthreads();
        double fct[2];
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
            const int idx = t + 64 * s2;
            fct[s2] = idx < B * W ? sW[(idx / W) * W + col] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
            const int idx = t + 64 * s2;
            if (idx < B * W) {
                const int rr = idx / W;
                const int cc = idx - rr * W;
                if (rr != col) sW[idx] -= fct[s2] * sW[col * W + cc];
            }
        }
        __syncthreads();
    }
    if (t < BB) Dinv[static_cast<int64_t>(i) * BB + t] = sW[r * W + B + c];
    if (t == 0 && sBad) atomicMin(bad_row, i);
}

// ---------------------------------------------------------------------------
// Block ILU(0) on P (Algorithm 4), all levels in one persistent launch with
// the arithmetic of k_factor_rows_lds: a workgroup of NWV wavefronts (16, 8,
// 4, 2 or 1, as the LDS each row needs allows) takes NWV consecutive rows of
// the L level order from a ticket and
// each wavefront factors one of them, in its own part of the LDS, with
// wavefront-level ordering instead of workgroup barriers.  A row reads its
// own blocks straight from A (PtoA: the backfill of Algorithm 5, zero at fill
// positions) and its pivot rows' finished blocks -- D_p^{-1} and the A_pj of
// its update pairs -- from P and Dinv, which start at kNotReady and receive
// each value once, final, through a device-coherent store; the wavefront
// polls those values (bounded) until none shows kNotReady.  Every pivot row
// lies earlier in the level order: in an earlier ticket, held by a running
// workgroup, or in a wavefront of the same workgroup, which progresses on
// its own, so the launch drains.
// ---------------------------------------------------------------------------
constexpr int kFacWaves = 16;     // wavefronts per workgroup, at most

struct FactorWaveArgs {
    const int4* rec;          // per position: {row, e0, nrow, dk}, {u0, npair, 0, 0}
    const int32_t* Pj;
    const int32_t* PtoA;
    const double* Ax;
    const int32_t* upd_ptr;
    const int32_t* upd_f;
    const int32_t* upd_g;
    double* P;
    double* Dinv;
    int* bad_row;
    unsigned int* ticket;     // zero at launch
    int* status;
    int nrows;
    int lds_per_wave;         // bytes, a multiple of 8
    unsigned int spin_limit;
};

// dst[y] = load(y) for y = t, t + 64, ... < n (lane t of a wavefront), G
// loads in flight per lane; true when some loaded value shows kNotReady.
template <int G, typename Load>
__device__ __forceinline__ bool gather(double* dst, int n, int t, Load load)
{
    bool pend = false;
    for (int y0 = t; y0 < n; y0 += 64 * G) {
        double v[G];
#pragma unroll
        for (int m = 0; m < G; ++m)
            if (y0 + 64 * m < n) v[m] = load(y0 + 64 * m);
#pragma unroll
        for (int m = 0; m < G; ++m)
            if (y0 + 64 * m < n) {
                dst[y0 + 64 * m] = v[m];
                pend |= is_not_ready(v[m]);
            }
    }
    return pend;
}

#define BILU_WAVE_SYNC()                      \
    do {                                      \
        __builtin_amdgcn_wave_barrier();      \
        asm volatile("" ::: "memory");        \
    } while (0)

template <int B, int NWV>
__global__ __launch_bounds__(64 * NWV) void k_factor_waves(FactorWaveArgs a)
{
    constexpr int BB = B * B;
    constexpr int W = 2 * B;
    constexpr int kPairs = 64 / BB > 0 ? 64 / BB : 1;
    // loads in flight per lane while a row is staged: eight for b >= 4 (rows of
    // many blocks; Poisson 120^3 b = 8, k = 3 214 -> 160 ms), one below, where
    // the registers they take cost occupancy (60x220x85 b = 3, ILU(0): 2.45 ms
    // with eight against 2.06)
    constexpr int kG = B >= 4 ? 8 : 1;
    extern __shared__ double fw[];
    __shared__ double sWall[NWV][B * W];
    __shared__ int sPivAll[NWV];
    __shared__ int sBadAll[NWV];
    __shared__ unsigned int sTk;
    const int wave = static_cast<int>(threadIdx.x) >> 6;
    const int t = lane_id();
    const int r = t % B;
    const int c = t / B;
    const int sub = t / BB;
    const int el = t - sub * BB;
    const int er = el % B;
    const int ec = el / B;
    double* sW = sWall[wave];
    int& sPiv = sPivAll[wave];
    int& sBad = sBadAll[wave];
    double* mine = fw + static_cast<int64_t>(wave) * (a.lds_per_wave / 8);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) sTk = atomicAdd(a.ticket, 1u);
        __syncthreads();
        const int64_t x0 = static_cast<int64_t>(sTk) * NWV;
        if (x0 >= a.nrows) break;
        const int64_t x = x0 + wave;
        if (x < a.nrows) {
            const int4 ra = a.rec[2 * x];
            const int4 rb = a.rec[2 * x + 1];
            const int i = ra.x, e0 = ra.y, nrow = ra.z, dk = ra.w, u0 = rb.x, npair = rb.y;
            double* sRow = mine;
            double* sD = sRow + nrow * BB;
            double* sU = sD + dk * BB;
            // A_pj blocks that fit beside the row, its pivot inverses and its
            // lists: all of them, or (rows beyond the LDS per wavefront) the
            // pairs of a run of pivots at a time, each pivot's at least
            const int lists = ((2 * dk + 1 + 2 * npair) * 4 + 7) / 8 * 8;
            const int cap = min(npair, (a.lds_per_wave - lists) / (8 * BB) - nrow - dk);
            int* sQ = reinterpret_cast<int*>(sU + cap * BB);
            int* sF = sQ + dk + 1;
            int* sG = sF + npair;
            int* sPv = sG + npair;
            if (t == 0) sBad = 0;
            gather<kG>(sRow, nrow * BB, t, [&](int y) {
                const int k = y / BB;
                const int32_t src = a.PtoA[e0 + k];
                return src >= 0 ? a.Ax[static_cast<int64_t>(src) * BB + (y - k * BB)] : 0.0;
            });
            for (int y = t; y <= dk; y += 64) sQ[y] = a.upd_ptr[e0 + y] - u0;
            for (int y = t; y < npair; y += 64) {
                sF[y] = a.upd_f[u0 + y];
                sG[y] = a.upd_g[u0 + y];
            }
            for (int y = t; y < dk; y += 64) sPv[y] = a.Pj[e0 + y];
            BILU_WAVE_SYNC();
            for (int k0 = 0; k0 < dk;) {
                // the run of pivots k0 .. k1 - 1 whose pairs fit
                int k1 = k0 + 1;
                while (k1 < dk && sQ[k1 + 1] - sQ[k0] <= cap) ++k1;
                const int q0 = sQ[k0], nq = sQ[k1] - q0;
                // the pivot rows' finished blocks, polled together (the pivot
                // inverses with the first run)
                const int nd = k0 == 0 ? dk * BB : 0;
                // first pass: every value, eight loads in flight per lane; then
                // only the values still missing
                bool pend = gather<kG>(sD, nd, t, [&](int y) {
                    const int k = y / BB;
                    return coherent_load(a.Dinv + static_cast<int64_t>(sPv[k]) * BB + (y - k * BB));
                });
                pend |= gather<kG>(sU, nq * BB, t, [&](int y) {
                    const int qq = y / BB;
                    return coherent_load(a.P + static_cast<int64_t>(sG[q0 + qq]) * BB + (y - qq * BB));
                });
                BILU_WAVE_SYNC();
                for (unsigned int spins = 0; __any(pend);) {
                    if (++spins > a.spin_limit) {
                        if (t == 0) atomicOr(a.status, 1);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    pend = false;
                    for (int y = t; y < nd; y += 64) {
                        const int k = y / BB;
                        double v = sD[y];
                        if (is_not_ready(v)) {
                            v = coherent_load(a.Dinv + static_cast<int64_t>(sPv[k]) * BB + (y - k * BB));
                            sD[y] = v;
                        }
                        pend |= is_not_ready(v);
                    }
                    for (int y = t; y < nq * BB; y += 64) {
                        const int qq = y / BB;
                        double v = sU[y];
                        if (is_not_ready(v)) {
                            v = coherent_load(a.P + static_cast<int64_t>(sG[q0 + qq]) * BB + (y - qq * BB));
                            sU[y] = v;
                        }
                        pend |= is_not_ready(v);
                    }
                    BILU_WAVE_SYNC();
                }
                // elimination (k_factor_rows_lds, wavefront-ordered)
                for (int k = k0; k < k1; ++k) {
                    double tv = 0.0;
                    if (t < BB) {
#pragma unroll
                        for (int u = 0; u < B; ++u) tv += sRow[k * BB + u * B + r] * sD[k * BB + c * B + u];
                    }
                    BILU_WAVE_SYNC();
                    if (t < BB) sRow[k * BB + t] = tv;
                    BILU_WAVE_SYNC();
                    if (sub < kPairs)
                        for (int qq = sQ[k] + sub; qq < sQ[k + 1]; qq += kPairs) {
                            double acc = 0.0;
#pragma unroll
                            for (int u = 0; u < B; ++u)
                                acc += sRow[k * BB + u * B + er] * sU[(qq - q0) * BB + ec * B + u];
                            sRow[sF[qq] * BB + el] -= acc;
                        }
                    BILU_WAVE_SYNC();
                }
                k0 = k1;
            }
            if (t < BB) {
                sW[r * W + c] = sRow[dk * BB + t];
                sW[r * W + B + c] = (r == c) ? 1.0 : 0.0;
            }
            for (int y = t; y < nrow * BB; y += 64)
                coherent_store(a.P + static_cast<int64_t>(e0) * BB + y, publishable(sRow[y]));
            BILU_WAVE_SYNC();
            for (int col = 0; col < B; ++col) {
                if (t == 0) {
                    int piv = col;
                    double best = fabs(sW[col * W + col]);
                    for (int rr = col + 1; rr < B; ++rr) {
                        const double v = fabs(sW[rr * W + col]);
                        if (v > best) {
                            best = v;
                            piv = rr;
                        }
                    }
                    if (!(best > 0.0) || !isfinite(best)) sBad = 1;
                    sPiv = piv;
                }
                BILU_WAVE_SYNC();
                const int piv = sPiv;
                if (piv != col && t < W) {
                    const double tmp = sW[col * W + t];
                    sW[col * W + t] = sW[piv * W + t];
                    sW[piv * W + t] = tmp;
                }
                BILU_WAVE_SYNC();
                const double dd = sW[col * W + col];
                BILU_WAVE_SYNC();
                if (t < W) sW[col * W + t] /= dd;
                BILU_WAVE_SYNC();
                double fct[2];
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) {
                    const int idx = t + 64 * s2;
                    fct[s2] = idx < B * W ? sW[(idx / W) * W + col] : 0.0;
                }
                BILU_WAVE_SYNC();
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) {
                    const int idx = t + 64 * s2;
                    if (idx < B * W) {
                        const int rr = idx / W;
                        const int cc = idx - rr * W;
                        if (rr != col) sW[idx] -= fct[s2] * sW[col * W + cc];
                    }
                }
                BILU_WAVE_SYNC();
            }
            if (t < BB)
                coherent_store(a.Dinv + static_cast<int64_t>(i) * BB + t, publishable(sW[r * W + B + c]));
            if (t == 0 && sBad) atomicMin(a.bad_row, i);
            BILU_WAVE_SYNC();
        }
    }
}

#undef BILU_WAVE_SYNC

// ---------------------------------------------------------------------------
// Point-granularity view of the factors (the point-wise solver the paper
// feeds with its block factors, Section 2.4 / Alg 6): every point entry of
// the expanded unit-diagonal L and U' takes its value from element (r, c) of
// a block of F (src = block * b*b + c*b + r), the unit diagonal 1 (src < 0).
// ---------------------------------------------------------------------------
__global__ void k_expand_point(int64_t n, const int64_t* __restrict__ src, const double* __restrict__ F,
                               double* __restrict__ Ppt)
{
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t k = src[e];
        Ppt[e] = k >= 0 ? F[k] : 1.0;
    }
}

// y = D^{-1} x with D^{-1} block diagonal (b x b blocks, column-major), one
// thread per point row; the products summed over c in order, as in the
// block sweep that fuses D^{-1}.  F32: D^{-1} taken as the FP32-stored
// factors hold it (rounded to nearest even, widened back), as the fused
// sweep of FP32 factors multiplies by it.
template <int B, bool F32 = false>
__global__ void k_block_dinv(int64_t nb, const double* __restrict__ Dinv, const double* __restrict__ x,
                             double* __restrict__ y, const int* gate)
{
    if (gated_off(gate)) return;
    constexpr int BB = B * B;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nb * B;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t I = i / B;
        const int r = static_cast<int>(i - I * B);
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < B; ++c) {
            const double d = Dinv[I * BB + c * B + r];
            acc += (F32 ? static_cast<double>(static_cast<float>(d)) : d) * x[I * B + c];
        }
        y[i] = acc;
    }
}

// ---------------------------------------------------------------------------
// Block sizes above the ones the templated kernels are built for (9..32):
// the same operations with the block size a run-time value and a workgroup
// of 256 threads per block row.  The sweeps of such systems run at point
// granularity (bilu_apply_point), so only the factorisation, the split, the
// block D^{-1} and the SpMV need these.
// ---------------------------------------------------------------------------
// Block ILU(0) on P (Algorithm 4) for the block rows of one L level, block
// size bs: for each pivot entry (i, p) in order, A_ip <- A_ip D_p^{-1}
// (staged in LDS), then the update pairs of the host-built lists,
// A_ij <- A_ij - A_ip A_pj, over (pair, element) in parallel (distinct
// targets); then D_i^{-1} by Gauss-Jordan with partial pivoting on
// [A_ii | I].  LDS: bs*bs + 2*bs*bs + bs doubles.
__global__ __launch_bounds__(256) void k_factor_rows_gen(int bs, const int32_t* __restrict__ rows, int nrows,
                                                         const int32_t* __restrict__ Pp,
                                                         const int32_t* __restrict__ Pj,
                                                         const int32_t* __restrict__ Pdiag,
                                                         const int32_t* __restrict__ upd_ptr,
                                                         const int32_t* __restrict__ upd_f,
                                                         const int32_t* __restrict__ upd_g, double* __restrict__ P,
                                                         double* __restrict__ Dinv, int* bad_row)
{
    extern __shared__ double gsm[];
    __shared__ int sPiv;
    __shared__ int sBad;
    if (static_cast<int>(blockIdx.x) >= nrows) return;
    const int bb = bs * bs;
    const int w2 = 2 * bs;
    double* sT = gsm;
    double* sW = gsm + bb;
    double* sF = sW + 2 * bb;
    const int i = rows[blockIdx.x];
    const int e0 = Pp[i];
    const int d = Pdiag[i];
    const int t = threadIdx.x;
    const int nt = blockDim.x;
    if (t == 0) sBad = 0;
    for (int e = e0; e < d; ++e) {
        const int p = Pj[e];
        const double* Aip = P + static_cast<int64_t>(e) * bb;
        const double* Dp = Dinv + static_cast<int64_t>(p) * bb;
        for (int el = t; el < bb; el += nt) {
            const int c = el / bs, r = el - (el / bs) * bs;
            double v = 0.0;
            for (int u = 0; u < bs; ++u) v += Aip[u * bs + r] * Dp[c * bs + u];
            sT[el] = v;
        }
        __syncthreads();
        for (int el = t; el < bb; el += nt) P[static_cast<int64_t>(e) * bb + el] = sT[el];
        const int q0 = upd_ptr[e];
        const int64_t work = static_cast<int64_t>(upd_ptr[e + 1] - q0) * bb;
        for (int64_t x = t; x < work; x += nt) {
            const int q = q0 + static_cast<int>(x / bb);
            const int el = static_cast<int>(x % bb);
            const int c = el / bs, r = el - (el / bs) * bs;
            const double* Apj = P + static_cast<int64_t>(upd_g[q]) * bb;
            double acc = 0.0;
            for (int u = 0; u < bs; ++u) acc += sT[u * bs + r] * Apj[c * bs + u];
            P[static_cast<int64_t>(e0 + upd_f[q]) * bb + el] -= acc;
        }
        __syncthreads();
    }
    // Gauss-Jordan on [A_ii | I], row-major in LDS
    for (int x = t; x < bs * w2; x += nt) {
        const int r = x / w2, c = x - (x / w2) * w2;
        sW[x] = c < bs ? P[static_cast<int64_t>(d) * bb + c * bs + r] : (c - bs == r ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int col = 0; col < bs; ++col) {
        if (t == 0) {
            int piv = col;
            double best = fabs(sW[col * w2 + col]);
            for (int rr = col + 1; rr < bs; ++rr) {
                const double v = fabs(sW[rr * w2 + col]);
                if (v > best) {
                    best = v;
                    piv = rr;
                }
            }
            if (!(best > 0.0) || !isfinite(best)) sBad = 1;
            sPiv = piv;
        }
        __syncthreads();
        const int piv = sPiv;
        if (piv != col)
            for (int x = t; x < w2; x += nt) {
                const double tmp = sW[col * w2 + x];
                sW[col * w2 + x] = sW[piv * w2 + x];
                sW[piv * w2 + x] = tmp;
            }
        __syncthreads();
        const double dd = sW[col * w2 + col];
        __syncthreads();
        for (int x = t; x < w2; x += nt) sW[col * w2 + x] /= dd;
        __syncthreads();
        for (int rr = t; rr < bs; rr += nt) sF[rr] = sW[rr * w2 + col];
        __syncthreads();
        for (int x = t; x < bs * w2; x += nt) {
            const int rr = x / w2, cc = x - (x / w2) * w2;
            if (rr != col) sW[x] -= sF[rr] * sW[col * w2 + cc];
        }
        __syncthreads();
    }
    for (int el = t; el < bb; el += nt) {
        const int c = el / bs, r = el - (el / bs) * bs;
        Dinv[static_cast<int64_t>(i) * bb + el] = sW[r * w2 + bs + c];
    }
    if (t == 0 && sBad) atomicMin(bad_row, i);
}

// F from P and D^{-1} (as k_split), block size bs at run time
__global__ void k_split_gen(int64_t nP, int bs, const int32_t* __restrict__ Prow, const int32_t* __restrict__ Pj,
                            const double* __restrict__ P, const double* __restrict__ Dinv, double* __restrict__ F)
{
    const int64_t bb = static_cast<int64_t>(bs) * bs;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < nP * bb;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t e = g / bb;
        const int el = static_cast<int>(g - e * bb);
        const int c = el / bs, r = el - (el / bs) * bs;
        const int i = Prow[e], j = Pj[e];
        double v;
        if (j < i) {
            v = P[g];
        } else if (j == i) {
            v = r == c ? 1.0 : 0.0;
        } else {
            const double* Di = Dinv + static_cast<int64_t>(i) * bb;
            const double* U = P + e * bb;
            v = 0.0;
            for (int u = 0; u < bs; ++u) v += Di[u * bs + r] * U[c * bs + u];
        }
        F[g] = v;
    }
}

// y = D^{-1} x by blocks (as k_block_dinv), block size bs at run time
__global__ void k_block_dinv_gen(int64_t nb, int bs, const double* __restrict__ Dinv, const double* __restrict__ x,
                                 double* __restrict__ y, const int* gate)
{
    if (gated_off(gate)) return;
    const int64_t bb = static_cast<int64_t>(bs) * bs;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nb * bs;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t I = i / bs;
        const int r = static_cast<int>(i - I * bs);
        double acc = 0.0;
        for (int c = 0; c < bs; ++c) acc += Dinv[I * bb + c * bs + r] * x[I * bs + c];
        y[i] = acc;
    }
}

// y = A x (or A^T x through the transposed structure), one right-hand side,
// one thread per point row, products summed as in spmv_rows (blocks in
// order, components in order); block size bs at run time
__global__ void k_spmv_gen(int nb, int bs, const int32_t* __restrict__ rp, const int32_t* __restrict__ cj,
                           const int64_t* __restrict__ srcpos, const double* __restrict__ Ax,
                           const double* __restrict__ x, double* __restrict__ y, const int* gate)
{
    if (gated_off(gate)) return;
    const int64_t bb = static_cast<int64_t>(bs) * bs;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < static_cast<int64_t>(nb) * bs;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t I = i / bs;
        const int r = static_cast<int>(i - I * bs);
        double acc = 0.0;
        for (int e = rp[I]; e < rp[I + 1]; ++e) {
            const int64_t j = cj[e];
            const double* A = Ax + (srcpos ? srcpos[e] : static_cast<int64_t>(e)) * bb;
            for (int c = 0; c < bs; ++c) acc += (srcpos ? A[r * bs + c] : A[c * bs + r]) * x[j * bs + c];
        }
        y[i] = acc;
    }
}

// ---------------------------------------------------------------------------
// U = D U' (Eq 5): F = L below the diagonal, U'_ij = D_i^{-1} U_ij above
// it, the identity on the diagonal.
// ---------------------------------------------------------------------------
template <int B>
__global__ void k_split(int64_t nP, const int32_t* __restrict__ Prow, const int32_t* __restrict__ Pj,
                        const double* __restrict__ P, const double* __restrict__ Dinv,
                        double* __restrict__ F)
{
    constexpr int BB = B * B;
    const int64_t total = nP * BB;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t e = g / BB;
        const int el = static_cast<int>(g - e * BB);
        const int c = el / B;
        const int r = el - c * B;
        const int i = Prow[e];
        const int j = Pj[e];
        double v;
        if (j < i) {
            v = P[g];
        } else if (j == i) {
            v = (r == c) ? 1.0 : 0.0;
        } else {
            const double* Di = Dinv + static_cast<int64_t>(i) * BB;
            const double* U = P + e * BB;
            v = 0.0;
#pragma unroll
            for (int u = 0; u < B; ++u) v += Di[u * B + r] * U[c * B + u];
        }
        F[g] = v;
    }
}

// Factor blocks gathered into a sweep layout ([k][c][r][q] per chunk),
// transposed for the U'^T / L^T sweeps, converted to T (FP64 or FP32, RNE).
// The blocks are formed from P and D^-1 as k_split forms them (same
// operations in the same order), so the layouts need no split pass.  A
// sweep reads blocks of one triangle only: upper (U', U'^T) = D_i^-1 U_ij,
// else L_ij itself.
template <typename T>
__global__ void k_layout(int64_t nslots, int B, int rpc, const int64_t* __restrict__ src,
                         const int32_t* __restrict__ Prow, const double* __restrict__ P,
                         const double* __restrict__ Dinv, int upper, int transposed, T* __restrict__ vals)
{
    const int BB = B * B;
    const int64_t total = nslots * BB;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t s = g / BB;
        const int el = static_cast<int>(g - s * BB);   // el = c*B + r
        const int c = el / B;
        const int r = el - c * B;
        const int q = static_cast<int>(s % rpc);
        const int64_t sp = src[s];
        double v = 0.0;
        if (sp >= 0) {
            // element (fr, fc) of the factor block
            const int fr = transposed ? c : r;
            const int fc = transposed ? r : c;
            if (!upper) {
                v = P[sp * BB + fc * B + fr];
            } else {
                const double* Di = Dinv + static_cast<int64_t>(Prow[sp]) * BB;
                const double* U = P + sp * BB;
                for (int u = 0; u < B; ++u) v += Di[u * B + fr] * U[fc * B + u];
            }
        }
        vals[(s - q) * BB + static_cast<int64_t>(el) * rpc + q] = static_cast<T>(v);
    }
}

// k_layout for a compile-time block size (rpc = 64/B), one thread per output
// element in output order: the stores of a wavefront are contiguous and the
// index arithmetic divides by constants.  Same values, same operations.
template <int B, typename T>
__global__ void k_layout_b(int64_t nslots, const int64_t* __restrict__ src, const int32_t* __restrict__ Prow,
                           const double* __restrict__ P, const double* __restrict__ Dinv, int upper, int transposed,
                           T* __restrict__ vals)
{
    constexpr int BB = B * B;
    constexpr int RPC = 64 / B;
    const int64_t total = nslots * BB;
    for (int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; o < total;
         o += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t grp = o / (BB * RPC);
        const int rem = static_cast<int>(o - grp * (BB * RPC));
        const int el = rem / RPC;                       // el = c*B + r
        const int q = rem - el * RPC;
        const int c = el / B;
        const int r = el - c * B;
        const int64_t sp = src[grp * RPC + q];
        double v = 0.0;
        if (sp >= 0) {
            const int fr = transposed ? c : r;
            const int fc = transposed ? r : c;
            if (!upper) {
                v = P[sp * BB + fc * B + fr];
            } else {
                const double* Di = Dinv + static_cast<int64_t>(Prow[sp]) * BB;
                const double* U = P + sp * BB;
                for (int u = 0; u < B; ++u) v += Di[u * B + fr] * U[fc * B + u];
            }
        }
        vals[o] = static_cast<T>(v);
    }
}

template <int B, typename T>
__global__ void k_layout_dinv_b(int64_t nrowslots, const int32_t* __restrict__ rows, const double* __restrict__ Dinv,
                                int transposed, T* __restrict__ out)
{
    constexpr int BB = B * B;
    constexpr int RPC = 64 / B;
    const int64_t total = nrowslots * BB;
    for (int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; o < total;
         o += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t grp = o / (BB * RPC);
        const int rem = static_cast<int>(o - grp * (BB * RPC));
        const int el = rem / RPC;
        const int q = rem - el * RPC;
        const int c = el / B;
        const int r = el - c * B;
        const int row = rows[grp * RPC + q];
        double v = 0.0;
        if (row >= 0)
            v = transposed ? Dinv[static_cast<int64_t>(row) * BB + r * B + c]
                           : Dinv[static_cast<int64_t>(row) * BB + c * B + r];
        out[o] = static_cast<T>(v);
    }
}

template <typename T>
__global__ void k_layout_dinv(int64_t nrowslots, int B, int rpc, const int32_t* __restrict__ rows,
                              const double* __restrict__ Dinv, int transposed, T* __restrict__ out)
{
    const int BB = B * B;
    const int64_t total = nrowslots * BB;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t s = g / BB;
        const int el = static_cast<int>(g - s * BB);
        const int c = el / B;
        const int r = el - c * B;
        const int q = static_cast<int>(s % rpc);
        const int row = rows[s];
        double v = 0.0;
        if (row >= 0)
            v = transposed ? Dinv[static_cast<int64_t>(row) * BB + r * B + c]
                           : Dinv[static_cast<int64_t>(row) * BB + c * B + r];
        out[(s - q) * BB + static_cast<int64_t>(el) * rpc + q] = static_cast<T>(v);
    }
}

// Inverse of k_layout for the non-transposed sweeps: FP32 values back to
// pattern order (used to hand the exact FP32 factor bytes to a caller).
__global__ void k_unlayout_f32(int64_t nslots, int B, int rpc, const int64_t* __restrict__ src,
                               const float* __restrict__ vals, float* __restrict__ F)
{
    const int BB = B * B;
    const int64_t total = nslots * BB;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t s = g / BB;
        const int el = static_cast<int>(g - s * BB);
        const int q = static_cast<int>(s % rpc);
        const int64_t sp = src[s];
        if (sp >= 0) F[sp * BB + el] = vals[(s - q) * BB + static_cast<int64_t>(el) * rpc + q];
    }
}

__global__ void k_unlayout_dinv_f32(int64_t nrowslots, int B, int rpc, const int32_t* __restrict__ rows,
                                    const float* __restrict__ in, float* __restrict__ Dinv)
{
    const int BB = B * B;
    const int64_t total = nrowslots * BB;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t s = g / BB;
        const int el = static_cast<int>(g - s * BB);
        const int q = static_cast<int>(s % rpc);
        const int row = rows[s];
        if (row >= 0) Dinv[static_cast<int64_t>(row) * BB + el] = in[(s - q) * BB + static_cast<int64_t>(el) * rpc + q];
    }
}

__global__ void k_identity_f32(int nb, int B, const int32_t* __restrict__ Pdiag, float* __restrict__ F)
{
    const int BB = B * B;
    const int64_t total = static_cast<int64_t>(nb) * BB;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t i = g / BB;
        const int el = static_cast<int>(g - i * BB);
        F[static_cast<int64_t>(Pdiag[i]) * BB + el] = (el % (B + 1) == 0) ? 1.0f : 0.0f;
    }
}

// dA_ij = -lambda_i x_j^T on A's blocks.
__global__ void k_grad_A(int64_t nA, int B, const int32_t* __restrict__ Arow, const int32_t* __restrict__ Aj,
                         const double* __restrict__ lam, const double* __restrict__ x,
                         double* __restrict__ dA)
{
    const int BB = B * B;
    const int64_t total = nA * BB;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t e = g / BB;
        const int el = static_cast<int>(g - e * BB);
        const int c = el / B;
        const int r = el - c * B;
        dA[g] = -lam[static_cast<int64_t>(Arow[e]) * B + r] * x[static_cast<int64_t>(Aj[e]) * B + c];
    }
}

__global__ void k_fill_i32(int64_t n, int32_t* p, int32_t v)
{
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[g] = v;
}

// *dst |= *src (one thread): a sweep status kept elsewhere joins the context's.
__global__ void k_merge_status(const int* src, int* dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && *src) atomicOr(dst, *src);
}

__global__ void k_fill_not_ready(int64_t n, double* p)
{
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[g] = not_ready();
}

__global__ void k_fill_f64(int64_t n, double* p, double v)
{
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[g] = v;
}

// ---------------------------------------------------------------------------
// Krylov vector kernels.  Vectors are n x R row-major (n = nb*B).  Dot
// products are deterministic two-stage sums: the reduction kernels run on a
// fixed grid of kRedBlocks workgroups with a grid stride that is a multiple
// of R, so every thread stays on one column; each workgroup writes one
// partial per column, summed in a fixed order by the scalar kernels.
// Per-column scalars live in a device KState.
// ---------------------------------------------------------------------------
struct KState {
    double rho[kMaxRhs], rho_old[kMaxRhs], alpha[kMaxRhs], omega[kMaxRhs], beta[kMaxRhs];
    double bnorm2[kMaxRhs], tol2[kMaxRhs], snorm2[kMaxRhs], rnorm2[kMaxRhs], tnorm2[kMaxRhs];
    int active[kMaxRhs], fresh[kMaxRhs], half[kMaxRhs], status[kMaxRhs], restart[kMaxRhs];
    int check[kMaxRhs];      // the recurrence passed the test this step: compute the true residual
    int nrestart[kMaxRhs];   // restarts from the true residual so far
    int done_it[kMaxRhs];    // step at which the column stopped (-1: still running)
    int any_check;           // some column has check set (gates the true-residual pass)
    int any_restart;         // some column restarts (gates the restart pass)
    int any_active;          // some column still iterates (gates every kernel of a step)
    int sweep_status;
};

enum { ST_OK = 0, ST_NOT_CONV = 2, ST_BREAKDOWN = 3, ST_NONFINITE = 4 };

// Per-thread column and the stride of the reduction loop.
struct RedIdx {
    int64_t start, stride;
    int col;
    bool live;
};

// Grid-stride loops of the reductions below are unrolled by 4 (several
// loads in flight per thread); the single accumulator keeps the order.
__device__ __forceinline__ RedIdx red_index(int R)
{
    const int64_t nthreads = static_cast<int64_t>(kRedBlocks) * kThreads;
    const int64_t stride = (nthreads / R) * R;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    RedIdx ri;
    ri.start = gid;
    ri.stride = stride;
    ri.col = static_cast<int>(gid % R);
    ri.live = gid < stride;
    return ri;
}

// Sums, per column, the thread values of one workgroup in a fixed order and
// stores the partial for this workgroup.  (A serial sum by one thread per
// column cost 2-5 us at the end of every workgroup with one column.)
__device__ __forceinline__ void block_partial(double v, int R, double* part_slot)
{
    __shared__ double sred[kThreads];
    if ((R & (R - 1)) == 0 && R <= 64) {
        // R a power of two: thread t holds column t mod R, so a butterfly
        // over lane offsets 32, 16, ..., R leaves in lane c < R the sum of
        // its wavefront's column c; the wavefronts' sums are then added in
        // wavefront order.
        for (int off = 32; off >= R; off >>= 1) v += __shfl_xor(v, off);
        const int lane = lane_id();
        const int wave = static_cast<int>(threadIdx.x) >> 6;
        __syncthreads();
        if (lane < R) sred[wave * 64 + lane] = v;
        __syncthreads();
        if (static_cast<int>(threadIdx.x) < R) {
            const int col = threadIdx.x;
            double s = sred[col];
#pragma unroll
            for (int w = 1; w < kWavesPerBlock; ++w) s += sred[w * 64 + col];
            part_slot[static_cast<int64_t>(col) * kRedBlocks + blockIdx.x] = s;
        }
        return;
    }
    __syncthreads();
    sred[threadIdx.x] = v;
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < R) {
        // threads of this workgroup whose global index is == col (mod R)
        const int col = threadIdx.x;
        const int base = static_cast<int>((static_cast<int64_t>(blockIdx.x) * kThreads) % R);
        double s = 0.0;
        for (int t = (col - base + R) % R; t < kThreads; t += R) s += sred[t];
        part_slot[static_cast<int64_t>(col) * kRedBlocks + blockIdx.x] = s;
    }
}

// part[slot][col][block]
__device__ __forceinline__ double* slot_ptr(double* part, int slot)
{
    return part + static_cast<int64_t>(slot) * kMaxRhs * kRedBlocks;
}

__global__ __launch_bounds__(kThreads) void k_dot(int64_t n, int R, const double* __restrict__ a,
                                                  const double* __restrict__ b, double* part, int slot,
                                                  const int* gate = nullptr)
{
    if (gated_off(gate)) return;
    const RedIdx ri = red_index(R);
    double acc = 0.0;
    if (ri.live)
#pragma unroll 4
        for (int64_t g = ri.start; g < n * R; g += ri.stride) acc += a[g] * b[g];
    block_partial(acc, R, slot_ptr(part, slot));
}

// t.s and t.t in one pass
__global__ __launch_bounds__(kThreads) void k_dot2(int64_t n, int R, const double* __restrict__ t,
                                                   const double* __restrict__ s, double* part,
                                                   int slot_ts, int slot_tt, const int* gate = nullptr)
{
    if (gated_off(gate)) return;
    const RedIdx ri = red_index(R);
    double ts = 0.0, tt = 0.0;
    if (ri.live)
#pragma unroll 4
        for (int64_t g = ri.start; g < n * R; g += ri.stride) {
            const double tv = t[g];
            ts += tv * s[g];
            tt += tv * tv;
        }
    block_partial(ts, R, slot_ptr(part, slot_ts));
    block_partial(tt, R, slot_ptr(part, slot_tt));
}

// Sum of the kRedBlocks partials of (slot, col), by one whole wavefront in a
// fixed order (lane l adds partials l, l+64, ... in turn, then a fixed
// butterfly over the lanes); lane 0's value, so every call on the same
// partials gives the same bits.
__device__ __forceinline__ double sum_partials(const double* part, int slot, int col)
{
    static_assert(kRedBlocks % 64 == 0, "partials per lane");
    const double* p = part + static_cast<int64_t>(slot) * kMaxRhs * kRedBlocks +
                      static_cast<int64_t>(col) * kRedBlocks;
    const int lane = lane_id();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kRedBlocks / 64; ++k) s += p[lane + 64 * k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
    return __shfl(s, 0);
}

enum { SL_RHO = 0, SL_RV = 1, SL_SS = 2, SL_TS = 3, SL_TT = 4, SL_RR = 5, SL_BB = 6, SL_TRUE = 7 };
constexpr int kSlots = 8;

// Scalar steps of right-preconditioned BiCGSTAB for recurrence c of a state
// S: KState holds the right-hand-side columns of one system, BatchState the
// systems of a batch; both expose their per-recurrence values as arrays of
// the same names.  A recurrence that breaks down or turns non-finite is
// frozen with its status.
template <class S>
__device__ __forceinline__ void bicg_init_one(S& st, int c, double b2, double rtol)
{
    st.bnorm2[c] = b2;
    st.tol2[c] = rtol * rtol * b2;
    st.active[c] = b2 > 0.0 ? 1 : 0;
    st.status[c] = b2 > 0.0 ? ST_NOT_CONV : ST_OK;
    st.fresh[c] = 1;
    st.half[c] = 0;
    st.restart[c] = 0;
    st.rho_old[c] = 1.0;
    st.alpha[c] = 1.0;
    st.omega[c] = 1.0;
    st.rnorm2[c] = b2;
    st.tnorm2[c] = b2;
}

template <class S>
__device__ __forceinline__ void bicg_freeze(S& st, int c, int status)
{
    st.status[c] = status;
    st.active[c] = 0;
}

// rho = <r^, r>; beta for the direction update
template <class S>
__device__ __forceinline__ void bicg_rho_one(S& st, int c, double rho)
{
    if (!st.active[c]) return;
    st.rho[c] = rho;
    st.half[c] = 0;
    if (!isfinite(rho)) bicg_freeze(st, c, ST_NONFINITE);
    else if (rho == 0.0) bicg_freeze(st, c, ST_BREAKDOWN);
    else st.beta[c] = st.fresh[c] ? 0.0 : (rho / st.rho_old[c]) * (st.alpha[c] / st.omega[c]);
}

// alpha = rho / <r^, v>
template <class S>
__device__ __forceinline__ void bicg_alpha_one(S& st, int c, double rv)
{
    if (!st.active[c]) return;
    st.fresh[c] = 0;
    if (!isfinite(rv)) bicg_freeze(st, c, ST_NONFINITE);
    else if (rv == 0.0) bicg_freeze(st, c, ST_BREAKDOWN);
    else st.alpha[c] = st.rho[c] / rv;
}

// ||s||^2: the half step may already meet the tolerance
template <class S>
__device__ __forceinline__ void bicg_snorm_one(S& st, int c, double s2)
{
    if (!st.active[c]) return;
    st.snorm2[c] = s2;
    st.half[c] = (s2 <= st.tol2[c]) ? 1 : 0;
    if (!isfinite(s2)) bicg_freeze(st, c, ST_NONFINITE);
}

// omega = <t, s> / <t, t>
template <class S>
__device__ __forceinline__ void bicg_omega_one(S& st, int c, double ts, double tt)
{
    if (!st.active[c] || st.half[c]) return;
    if (!isfinite(ts) || !isfinite(tt)) bicg_freeze(st, c, ST_NONFINITE);
    else if (tt == 0.0) bicg_freeze(st, c, ST_BREAKDOWN);
    else st.omega[c] = ts / tt;
}

// ||r||^2 at the end of a full step
template <class S>
__device__ __forceinline__ void bicg_end_one(S& st, int c, double r2)
{
    if (!st.active[c] || st.half[c]) return;
    st.rnorm2[c] = r2;
    st.rho_old[c] = st.rho[c];
    if (!isfinite(r2)) bicg_freeze(st, c, ST_NONFINITE);
    else if (st.omega[c] == 0.0) bicg_freeze(st, c, ST_BREAKDOWN);
}

// BiCGSTAB setup: ||b||, tolerance, flags.  r = b, r^ = r, x = 0 are done
// by copies on the host side; k_bicg_decide(it = 0) follows and sets the
// flags that gate the first step.
// Scalar kernels: one wavefront (workgroup) per right-hand side c.
__global__ __launch_bounds__(64) void k_bicg_init(int R, const double* part, KState* st, double rtol)
{
    const int c = blockIdx.x;
    if (c >= R) return;
    const double b2 = sum_partials(part, SL_BB, c);
    if (lane_id() != 0) return;
    bicg_init_one(*st, c, b2, rtol);
    st->check[c] = 0;
    st->nrestart[c] = 0;
    st->done_it[c] = -1;
    if (c == 0) st->sweep_status = 0;
}

__global__ __launch_bounds__(64) void k_bicg_s_rho(int R, const double* part, KState* st)
{
    if (!st->any_active) return;
    const int c = blockIdx.x;
    if (c >= R) return;
    const double v = sum_partials(part, SL_RHO, c);
    if (lane_id() == 0) bicg_rho_one(*st, c, v);
}

__global__ void k_bicg_p(int64_t n, int R, const double* __restrict__ r, const double* __restrict__ v,
                         double* __restrict__ p, const KState* st)
{
    if (!st->any_active) return;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n * R;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int c = static_cast<int>(g % R);
        if (!st->active[c]) continue;
        p[g] = st->fresh[c] ? r[g] : r[g] + st->beta[c] * (p[g] - st->omega[c] * v[g]);
    }
}

__global__ __launch_bounds__(64) void k_bicg_s_alpha(int R, const double* part, KState* st)
{
    if (!st->any_active) return;
    const int c = blockIdx.x;
    if (c >= R) return;
    const double v = sum_partials(part, SL_RV, c);
    if (lane_id() == 0) bicg_alpha_one(*st, c, v);
}

// s = r - alpha v, partial of s.s
__global__ __launch_bounds__(kThreads) void k_bicg_s(int64_t n, int R, const double* __restrict__ r,
                                                     const double* __restrict__ v, double* __restrict__ s,
                                                     const KState* st, double* part)
{
    if (!st->any_active) return;
    const RedIdx ri = red_index(R);
    double acc = 0.0;
    if (ri.live && st->active[ri.col]) {
        const double al = st->alpha[ri.col];
#pragma unroll 4
        for (int64_t g = ri.start; g < n * R; g += ri.stride) {
            const double sv = r[g] - al * v[g];
            s[g] = sv;
            acc += sv * sv;
        }
    }
    block_partial(acc, R, slot_ptr(part, SL_SS));
}

__global__ __launch_bounds__(64) void k_bicg_s_snorm(int R, const double* part, KState* st)
{
    if (!st->any_active) return;
    const int c = blockIdx.x;
    if (c >= R) return;
    const double v = sum_partials(part, SL_SS, c);
    if (lane_id() == 0) bicg_snorm_one(*st, c, v);
}

__global__ __launch_bounds__(64) void k_bicg_s_omega(int R, const double* part, KState* st)
{
    if (!st->any_active) return;
    const int c = blockIdx.x;
    if (c >= R) return;
    const double ts = sum_partials(part, SL_TS, c);
    const double tt = sum_partials(part, SL_TT, c);
    if (lane_id() == 0) bicg_omega_one(*st, c, ts, tt);
}

// x += alpha p^ (+ omega s^ unless the half step already converged),
// r = s - omega t; partial of r.r
__global__ __launch_bounds__(kThreads) void k_bicg_xr(int64_t n, int R, double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      const double* __restrict__ ph,
                                                      const double* __restrict__ sh,
                                                      const double* __restrict__ s,
                                                      const double* __restrict__ t, const KState* st,
                                                      double* part)
{
    if (!st->any_active) return;
    const RedIdx ri = red_index(R);
    double acc = 0.0;
    if (ri.live && st->active[ri.col]) {
        const int c = ri.col;
        const double al = st->alpha[c];
        if (st->half[c]) {
#pragma unroll 4
            for (int64_t g = ri.start; g < n * R; g += ri.stride) x[g] += al * ph[g];
        } else {
            const double om = st->omega[c];
#pragma unroll 4
            for (int64_t g = ri.start; g < n * R; g += ri.stride) {
                x[g] += al * ph[g] + om * sh[g];
                const double rv = s[g] - om * t[g];
                r[g] = rv;
                acc += rv * rv;
            }
        }
    }
    block_partial(acc, R, slot_ptr(part, SL_RR));
}

// End of a step: ||r||^2; a column whose recurrence residual (or the half
// step) meets the tolerance is marked for the true-residual test.
__global__ __launch_bounds__(64) void k_bicg_s_end(int R, const double* part, KState* st)
{
    if (!st->any_active) return;
    const int c = blockIdx.x;
    if (c >= R) return;
    const double v = sum_partials(part, SL_RR, c);
    if (lane_id() != 0) return;
    bicg_end_one(*st, c, v);
    const int chk = st->active[c] && (st->half[c] || st->rnorm2[c] <= st->tol2[c]);
    st->check[c] = chk;
    if (chk) atomicOr(&st->any_check, 1);
}

// After step `it` (0: after the setup), one wavefront, lane c for column c:
// a column marked for the test converges if its true residual meets the
// tolerance, else it restarts from it (r = r^ = b - A x).  Records the step
// at which each column stopped, sets the flags that gate the next step and
// copies any_active to *host_flag (mapped host memory, may be null), which
// the host reads a step later to stop queueing steps.
__global__ __launch_bounds__(64) void k_bicg_decide(int R, KState* st, int it, int* host_flag)
{
    const int c = lane_id();
    int restart = 0, active = 0;
    if (c < R) {
        if (st->check[c] && st->active[c]) {
            if (st->tnorm2[c] <= st->tol2[c]) {
                st->active[c] = 0;
                st->status[c] = ST_OK;
            } else {
                restart = 1;
                st->fresh[c] = 1;
                st->half[c] = 0;
                st->nrestart[c] += 1;
            }
        }
        st->check[c] = 0;
        st->restart[c] = restart;
        active = st->active[c];
        if (!active && st->done_it[c] < 0) st->done_it[c] = it;
    }
    const bool any_restart = __any(restart);
    const bool any_active = __any(active);
    if (c == 0) {
        st->any_check = 0;
        st->any_restart = any_restart ? 1 : 0;
        st->any_active = any_active ? 1 : 0;
        if (host_flag) __hip_atomic_store(host_flag, any_active ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// w = b - w (w holds A x on entry), partial of w.w
__global__ __launch_bounds__(kThreads) void k_resid(int64_t n, int R, const double* __restrict__ b,
                                                    double* __restrict__ w, double* part, int slot,
                                                    const int* gate = nullptr)
{
    if (gated_off(gate)) return;
    const RedIdx ri = red_index(R);
    double acc = 0.0;
    if (ri.live)
#pragma unroll 4
        for (int64_t g = ri.start; g < n * R; g += ri.stride) {
            const double v = b[g] - w[g];
            w[g] = v;
            acc += v * v;
        }
    block_partial(acc, R, slot_ptr(part, slot));
}

__global__ __launch_bounds__(64) void k_s_true(int R, const double* part, KState* st, const int* gate = nullptr)
{
    if (gated_off(gate)) return;
    const int c = blockIdx.x;
    if (c >= R) return;
    const double v = sum_partials(part, SL_TRUE, c);
    if (lane_id() == 0) st->tnorm2[c] = v;
}

// Restart of the columns flagged in st->restart: r = r^ = w (true residual).
__global__ void k_bicg_restart(int64_t n, int R, const double* __restrict__ w, double* __restrict__ r,
                               double* __restrict__ rh, KState* st)
{
    if (!st->any_restart) return;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n * R;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int c = static_cast<int>(g % R);
        if (!st->restart[c]) continue;
        r[g] = w[g];
        rh[g] = w[g];
    }
}

// ---------------------------------------------------------------------------
// GMRES(m) vector kernels (one right-hand side).  Modified Gram-Schmidt is
// run as a chain of fused passes over w: pass i subtracts the projection
// on v_{i-1} found by the previous pass (coefficient in *coef) and forms the
// partial dot product of the updated w with v_i; the last pass forms ||w||^2.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_gm_mgs(int64_t n, double* __restrict__ w,
                                                     const double* __restrict__ vprev,
                                                     const double* __restrict__ coef,
                                                     const double* __restrict__ vnext, double* part, int slot,
                                                     const int* gate = nullptr)
{
    if (gated_off(gate)) return;
    const RedIdx ri = red_index(1);
    double acc = 0.0;
    const double h = vprev ? *coef : 0.0;
    if (ri.live)
        for (int64_t g = ri.start; g < n; g += ri.stride) {
            double wv = w[g];
            if (vprev) {
                wv -= h * vprev[g];
                w[g] = wv;
            }
            acc += wv * (vnext ? vnext[g] : wv);
        }
    block_partial(acc, 1, slot_ptr(part, slot));
}

// h = sum of partials; mode 0: *hout = h, *coef = h (next projection);
// mode 1: h = sqrt(sum), *hout = h, *coef = 1/h (normalisation, 0 if h == 0).
__global__ __launch_bounds__(64) void k_gm_h(const double* part, int slot, double* hout, double* coef, int mode,
                                             const int* gate = nullptr)
{
    if (gated_off(gate)) return;
    double h = sum_partials(part, slot, 0);
    if (threadIdx.x != 0) return;
    if (mode == 1) {
        h = sqrt(h);
        *coef = h != 0.0 ? 1.0 / h : 0.0;
    } else {
        *coef = h;
    }
    *hout = h;
}

__global__ void k_gm_scale(int64_t n, const double* __restrict__ w, const double* __restrict__ coef,
                           double* __restrict__ v, const int* gate = nullptr)
{
    if (gated_off(gate)) return;
    const double s = *coef;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x)
        v[g] = w[g] * s;
}

// u = sum_k y_k v_k over the first m basis vectors (fixed order per entry);
// m is read from *mcount when given
__global__ void k_gm_combine(int64_t n, int m, const double* __restrict__ V, const double* __restrict__ y,
                             double* __restrict__ u, const int* mcount = nullptr)
{
    if (mcount) m = *mcount;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += y[k] * V[static_cast<int64_t>(k) * n + g];
        u[g] = s;
    }
}

// Device-side state of a GMRES(m) cycle: the Givens rotations and the
// rotated right-hand side g of the least-squares problem, beside the
// Hessenberg matrix (column j contiguous, m + 1 entries).
enum { GM_ACTIVE = 0, GM_JEND = 1, GM_BREAKDOWN = 2, GM_STEPS = 3, GM_NFLAGS = 4 };
struct GmView {
    double* H;          // (m+1) x m, column-major
    double* cs;         // [m]
    double* sn;         // [m]
    double* g;          // [m+1]
    double* y;          // [m]
    int* flags;         // [GM_NFLAGS]
    int m;
};

// Start of a cycle: g = (beta, 0, ...), beta = H[0] as left there by the
// true-residual norm; the cycle may take `steps` Arnoldi steps.
__global__ void k_gm_begin(GmView v, int steps)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    v.g[0] = v.H[0];
    for (int i = 1; i <= v.m; ++i) v.g[i] = 0.0;
    v.flags[GM_ACTIVE] = steps > 0 ? 1 : 0;
    v.flags[GM_JEND] = 0;
    v.flags[GM_BREAKDOWN] = 0;
    v.flags[GM_STEPS] = 0;
}

// After Arnoldi step j (column j of H complete): the earlier rotations on
// column j, the new rotation that zeroes H[j+1][j], g rotated.  The cycle
// stops when |g[j+1]| <= tol, when H[j+1][j] was 0 (the Krylov space is
// invariant) or after `steps` steps; the step count and "still active" are
// recorded, and the latter copied to *host_flag (mapped host memory).
__global__ void k_gm_givens(GmView v, int j, int steps, double tol, int* host_flag)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (!v.flags[GM_ACTIVE]) {
        if (host_flag) __hip_atomic_store(host_flag, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        return;
    }
    double* col = v.H + static_cast<int64_t>(j) * (v.m + 1);
    const double hnext = col[j + 1];
    for (int i = 0; i < j; ++i) {
        const double a1 = col[i], a2 = col[i + 1];
        col[i] = v.cs[i] * a1 + v.sn[i] * a2;
        col[i + 1] = -v.sn[i] * a1 + v.cs[i] * a2;
    }
    const double a1 = col[j], a2 = col[j + 1];
    const double rr = hypot(a1, a2);
    if (rr == 0.0) {
        v.cs[j] = 1.0;
        v.sn[j] = 0.0;
    } else {
        v.cs[j] = a1 / rr;
        v.sn[j] = a2 / rr;
    }
    col[j] = v.cs[j] * a1 + v.sn[j] * a2;
    col[j + 1] = 0.0;
    v.g[j + 1] = -v.sn[j] * v.g[j];
    v.g[j] = v.cs[j] * v.g[j];
    v.flags[GM_JEND] = j + 1;
    v.flags[GM_STEPS] = j + 1;
    const bool stop = fabs(v.g[j + 1]) <= tol || j + 1 >= steps || hnext == 0.0;
    if (stop) v.flags[GM_ACTIVE] = 0;
    if (host_flag) __hip_atomic_store(host_flag, stop ? 0 : 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// End of a cycle: y from the triangular system H[0:k, 0:k] y = g[0:k],
// k = the cycle's step count; a zero diagonal entry records a breakdown
// and leaves no update (step count set to 0).
__global__ void k_gm_solve_y(GmView v)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int k = v.flags[GM_JEND];
    const int ld = v.m + 1;
    for (int i = k - 1; i >= 0; --i) {
        double sum = v.g[i];
        for (int q = i + 1; q < k; ++q) sum -= v.H[static_cast<int64_t>(q) * ld + i] * v.y[q];
        const double d = v.H[static_cast<int64_t>(i) * ld + i];
        if (d == 0.0) {
            v.flags[GM_BREAKDOWN] = 1;
            v.flags[GM_JEND] = 0;
            return;
        }
        v.y[i] = sum / d;
    }
}

__global__ void k_axpy1(int64_t n, double* __restrict__ x, const double* __restrict__ z)
{
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x)
        x[g] += z[g];
}

// ---------------------------------------------------------------------------
// ORTHOMIN(k), right-preconditioned, one right-hand side, every decision on
// the device.  The directions p and their A-images q sit in rings of k + 1
// vectors; the direction of iteration it (1-based) is ring slot (it-1) mod
// (k+1), and the `count` kept directions are the slots before it, oldest
// first.  A restart from the true residual drops them (count = 0).
// ---------------------------------------------------------------------------
constexpr int kOmMax = 16;            // most directions kept

struct OmState {
    double qq[kOmMax + 1];            // (q_i, q_i) per ring slot
    double beta[kOmMax];              // coefficients of the kept directions, oldest first
    double alpha, bnorm2, tol2, rnorm2, tnorm2;
    int count;                        // directions kept before the current one
    int active, check, restart, status, done_it, nrestart, pad;
};

__device__ __forceinline__ int om_slot(int s, int count, int i, int K1)
{
    return ((s - count + i) % K1 + K1) % K1;
}

// setup: ||b||^2 from the partials, tolerance, flags (x = 0, r = b by the host)
__global__ __launch_bounds__(64) void k_om_init(const double* part, OmState* st, double rtol)
{
    const double b2 = sum_partials(part, SL_BB, 0);
    if (lane_id() != 0) return;
    st->bnorm2 = b2;
    st->tol2 = rtol * rtol * b2;
    st->rnorm2 = b2;
    st->tnorm2 = b2;
    st->active = b2 > 0.0 ? 1 : 0;
    st->status = b2 > 0.0 ? ST_NOT_CONV : ST_OK;
    st->count = 0;
    st->check = 0;
    st->restart = 0;
    st->done_it = st->active ? -1 : 0;
    st->nrestart = 0;
}

// partials of (q_s, q_i) for the kept directions i (column i of slot SL_RHO)
__global__ __launch_bounds__(kThreads) void k_om_dots(int64_t n, const double* __restrict__ Q, int s, int K1,
                                                      const OmState* st, double* part)
{
    if (!st->active) return;
    const int count = st->count;
    const RedIdx ri = red_index(1);
    const double* q = Q + static_cast<int64_t>(s) * n;
    double acc[kOmMax];
#pragma unroll
    for (int i = 0; i < kOmMax; ++i) acc[i] = 0.0;
    if (ri.live)
        for (int64_t g = ri.start; g < n; g += ri.stride) {
            const double qv = q[g];
#pragma unroll
            for (int i = 0; i < kOmMax; ++i)
                if (i < count) acc[i] += qv * Q[static_cast<int64_t>(om_slot(s, count, i, K1)) * n + g];
        }
    double* ps = slot_ptr(part, SL_RHO);
    for (int i = 0; i < count; ++i) block_partial(acc[i], 1, ps + static_cast<int64_t>(i) * kRedBlocks);
}

// beta_i = -(q_s, q_i) / (q_i, q_i)
__global__ __launch_bounds__(64) void k_om_beta(const double* part, OmState* st, int s, int K1)
{
    if (!st->active) return;
    const int count = st->count;
    for (int i = 0; i < count; ++i) {
        const double d = sum_partials(part, SL_RHO, i);
        if (lane_id() == 0) st->beta[i] = -d / st->qq[om_slot(s, count, i, K1)];
    }
}

// p_s += sum_i beta_i p_i, q_s += sum_i beta_i q_i (oldest first), partials
// of (q_s, q_s) and (r, q_s)
__global__ __launch_bounds__(kThreads) void k_om_update(int64_t n, double* __restrict__ P, double* __restrict__ Q,
                                                        const double* __restrict__ r, int s, int K1,
                                                        const OmState* st, double* part)
{
    if (!st->active) return;
    const int count = st->count;
    const RedIdx ri = red_index(1);
    double* p = P + static_cast<int64_t>(s) * n;
    double* q = Q + static_cast<int64_t>(s) * n;
    double qq = 0.0, rq = 0.0;
    if (ri.live)
        for (int64_t g = ri.start; g < n; g += ri.stride) {
            double pv = p[g], qv = q[g];
            for (int i = 0; i < count; ++i) {
                const int64_t o = static_cast<int64_t>(om_slot(s, count, i, K1)) * n + g;
                const double bt = st->beta[i];
                pv += bt * P[o];
                qv += bt * Q[o];
            }
            p[g] = pv;
            q[g] = qv;
            qq += qv * qv;
            rq += r[g] * qv;
        }
    block_partial(qq, 1, slot_ptr(part, SL_TT));
    block_partial(rq, 1, slot_ptr(part, SL_TS));
}

// alpha = (r, q_s) / (q_s, q_s); a zero (q, q) is a breakdown
__global__ __launch_bounds__(64) void k_om_alpha(const double* part, OmState* st, int s)
{
    if (!st->active) return;
    const double qq = sum_partials(part, SL_TT, 0);
    const double rq = sum_partials(part, SL_TS, 0);
    if (lane_id() != 0) return;
    st->qq[s] = qq;
    if (!isfinite(qq) || !isfinite(rq)) {
        st->status = ST_NONFINITE;
        st->active = 0;
    } else if (qq == 0.0) {
        st->status = ST_BREAKDOWN;
        st->active = 0;
    } else {
        st->alpha = rq / qq;
    }
}

// x += alpha p_s, r -= alpha q_s, partial of (r, r)
__global__ __launch_bounds__(kThreads) void k_om_xr(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ P, const double* __restrict__ Q,
                                                    int s, const OmState* st, double* part)
{
    if (!st->active) return;
    const RedIdx ri = red_index(1);
    const double al = st->alpha;
    const double* p = P + static_cast<int64_t>(s) * n;
    const double* q = Q + static_cast<int64_t>(s) * n;
    double rr = 0.0;
    if (ri.live)
        for (int64_t g = ri.start; g < n; g += ri.stride) {
            x[g] += al * p[g];
            const double rv = r[g] - al * q[g];
            r[g] = rv;
            rr += rv * rv;
        }
    block_partial(rr, 1, slot_ptr(part, SL_RR));
}

// End of an iteration: ||r||^2, one more kept direction (at most k), and
// the mark for the true-residual test when the recurrence residual passes.
__global__ __launch_bounds__(64) void k_om_end(const double* part, OmState* st, int k)
{
    if (!st->active) return;
    const double r2 = sum_partials(part, SL_RR, 0);
    if (lane_id() != 0) return;
    st->rnorm2 = r2;
    st->count = st->count < k ? st->count + 1 : k;
    if (!isfinite(r2)) {
        st->status = ST_NONFINITE;
        st->active = 0;
        return;
    }
    st->check = r2 <= st->tol2 ? 1 : 0;
}

// After iteration `it` (0: after the setup): a marked iteration stops if the
// true residual meets the tolerance, else restarts from it (r = b - A x,
// kept directions dropped).  Records the stopping iteration and copies
// "still active" to *host_flag (mapped host memory).
__global__ __launch_bounds__(64) void k_om_decide(const double* part, OmState* st, int it, int* host_flag)
{
    const bool checked = st->check && st->active;
    const double t2 = checked ? sum_partials(part, SL_TRUE, 0) : 0.0;
    if (lane_id() != 0) return;
    st->restart = 0;
    if (checked) {
        st->tnorm2 = t2;
        if (t2 <= st->tol2) {
            st->active = 0;
            st->status = ST_OK;
        } else {
            st->restart = 1;
            st->count = 0;
            st->nrestart += 1;
        }
    }
    st->check = 0;
    if (!st->active && st->done_it < 0) st->done_it = it;
    if (host_flag) __hip_atomic_store(host_flag, st->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// r = w (the true residual) after a restart
__global__ void k_om_restart(int64_t n, const double* __restrict__ w, double* __restrict__ r, const OmState* st)
{
    if (!st->restart) return;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n;
         g += static_cast<int64_t>(gridDim.x) * blockDim.x)
        r[g] = w[g];
}

// ||b - A x||^2 of the final x into tnorm2 (whatever the flags)
__global__ __launch_bounds__(64) void k_om_final(const double* part, OmState* st)
{
    const double t2 = sum_partials(part, SL_TRUE, 0);
    if (lane_id() == 0) st->tnorm2 = t2;
}

}  // namespace dev
}  // namespace bilu
