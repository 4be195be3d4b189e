// Kernels for a batch of independent systems of uneven sizes and block
// sizes, solved together: each sweep and each SpMV over the whole batch is
// one launch with a work queue of (system, tile) or (system, rows) items,
// and the Krylov scalars live per system in device memory.  Included once, by
// bilu_api.hip, after kernels.h.
//
// Batch vectors are the systems' vectors laid end to end: system s owns
// unknowns [voff_s, voff_s + nb_s * bs_s).
#pragma once

#include "kernels.h"

namespace bilu {
namespace dev {

// One system as the batch kernels see it.
struct BatchSys {
    const int32_t* Ap;      // A's block structure and values, for the SpMV
    const int32_t* Aj;
    const double* Ax;
    int64_t voff;           // first unknown of the system in the batch vectors
    int nb;
    int bs;
};

// Krylov scalars of every system (arrays of length nsys, device memory),
// the per-system bookkeeping of the true-residual test (check: marked for
// it this step; nrestart: restarts so far; done_it: step at which the
// system stopped, -1 while it runs) and three batch-wide flags that gate
// the kernels of a step: flags[0] some system is active, flags[1] some
// system is marked for the test, flags[2] some system restarts.
struct BatchState {
    double *rho, *rho_old, *alpha, *omega, *beta, *bnorm2, *tol2, *snorm2, *rnorm2, *tnorm2;
    int *active, *fresh, *half, *status, *restart, *check, *nrestart, *done_it;
    int* flags;
};

// A piece of the batch vectors: a range of unknowns inside one system.
// Pieces are the work units of the vector kernels and the leaves of the
// per-system reductions (fixed, so every sum has a fixed order).
struct Piece {
    int64_t begin, end;
    int sys;
    int pad;
};

constexpr int kPieceLen = 16384;

#define BILU_BATCH_SWITCH_B(bs, CALL)                   \
    switch (bs) {                                       \
    case 1: { constexpr int B = 1; CALL; } break;       \
    case 2: { constexpr int B = 2; CALL; } break;       \
    case 3: { constexpr int B = 3; CALL; } break;       \
    case 4: { constexpr int B = 4; CALL; } break;       \
    case 5: { constexpr int B = 5; CALL; } break;       \
    case 6: { constexpr int B = 6; CALL; } break;       \
    case 7: { constexpr int B = 7; CALL; } break;       \
    case 8: { constexpr int B = 8; CALL; } break;       \
    default: break;                                     \
    }

// ---------------------------------------------------------------------------
// y = A x over the batch: items are (system, first block row of a
// wavefront's 64/b rows); wavefronts take items grid-stride.
// ---------------------------------------------------------------------------
struct BatchSpmvArgs {
    const BatchSys* sys;
    const int2* items;
    int nitems;
    const double* x;
    double* y;
    const int* active;        // per system, or null
    const int* gate;          // nothing runs when given and *gate == 0
};

__global__ __launch_bounds__(kThreads) void k_spmv_batch(BatchSpmvArgs a)
{
    const int waves = static_cast<int>(gridDim.x) * kWavesPerBlock;
    if (gated_off(a.gate)) return;
    const int first = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x) * kWavesPerBlock +
                                                     static_cast<int>(threadIdx.x >> 6));
    for (int w = first; w < a.nitems; w += waves) {
        const int2 it = uniform_record(a.items, w);
        if (a.active && !uniform_load(a.active, it.x)) continue;
        const BatchSys S = uniform_record(a.sys, it.x);
        BILU_BATCH_SWITCH_B(S.bs, (spmv_rows<B, 1, false>(it.y, S.nb, S.Ap, S.Aj, nullptr, S.Ax, 0, a.x + S.voff,
                                                          a.y + S.voff, 1)))
    }
}

// ---------------------------------------------------------------------------
// Vector kernels: one workgroup per piece.  Partials are stored as
// part[slot * npieces + piece]; the per-system sums run over the system's
// pieces in order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v)
{
    __shared__ double sred[kThreads];
    __syncthreads();
    sred[threadIdx.x] = v;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (static_cast<int>(threadIdx.x) < h) sred[threadIdx.x] += sred[threadIdx.x + h];
        __syncthreads();
    }
    return sred[0];
}

__device__ __forceinline__ bool piece_live(const Piece& pc, const int* active)
{
    return !active || active[pc.sys];
}

// part[slot] = <a, b> per piece (0 for frozen systems when active is given);
// nothing runs when gate is given and *gate == 0
__global__ __launch_bounds__(kThreads) void kb_dot(const Piece* pieces, int npieces, const double* __restrict__ a,
                                                   const double* __restrict__ b, const int* active, double* part,
                                                   int slot, const int* gate)
{
    if (gated_off(gate)) return;
    const Piece pc = pieces[blockIdx.x];
    double acc = 0.0;
    if (piece_live(pc, active))
        for (int64_t g = pc.begin + threadIdx.x; g < pc.end; g += kThreads) acc += a[g] * b[g];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) part[static_cast<int64_t>(slot) * npieces + blockIdx.x] = s;
}

// <t, s> and <t, t>
__global__ __launch_bounds__(kThreads) void kb_dot2(const Piece* pieces, int npieces, const double* __restrict__ t,
                                                    const double* __restrict__ s, const int* active, double* part,
                                                    int slot_ts, int slot_tt, const int* gate)
{
    if (gated_off(gate)) return;
    const Piece pc = pieces[blockIdx.x];
    double ts = 0.0, tt = 0.0;
    if (piece_live(pc, active))
        for (int64_t g = pc.begin + threadIdx.x; g < pc.end; g += kThreads) {
            const double tv = t[g];
            ts += tv * s[g];
            tt += tv * tv;
        }
    const double a1 = block_sum(ts);
    const double a2 = block_sum(tt);
    if (threadIdx.x == 0) {
        part[static_cast<int64_t>(slot_ts) * npieces + blockIdx.x] = a1;
        part[static_cast<int64_t>(slot_tt) * npieces + blockIdx.x] = a2;
    }
}

__device__ __forceinline__ double sum_pieces(const double* part, int slot, int npieces, int p0, int p1)
{
    const double* q = part + static_cast<int64_t>(slot) * npieces;
    double s = 0.0;
    for (int p = p0; p < p1; ++p) s += q[p];
    return s;
}

// The scalar steps of BiCGSTAB for every system (one thread per system).
// KB_END also marks a system whose recurrence residual (or half step) meets
// the tolerance for the true-residual test; KB_TRUE_CHECKED takes the true
// residual of the marked systems only, KB_TRUE of every system.  Nothing
// runs when gate is given and *gate == 0.
enum { KB_INIT = 0, KB_RHO, KB_ALPHA, KB_SNORM, KB_OMEGA, KB_END, KB_TRUE, KB_TRUE_CHECKED };

__global__ void kb_scalar(int nsys, const int32_t* __restrict__ piece_ptr, int npieces, const double* part,
                          BatchState st, int op, double rtol, const int* gate)
{
    if (gated_off(gate)) return;
    const int c = static_cast<int>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= nsys) return;
    const int p0 = piece_ptr[c], p1 = piece_ptr[c + 1];
    switch (op) {
    case KB_INIT:
        bicg_init_one(st, c, sum_pieces(part, SL_BB, npieces, p0, p1), rtol);
        st.check[c] = 0;
        st.nrestart[c] = 0;
        st.done_it[c] = -1;
        break;
    case KB_RHO: bicg_rho_one(st, c, sum_pieces(part, SL_RHO, npieces, p0, p1)); break;
    case KB_ALPHA: bicg_alpha_one(st, c, sum_pieces(part, SL_RV, npieces, p0, p1)); break;
    case KB_SNORM: bicg_snorm_one(st, c, sum_pieces(part, SL_SS, npieces, p0, p1)); break;
    case KB_OMEGA:
        bicg_omega_one(st, c, sum_pieces(part, SL_TS, npieces, p0, p1), sum_pieces(part, SL_TT, npieces, p0, p1));
        break;
    case KB_END: {
        bicg_end_one(st, c, sum_pieces(part, SL_RR, npieces, p0, p1));
        const int chk = st.active[c] && (st.half[c] || st.rnorm2[c] <= st.tol2[c]);
        st.check[c] = chk;
        if (chk) atomicOr(st.flags + 1, 1);
        break;
    }
    case KB_TRUE: st.tnorm2[c] = sum_pieces(part, SL_TRUE, npieces, p0, p1); break;
    case KB_TRUE_CHECKED:
        if (st.check[c]) st.tnorm2[c] = sum_pieces(part, SL_TRUE, npieces, p0, p1);
        break;
    default: break;
    }
}

// p = r (first step) or r + beta (p - omega v)
__global__ __launch_bounds__(kThreads) void kb_p(const Piece* pieces, const double* __restrict__ r,
                                                 const double* __restrict__ v, double* __restrict__ p, BatchState st)
{
    if (!st.flags[0]) return;
    const Piece pc = pieces[blockIdx.x];
    const int c = pc.sys;
    if (!st.active[c]) return;
    const bool fresh = st.fresh[c] != 0;
    const double be = st.beta[c], om = st.omega[c];
    for (int64_t g = pc.begin + threadIdx.x; g < pc.end; g += kThreads)
        p[g] = fresh ? r[g] : r[g] + be * (p[g] - om * v[g]);
}

// s = r - alpha v, partial of <s, s>
__global__ __launch_bounds__(kThreads) void kb_s(const Piece* pieces, int npieces, const double* __restrict__ r,
                                                 const double* __restrict__ v, double* __restrict__ s, BatchState st,
                                                 double* part)
{
    if (!st.flags[0]) return;
    const Piece pc = pieces[blockIdx.x];
    const int c = pc.sys;
    double acc = 0.0;
    if (st.active[c]) {
        const double al = st.alpha[c];
        for (int64_t g = pc.begin + threadIdx.x; g < pc.end; g += kThreads) {
            const double sv = r[g] - al * v[g];
            s[g] = sv;
            acc += sv * sv;
        }
    }
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) part[static_cast<int64_t>(SL_SS) * npieces + blockIdx.x] = tot;
}

// x += alpha p^ (+ omega s^ unless the half step converged), r = s - omega t,
// partial of <r, r>
__global__ __launch_bounds__(kThreads) void kb_xr(const Piece* pieces, int npieces, double* __restrict__ x,
                                                  double* __restrict__ r, const double* __restrict__ ph,
                                                  const double* __restrict__ sh, const double* __restrict__ s,
                                                  const double* __restrict__ t, BatchState st, double* part)
{
    if (!st.flags[0]) return;
    const Piece pc = pieces[blockIdx.x];
    const int c = pc.sys;
    double acc = 0.0;
    if (st.active[c]) {
        const double al = st.alpha[c];
        if (st.half[c]) {
            for (int64_t g = pc.begin + threadIdx.x; g < pc.end; g += kThreads) x[g] += al * ph[g];
        } else {
            const double om = st.omega[c];
            for (int64_t g = pc.begin + threadIdx.x; g < pc.end; g += kThreads) {
                x[g] += al * ph[g] + om * sh[g];
                const double rv = s[g] - om * t[g];
                r[g] = rv;
                acc += rv * rv;
            }
        }
    }
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) part[static_cast<int64_t>(SL_RR) * npieces + blockIdx.x] = tot;
}

// w = b - w (w holds A x on entry), partial of <w, w>, for the systems
// marked in `active` (all if null); nothing runs when gate is given and
// *gate == 0
__global__ __launch_bounds__(kThreads) void kb_resid(const Piece* pieces, int npieces, const double* __restrict__ b,
                                                     double* __restrict__ w, double* part, int slot,
                                                     const int* active, const int* gate)
{
    if (gated_off(gate)) return;
    const Piece pc = pieces[blockIdx.x];
    double acc = 0.0;
    if (piece_live(pc, active))
        for (int64_t g = pc.begin + threadIdx.x; g < pc.end; g += kThreads) {
            const double v = b[g] - w[g];
            w[g] = v;
            acc += v * v;
        }
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) part[static_cast<int64_t>(slot) * npieces + blockIdx.x] = tot;
}

// r = r^ = w for the systems flagged for a restart
__global__ __launch_bounds__(kThreads) void kb_restart(const Piece* pieces, const double* __restrict__ w,
                                                       double* __restrict__ r, double* __restrict__ rh, BatchState st)
{
    if (!st.flags[2]) return;
    const Piece pc = pieces[blockIdx.x];
    if (!st.restart[pc.sys]) return;
    for (int64_t g = pc.begin + threadIdx.x; g < pc.end; g += kThreads) {
        r[g] = w[g];
        rh[g] = w[g];
    }
}

// After step `it` (0: after the setup), one workgroup over every system: a
// system marked for the test stops if its true residual meets the
// tolerance, else it restarts from it (r = r^ = b - A x).  Records the step
// at which each system stopped, sets the batch-wide flags that gate the
// next step and copies flags[0] to *host_flag (mapped host memory), which
// the host reads a step later to stop queueing steps.
__global__ __launch_bounds__(256) void kb_decide(int nsys, BatchState st, int it, int* host_flag)
{
    int any_restart = 0, any_active = 0;
    for (int c = static_cast<int>(threadIdx.x); c < nsys; c += static_cast<int>(blockDim.x)) {
        int restart = 0;
        if (st.check[c] && st.active[c]) {
            if (st.tnorm2[c] <= st.tol2[c]) {
                st.active[c] = 0;
                st.status[c] = ST_OK;
            } else {
                restart = 1;
                st.fresh[c] = 1;
                st.half[c] = 0;
                st.nrestart[c] += 1;
            }
        }
        st.check[c] = 0;
        st.restart[c] = restart;
        const int active = st.active[c];
        if (!active && st.done_it[c] < 0) st.done_it[c] = it;
        any_restart |= restart;
        any_active |= active;
    }
    any_restart = __syncthreads_or(any_restart);
    any_active = __syncthreads_or(any_active);
    if (threadIdx.x == 0) {
        st.flags[0] = any_active ? 1 : 0;
        st.flags[1] = 0;
        st.flags[2] = any_restart ? 1 : 0;
        if (host_flag) __hip_atomic_store(host_flag, any_active ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace dev
}  // namespace bilu
