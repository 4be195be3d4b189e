// Sweep and SpMV kernels for gfx950 (CDNA4, wave64): device helpers, the
// level-scheduled sweeps and the block SpMV.  Kernel templates are
// instantiated only in sweep_b.hip (one translation unit per block size)
// and batch_sweep.hip; other translation units use the types and helpers.
//
// Block values are column-major b x b (Section 2.1).  Vectors are
// (nb*b) x R row-major.  All floating-point accumulation is FP64; factor
// values may be stored as FP32 and are widened before they are multiplied.
#pragma once

#include <hip/hip_runtime.h>
#include <climits>
#include <cstdint>

#include "bilu_internal.h"

namespace bilu {
namespace dev {

constexpr int kThreads = 256;          // 4 wavefronts per workgroup
constexpr int kWavesPerBlock = kThreads / 64;
constexpr int kRedBlocks = 512;        // fixed grid of the two-stage reductions
constexpr int kMaxRhs = 32;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ double widen(float v) { return static_cast<double>(v); }

// ---------------------------------------------------------------------------
// Readiness inside one persistent sweep is carried by the values themselves.
// Before a sweep starts, every entry of its output vector holds kNotReady,
// a signalling-NaN bit pattern that no arithmetic result can have (results
// are quiet NaNs at worst, and a result that would copy the pattern is
// replaced by the canonical quiet NaN).  A row is published by writing its
// values with device-coherent stores; a reader polls each value it needs
// with device-coherent loads until it differs from kNotReady.  No flags, no
// fences, no cache maintenance: one memory round trip per dependency.
// The invariant "output starts at kNotReady" is kept by the two sweeps of
// an application: the first resets the second's output rows, the second
// resets the first's output rows after it has read them.
// ---------------------------------------------------------------------------
constexpr unsigned long long kNotReadyBits = 0x7FF4DEADBEEF1234ULL;
constexpr unsigned long long kQuietNaNBits = 0x7FF8000000000000ULL;

__device__ __forceinline__ double not_ready() { return __longlong_as_double(static_cast<long long>(kNotReadyBits)); }

__device__ __forceinline__ bool is_not_ready(double v)
{
    return static_cast<unsigned long long>(__double_as_longlong(v)) == kNotReadyBits;
}

__device__ __forceinline__ double publishable(double v)
{
    return is_not_ready(v) ? __longlong_as_double(static_cast<long long>(kQuietNaNBits)) : v;
}

__device__ __forceinline__ double coherent_load(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void coherent_store(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits (bounded) until *p is published; returns the value.  Past the limit
// the timeout is recorded in *status and whatever was read is returned, so
// the wavefront still finishes.
__device__ __forceinline__ double await_value(const double* p, double v, unsigned int limit, int* status)
{
    unsigned int spins = 0;
    while (is_not_ready(v)) {
        if (++spins > limit) {
            atomicOr(status, 1);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
        v = coherent_load(p);
    }
    return v;
}

// Waits (bounded) until none of the values v[(g*B + c)*RT + t] shows
// kNotReady, for the rows j[g] >= 0 (g < G), components c < B and columns
// t < RT with c0 + t < R; the value lives at out[(j[g]*B + c)*R + c0 + t].
// Each poll re-reads every value still missing with a device-coherent load,
// all in one round trip.  Past the limit the timeout is recorded in *status
// and whatever was read is kept, so the wavefront still finishes.
template <int G, int B, int RT>
__device__ __forceinline__ bool rows_missing(const double (&v)[G * B * RT], const int (&j)[G], int R, int c0)
{
    // bitwise, not short-circuit: no branches
    bool pending = false;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int c = 0; c < B; ++c)
#pragma unroll
            for (int t = 0; t < RT; ++t)
                pending |= (j[g] >= 0) & (RT == 1 || c0 + t < R) & is_not_ready(v[(g * B + c) * RT + t]);
    return pending;
}

template <int G, int B, int RT>
__device__ __forceinline__ void await_rows(double (&v)[G * B * RT], const int (&j)[G], const double* out, int R,
                                           int c0, unsigned int limit, int* status)
{
    // the first test reads only the values at hand, outside the loop, so
    // the common case waits for nothing else
    bool pending = rows_missing<G, B, RT>(v, j, R, c0);
    for (unsigned int spins = 0; pending;) {
        if (++spins > limit) {
            atomicOr(status, 1);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int c = 0; c < B; ++c)
#pragma unroll
                for (int t = 0; t < RT; ++t) {
                    const int i = (g * B + c) * RT + t;
                    if (j[g] >= 0 && (RT == 1 || c0 + t < R) && is_not_ready(v[i]))
                        v[i] = coherent_load(out + (static_cast<int64_t>(j[g]) * B + c) * R + c0 + t);
                }
        pending = rows_missing<G, B, RT>(v, j, R, c0);
    }
}

// Read-only, wave-uniform load through the constant address space, which
// the compiler turns into a scalar load (its own counter, so vector loads in
// flight are not waited for).  Only for data no kernel writes while it runs.
template <typename T>
__device__ __forceinline__ T uniform_load(const T* p, int64_t i)
{
    return ((const __attribute__((address_space(4))) T*)p)[i];
}

// The same for a trivially copyable record, word by word.
template <typename T>
__device__ __forceinline__ T uniform_record(const T* p, int64_t i)
{
    static_assert(sizeof(T) % 4 == 0, "record of whole words");
    constexpr int kWords = static_cast<int>(sizeof(T) / 4);
    const int* w = reinterpret_cast<const int*>(p + i);
    union {
        int words[kWords];
        T rec;
    } u;
#pragma unroll
    for (int k = 0; k < kWords; ++k) u.words[k] = uniform_load(w, k);
    return u.rec;
}

// A launch whose gate (a device flag written by an earlier kernel on the
// stream, or null) reads 0 does nothing: the solvers gate the work of an
// iteration that was queued after every right-hand side had finished.
__device__ __forceinline__ bool gated_off(const int* gate)
{
    return gate != nullptr && uniform_load(gate, 0) == 0;
}

__device__ __forceinline__ int grab_ticket(unsigned long long* ticket)
{
    unsigned long long t = 0;
    if (lane_id() == 0) t = atomicAdd(ticket, 1ULL);
    t = __shfl(t, 0);
    return t > 0x3fffffffULL ? 0x3fffffff : static_cast<int>(t);
}

// The last wavefront of a persistent launch to finish rewinds the ticket
// for the next launch on the stream (every wavefront takes exactly one
// ticket past the end, so all tickets have been taken by then).
__device__ __forceinline__ void finish_persistent(unsigned long long* ticket, unsigned int* done,
                                                  unsigned int total_waves)
{
    if (lane_id() == 0) {
        const unsigned int prev = atomicAdd(done, 1u);
        if (prev + 1 == total_waves) {
            __hip_atomic_store(ticket, 0ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// Level-scheduled sweep (Eq 4, Algorithm 6) of one unit-diagonal block
// triangular factor, optionally with the block-diagonal D^{-1} product of
// Algorithm 7 fused in front:
//     out_i = (fuse ? Dv_i rhs_i : rhs_i) - sum_k F_ik out_{col(i,k)}
// Level-chunk form: one wavefront per chunk of rpc = 64/B block rows of one
// level; lane (q, r) = (lane / B, lane % B) owns component r of the
// chunk's q-th row.  Values of a chunk are stored [k][c][r][q], so for a
// fixed dependency k and block column c the wavefront reads B*rpc
// consecutive values.
//
// persistent = 0: the launch covers the chunks [chunk_begin, chunk_end) of
// one level, all of whose dependencies were written by earlier launches.
// persistent = 1: one launch covers the whole sweep; wavefronts take chunks
// in level order from an atomic ticket and poll the values they read.  A
// chunk only reads rows of chunks with smaller tickets, held by wavefronts
// that are already running, so the sweep always drains.
// ---------------------------------------------------------------------------
struct SweepArgs {
    const int64_t* chunk_off;
    const int32_t* rows;
    const int32_t* cols;
    const void* vals;
    const void* dinv;
    const double* rhs;
    double* out;
    double* reset;      // rows of this buffer are set to kNotReady (may be null)
    unsigned long long* ticket;
    unsigned int* done;
    int* status;
    int nchunks;
    int chunk_begin;
    int chunk_end;
    int R;
    int fuse;
    int persistent;
    unsigned int total_waves;
    unsigned int spin_limit;
    const int* gate;    // nothing runs when *gate == 0 (may be null)
};

// One chunk of a level-chunk sweep, by one wavefront.
template <int B, typename T, int RT>
__device__ __forceinline__ void sweep_chunk(SweepArgs a, int chunk)
{
    constexpr int RPC = 64 / B;
    constexpr int BB = B * B;
    const int lane = lane_id();
    const int q = lane / B;
    const int r = lane - q * B;
    const bool lane_ok = q < RPC;
    const T* __restrict__ vals = static_cast<const T*>(a.vals);
    const T* __restrict__ dinv = static_cast<const T*>(a.dinv);
    const int R = a.R;
    const int row = lane_ok ? a.rows[static_cast<int64_t>(chunk) * RPC + q] : -1;
    const int64_t off = a.chunk_off[chunk];
    const int w = static_cast<int>((a.chunk_off[chunk + 1] - off) / RPC);
    if (row < 0) return;
    for (int c0 = 0; c0 < R; c0 += RT) {
        double acc[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[t] = 0.0;
        if (a.fuse) {
            const int64_t dbase = static_cast<int64_t>(chunk) * RPC * BB + r * RPC + q;
#pragma unroll
            for (int c = 0; c < B; ++c) {
                const double d = widen(dinv[dbase + c * B * RPC]);
                const double* src = a.rhs + (static_cast<int64_t>(row) * B + c) * R + c0;
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    if (RT == 1 || c0 + t < R) acc[t] += d * src[t];
            }
        } else {
            const double* src = a.rhs + (static_cast<int64_t>(row) * B + r) * R + c0;
#pragma unroll
            for (int t = 0; t < RT; ++t)
                if (RT == 1 || c0 + t < R) acc[t] = src[t];
        }
        // dependencies in groups of KG: all their values are requested
        // together and missing ones polled together (one round trip each)
        constexpr int KG = RT == 1 ? (B <= 4 ? 4 : 2) : 1;
        for (int k0 = 0; k0 < w; k0 += KG) {
            int j[KG];
#pragma unroll
            for (int g = 0; g < KG; ++g)
                j[g] = k0 + g < w ? a.cols[off + static_cast<int64_t>(k0 + g) * RPC + q] : -1;
            double xv[KG * B * RT];
#pragma unroll
            for (int g = 0; g < KG; ++g)
#pragma unroll
                for (int c = 0; c < B; ++c)
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        const double* xp = a.out + (static_cast<int64_t>(j[g]) * B + c) * R + c0 + t;
                        const bool want = j[g] >= 0 && (RT == 1 || c0 + t < R);
                        xv[(g * B + c) * RT + t] = want ? (a.persistent ? coherent_load(xp) : *xp) : 0.0;
                    }
            if (a.persistent) await_rows<KG, B, RT>(xv, j, a.out, R, c0, a.spin_limit, a.status);
#pragma unroll
            for (int g = 0; g < KG; ++g) {
                if (j[g] < 0) continue;
                const int64_t vbase = (off + static_cast<int64_t>(k0 + g) * RPC) * BB + r * RPC + q;
#pragma unroll
                for (int c = 0; c < B; ++c) {
                    const double v = widen(vals[vbase + c * B * RPC]);
#pragma unroll
                    for (int t = 0; t < RT; ++t)
                        if (RT == 1 || c0 + t < R) acc[t] -= v * xv[(g * B + c) * RT + t];
                }
            }
        }
        const int64_t o = (static_cast<int64_t>(row) * B + r) * R + c0;
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            if (RT == 1 || c0 + t < R) {
                if (a.reset) a.reset[o + t] = not_ready();
                if (a.persistent) coherent_store(a.out + o + t, publishable(acc[t]));
                else a.out[o + t] = publishable(acc[t]);
            }
        }
    }
}

template <int B, typename T, int RT>
__global__ __launch_bounds__(kThreads) void k_sweep(SweepArgs a)
{
    if (gated_off(a.gate)) return;
    if (a.persistent) {
        for (int chunk = grab_ticket(a.ticket); chunk < a.nchunks; chunk = grab_ticket(a.ticket))
            sweep_chunk<B, T, RT>(a, chunk);
        finish_persistent(a.ticket, a.done, a.total_waves);
    } else {
        const int chunk = a.chunk_begin + static_cast<int>(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6);
        if (chunk < a.chunk_end) sweep_chunk<B, T, RT>(a, chunk);
    }
}

// ---------------------------------------------------------------------------
// Tiled sweep: one wavefront owns a contiguous range of block rows (a tile)
// and walks it in its own level order (levels of Eq 4 restricted to the
// dependencies inside the tile), one chunk of up to 64/B rows at a time.
// A dependency inside the tile is read from LDS, where the wavefront keeps
// every row it has finished; a dependency on another tile is read from
// global memory.  Tiles are taken from a ticket in sweep order, and every
// row a tile reads from outside lies in an earlier tile, so the sweep
// drains.  Dependency codes are byte offsets: code >= 0 is row code/(8B) of
// the vectors, code < 0 is byte (code & INT32_MAX) of the tile's LDS; a
// padding slot points at LDS row tile_rows, kept at zero, and has zero
// factor values.  A wavefront sweeps one right-hand side (MULTI: one per
// (tile, column)); k_sweep_grouped runs several tiles per workgroup.
//
// The walk is software-pipelined over a ring of NR register states: at step
// i the wavefront issues the metadata loads of chunk i + 2(NR-1) (row ids,
// dependency codes), the data loads of chunk i + NR - 1 (factor values,
// right-hand side, D^{-1} row, values read from other tiles, addressed by
// metadata that arrived NR - 1 steps earlier) and computes chunk i.  Every
// batch is branch-free with a fixed instruction count: chunk indices past
// the tile clamp to its last chunk, and the first KMAX slot rows of a chunk
// are always read (every chunk has at least KMAX).  Chunk-wide addresses
// are scalar; a lane adds a fixed offset, so the per-slot loads need no
// vector address arithmetic.  Values from other tiles are prefetched with plain,
// cacheable loads: during a sweep an output location only ever holds
// kNotReady or its final value, so a stale cached copy can only show
// kNotReady, and the values still showing it are then polled together with
// device-coherent loads.  Dependencies past the first KMAX of a row take an
// unpipelined path.
// ---------------------------------------------------------------------------
struct TiledArgs {
    const int32_t* tile_chunk_ptr;
    const int32_t* tile_lo;
    const int32_t* chunk_row;     // first slot row of each chunk (slot offset / (64/B))
    const int32_t* rows;
    const int32_t* deps;
    const void* vals;
    const void* dinv;
    const double* rhs;
    double* out;
    double* reset;
    unsigned long long* ticket;
    unsigned int* done;
    int* status;
    int ntiles;
    int tile_rows;                // LDS row group*tile_rows is kept at zero (ring: ring*64/B)
    int ring;                     // > 0: LDS keeps the rows of the last `ring` chunks only
    int R;                        // right-hand sides (vectors are (n x R) row-major)
    unsigned int total_waves;     // grouped: workgroups
    unsigned int spin_limit;
    // tile groups (k_sweep_grouped): member m of group g sweeps
    // group_tiles[g*group + m]; chunk_wait[c*kGroupMax + m] chunks of member m
    // must be finished before chunk c reads the group's LDS
    const int32_t* group_tiles;
    const int32_t* chunk_wait;
    int group;
    int ngroups;
    const int* gate;              // nothing runs when *gate == 0 (may be null)
#ifdef BILU_TRACE
    long long* trace;             // [nchunks] finish time of each chunk, then [ntiles] start of each tile
    int trace_nchunks;
#endif
};

// Byte offset of component c of a block row (row_byte = row * B * 8) in the
// column this wavefront sweeps.  One right-hand side: row_byte + 8c.
// Several (MULTI): the vectors are (n x R) row-major, element (i, j) at
// i*R + j.
template <bool MULTI>
struct ColMap {
    uint32_t R;
    uint32_t j8;      // 8 * column
    __device__ __forceinline__ uint32_t at(uint32_t row_byte, int c) const
    {
        return MULTI ? row_byte * R + static_cast<uint32_t>(c) * 8u * R + j8 : row_byte + static_cast<uint32_t>(c) * 8u;
    }
};

// Load at a 32-bit byte offset from a (wave-uniform) base: the address is
// formed by the load itself.  Vectors of the tiled sweep are below 2 GiB.
template <typename T>
__device__ __forceinline__ T load_at(const T* base, uint32_t byte_off)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

template <int KMAX>
struct TileMeta {
    int64_t off;         // first slot of the chunk (wave-uniform)
    int w;               // slots per row (wave-uniform)
    int row;             // as loaded (unused row slots hold -1)
    int code[KMAX];      // dependency codes of slot rows 0..KMAX-1
};

template <int B, typename T, int KMAX, bool FUSE>
struct TileData {
    int64_t off;
    int w;
    int row;
    int code[KMAX];
    T f[KMAX][B];        // factor values as stored
    double x[KMAX][B];   // values read from other tiles (may show kNotReady)
    double h[FUSE ? B : 1];
    T d[FUSE ? B : 1];
};

// `chunk` is wave-uniform; its first slot row and width (srow, w) were
// read through the scalar cache a step earlier, and every address below is
// a scalar base plus a per-lane constant.
template <int B, int KMAX>
__device__ __forceinline__ void tile_meta(const TiledArgs& a, int chunk, int srow, int w, int qc,
                                          TileMeta<KMAX>& m)
{
    constexpr int RPC = 64 / B;
    m.off = static_cast<int64_t>(srow) * RPC;
    m.w = w;
    const int32_t* rp = a.rows + static_cast<int64_t>(chunk) * RPC;
    const int32_t* dp = a.deps + m.off;
    m.row = rp[qc];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) m.code[k] = dp[k * RPC + qc];
}

template <int B, typename T, int KMAX, bool FUSE, bool MULTI, bool HELP = false>
__device__ __forceinline__ void tile_data(const TiledArgs& a, int chunk, int qc, int r, const TileMeta<KMAX>& m,
                                          TileData<B, T, KMAX, FUSE>& s, const ColMap<MULTI>& cm)
{
    constexpr int RPC = 64 / B;
    constexpr int BB = B * B;
    const int lane_off = r * RPC + qc;
    s.off = m.off;
    s.w = m.w;
    s.row = m.row;
    const T* vp = static_cast<const T*>(a.vals) + m.off * BB;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        s.code[k] = m.code[k];
#pragma unroll
        for (int c = 0; c < B; ++c) s.f[k][c] = vp[k * RPC * BB + c * B * RPC + lane_off];
    }
    // unused row slots of a partly filled chunk hold -1: read row 0 instead
    const uint32_t rowc_b = static_cast<uint32_t>(m.row >= 0 ? m.row : 0) * (B * 8u);
    if (FUSE) {
        const T* dp = static_cast<const T*>(a.dinv) + static_cast<int64_t>(chunk) * RPC * BB;
#pragma unroll
        for (int c = 0; c < B; ++c) {
            s.h[c] = load_at(a.rhs, cm.at(rowc_b, c));
            s.d[c] = dp[c * B * RPC + lane_off];
        }
    } else {
        s.h[0] = load_at(a.rhs, cm.at(rowc_b, r));
    }
    // tile-local and padding slots do not use the value: every such lane
    // reads row 0, so the wavefront touches one cache line for them.  With a
    // helper wavefront the values of other tiles come through LDS instead.
    if constexpr (!HELP) {
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const uint32_t xb = s.code[k] >= 0 ? static_cast<uint32_t>(s.code[k]) : 0u;
#pragma unroll
            for (int c = 0; c < B; ++c) s.x[k][c] = load_at(static_cast<const double*>(a.out), cm.at(xb, c));
        }
    }
}

// Waits (bounded) until no value of another tile that a lane needs shows
// kNotReady; every value still missing is re-read with a device-coherent
// load, all in one round trip per poll.
template <int K, int B, bool MULTI>
__device__ __forceinline__ unsigned int await_tile(double (&v)[K * B], const int (&code)[K], const double* out,
                                                   const ColMap<MULTI>& cm, unsigned int limit, int* status)
{
    bool pending = false;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < B; ++c) pending |= (code[k] >= 0) & is_not_ready(v[k * B + c]);
    unsigned int spins = 0;
    while (pending) {
        if (++spins > limit) {
            atomicOr(status, 1);
            return spins;
        }
        __builtin_amdgcn_s_sleep(1);
        pending = false;
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < B; ++c)
                if (code[k] >= 0 && is_not_ready(v[k * B + c]))
                    v[k * B + c] = coherent_load(reinterpret_cast<const double*>(
                        reinterpret_cast<const char*>(out) + cm.at(static_cast<uint32_t>(code[k]), c)));
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < B; ++c) pending |= (code[k] >= 0) & is_not_ready(v[k * B + c]);
    }
    return spins;
}

// Tile groups: waits (bounded) until each earlier member of the workgroup has
// finished the chunks this chunk reads from it.  A member publishes its count
// of finished chunks in LDS after the chunk's rows; the LDS operations of one
// wavefront take effect in issue order, so a count that is seen covers every
// row written before it.
__device__ __forceinline__ void await_members(const int* prog, const int (&need)[kGroupMax], unsigned int limit,
                                              int* status)
{
    for (unsigned int spins = 0;;) {
        bool behind = false;
#pragma unroll
        for (int m = 0; m < kGroupMax; ++m)
            behind |= __hip_atomic_load(prog + m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < need[m];
        if (!behind) break;
        if (++spins > limit) {
            atomicOr(status, 1);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    // the row reads that follow stay after the counts
    asm volatile("" ::: "memory");
}

// Helper wavefronts (k_sweep_grouped<..., HELP>): next to each member
// wavefront of a tile group runs a helper wavefront that reads the member's
// values from other tiles, chunk by chunk in the member's order, polls those
// still showing kNotReady, and hands them over through an LDS ring of
// kHelpRing chunks ([chunk % kHelpRing][slot value][lane]), publishing its
// count of delivered chunks after them.  The member then issues no load of
// another tile's values: its vector loads are prefetches only, which
// complete in issue order, so no poll waits behind them, and it can keep a
// deeper prefetch ring.  The helper refills a ring entry once the member's
// progress count shows that the member has finished the chunk held there
// (kHelpRing: bilu_internal.h, shared with the host's LDS sizing).

// Waits (bounded) until the LDS count *cnt reaches need.
__device__ __forceinline__ void await_count(const int* cnt, int need, unsigned int limit, int* status)
{
    for (unsigned int spins = 0;
         __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < need;) {
        if (++spins > limit) {
            atomicOr(status, 1);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    asm volatile("" ::: "memory");
}

// The member side of a helper's ring: count of chunks delivered, the
// member's ring and the index of the chunk in the member's tile.
struct HelpView {
    const int* hprog;
    const double* ring;
    int idx;
};

// lds: the workgroup's LDS (dependency codes are offsets into it);
// tile_vals: this tile's rows in it.
template <int B, typename T, int KMAX, bool FUSE, bool MULTI, bool GROUPED, bool HELP = false>
__device__ __forceinline__ void tile_compute(const TiledArgs& a, int lo, int qc, int r, bool active,
                                             const double* lds_base, double* tile_vals,
                                             const TileData<B, T, KMAX, FUSE>& s, const int (&need)[kGroupMax],
                                             const int* prog, const ColMap<MULTI>& cm, int wbase, const HelpView& hv
#ifdef BILU_TRACE
                                             , long long* trc
#endif
)
{
    constexpr int RPC = 64 / B;
    constexpr int BB = B * B;
    // Every lane takes delivery of the whole batch here, also lanes that
    // compute nothing: the compiler then never finds a load of this batch
    // still in flight when it reuses its registers, which would cost a wait
    // for all later loads.
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
#pragma unroll
        for (int c = 0; c < B; ++c) {
            asm volatile("" ::"v"(s.f[k][c]));
            if constexpr (!HELP) asm volatile("" ::"v"(s.x[k][c]));
        }
    }
#pragma unroll
    for (int c = 0; c < (FUSE ? B : 1); ++c) asm volatile("" ::"v"(s.h[c]), "v"(s.d[c]));
    // values from other tiles: the prefetched copies, the ones still showing
    // kNotReady polled together; with a helper, its ring entry once the
    // helper has delivered this chunk
    double xg[KMAX * B];
    if constexpr (HELP) {
        await_count(hv.hprog, hv.idx + 1, a.spin_limit, a.status);
        const double* rs = hv.ring + (hv.idx % kHelpRing) * (KMAX * B * 64) + lane_id();
#pragma unroll
        for (int j = 0; j < KMAX * B; ++j) xg[j] = rs[j * 64];
        if (GROUPED) await_members(prog, need, a.spin_limit, a.status);
    } else {
#pragma unroll
        for (int k = 0; k < KMAX; ++k)
#pragma unroll
            for (int c = 0; c < B; ++c) xg[k * B + c] = s.x[k][c];
#ifdef BILU_TRACE
        if (trc && lane_id() == 0) trc[1] = wall_clock64();
        const unsigned int spins_ = await_tile<KMAX, B, MULTI>(xg, s.code, a.out, cm, a.spin_limit, a.status);
        if (GROUPED) await_members(prog, need, a.spin_limit, a.status);
        if (trc && lane_id() == 0) { trc[2] = wall_clock64(); trc[3] = spins_; }
#else
        await_tile<KMAX, B, MULTI>(xg, s.code, a.out, cm, a.spin_limit, a.status);
        if (GROUPED) await_members(prog, need, a.spin_limit, a.status);
#endif
    }
    if (!active || s.row < 0) return;
    double acc;
    if (FUSE) {
        acc = 0.0;
#pragma unroll
        for (int c = 0; c < B; ++c) acc += widen(s.d[c]) * s.h[c];
    } else {
        acc = s.h[0];
    }
    // branch-free: every slot reads LDS (its own row for tile-local and
    // padding slots, row 0 otherwise) and selects.  Each LDS value is handed
    // to an empty asm statement once all are issued, so the compiler keeps
    // the reads unconditional (instead of turning each select into a branch
    // around its read) and waits for them once.
    const char* lds = reinterpret_cast<const char*>(lds_base);
    double lv[KMAX * B];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const uint32_t lb = s.code[k] < 0 ? static_cast<uint32_t>(s.code[k]) & 0x7fffffffu : 0u;
#pragma unroll
        for (int c = 0; c < B; ++c) lv[k * B + c] = *reinterpret_cast<const double*>(lds + lb + c * 8u);
    }
#pragma unroll
    for (int i = 0; i < KMAX * B; ++i) asm volatile("" : "+v"(lv[i]));
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const bool local = s.code[k] < 0;
#pragma unroll
        for (int c = 0; c < B; ++c) acc -= widen(s.f[k][c]) * (local ? lv[k * B + c] : xg[k * B + c]);
    }
    if (s.w > KMAX) {
        // slots past the first KMAX, XB at a time: their codes in one round
        // trip, then factor values and dependency values (LDS, or other
        // tiles' values polled together) in the next; products subtracted
        // in slot order, as for the first KMAX
        constexpr int XB = B == 1 ? 16 : B == 2 ? 8 : (16 / B > 2 ? 16 / B : 2);
        const T* __restrict__ vals = static_cast<const T*>(a.vals);
        const char* ob = reinterpret_cast<const char*>(a.out);
        for (int k0 = KMAX; k0 < s.w; k0 += XB) {
            int code[XB];
#pragma unroll
            for (int j = 0; j < XB; ++j)
                code[j] = k0 + j < s.w ? a.deps[s.off + static_cast<int64_t>(k0 + j) * RPC + qc] : INT_MIN;
            double xv[XB * B];
            T fv[XB][B];
#pragma unroll
            for (int j = 0; j < XB; ++j) {
                const int k = k0 + j < s.w ? k0 + j : k0;
                const int64_t vbase = (s.off + static_cast<int64_t>(k) * RPC) * BB + r * RPC + qc;
                const uint32_t lb = code[j] < 0 ? static_cast<uint32_t>(code[j]) & 0x7fffffffu : 0u;
                const uint32_t gb = code[j] >= 0 ? static_cast<uint32_t>(code[j]) : 0u;
#pragma unroll
                for (int c = 0; c < B; ++c) {
                    fv[j][c] = vals[vbase + c * B * RPC];
                    const double lx = *reinterpret_cast<const double*>(lds + lb + c * 8u);
                    const double gx = *reinterpret_cast<const double*>(ob + cm.at(gb, c));
                    xv[j * B + c] = code[j] < 0 ? lx : gx;
                }
            }
            await_tile<XB, B, MULTI>(xv, code, a.out, cm, a.spin_limit, a.status);
#pragma unroll
            for (int j = 0; j < XB; ++j)
                if (k0 + j < s.w)
#pragma unroll
                    for (int c = 0; c < B; ++c) acc -= widen(fv[j][c]) * xv[j * B + c];
        }
    }
    const double v = publishable(acc);
    const uint32_t ob = cm.at(static_cast<uint32_t>(s.row) * (B * 8u), r);
    if (a.reset) *reinterpret_cast<double*>(reinterpret_cast<char*>(a.reset) + ob) = not_ready();
    coherent_store(reinterpret_cast<double*>(reinterpret_cast<char*>(a.out) + ob), v);
    // the row's LDS slot: its place in the tile, or in the ring (wbase >= 0)
    tile_vals[(wbase >= 0 ? wbase + qc : s.row - lo) * B + r] = v;
}

// Ring depth: three register states where they fit in half the register
// file (two wavefronts per SIMD), else two.  Tile groups take two: measured on
// MI355X, the member wavefronts of a group (one compute unit, all near the
// sweep front) run their sweeps faster with fewer loads in flight (60x220x85
// ILU(0), groups of 3: U' sweep 528 -> 497 us), while a wavefront on its own
// gains from the deeper ring.
template <int B, typename T, bool FUSE, int KMAX, bool GROUPED, bool HELP = false>
struct TiledRing {
    static constexpr int w = sizeof(T) == 8 ? 2 : 1;
    static constexpr int state = KMAX * B * ((HELP ? 0 : 2) + w) + KMAX + (FUSE ? B * (2 + w) : 2) + 4 + KMAX + 3;
    // with a helper the member's loads are prefetches only: a deeper ring
    static constexpr int value = HELP ? (4 * state + 40 <= 200 ? 4 : 3 * state + 40 <= 220 ? 3 : 2)
                                      : (!GROUPED && 3 * state + 40 <= 240 ? 3 : 2);
};

// One tile of a tiled sweep by one wavefront (column cm of the vectors).
// tile_vals: the wavefront's LDS, row a.tile_rows already zero.
template <int B, typename T, bool FUSE, int KMAX, bool MULTI, bool GROUPED, bool HELP = false>
__device__ __forceinline__ void run_tile(const TiledArgs& a, int t, const ColMap<MULTI>& cm, const double* lds_base,
                                         double* tile_vals, int* prog, int member, const int* hprog = nullptr,
                                         const double* ring = nullptr)
{
    constexpr int RPC = 64 / B;
    constexpr int NR = TiledRing<B, T, FUSE, KMAX, GROUPED, HELP>::value;   // register states in flight
    constexpr int LD = NR - 1;                               // data lookahead
    constexpr int LM = 2 * LD;                               // metadata lookahead
    const int lane = lane_id();
    const int q = lane / B;
    const int r = lane - q * B;
    const bool lane_ok = q < RPC;
    const int qc = lane_ok ? q : RPC - 1;
    TileMeta<KMAX> mr[NR];
    TileData<B, T, KMAX, FUSE> dr[NR];
    int wr[NR][kGroupMax];                                   // grouped: the chunks' waits
    const int lo = uniform_load(a.tile_lo, t);
    const int c0 = uniform_load(a.tile_chunk_ptr, t);
    const int nch = uniform_load(a.tile_chunk_ptr, t + 1) - c0;
    if (nch <= 0) return;
#ifdef BILU_TRACE
    if (a.trace && lane == 0) a.trace[4 * a.trace_nchunks + t] = wall_clock64();
#endif
    const int clast = c0 + nch - 1;
    auto chunk_at = [&](int i) { return min(c0 + i, clast); };
    auto meta_at = [&](int i, TileMeta<KMAX>& m) {
        const int ch = chunk_at(i);
        const int sr = uniform_load(a.chunk_row, ch);
        tile_meta<B, KMAX>(a, ch, sr, uniform_load(a.chunk_row, ch + 1) - sr, qc, m);
    };
    // waits of chunk i, read with its data (scalar loads)
    auto wait_at = [&](int i, int (&w)[kGroupMax]) {
#pragma unroll
        for (int m = 0; m < kGroupMax; ++m)
            w[m] = GROUPED && a.group > 1 ? uniform_load(a.chunk_wait, chunk_at(i) * kGroupMax + m) : 0;
    };
    // prologue: metadata of chunks 0..NR-1, then data of 0..LD-1 with the
    // metadata of LD..LM-1 issued as their slots free up
#pragma unroll
    for (int i = 0; i < NR; ++i) meta_at(i, mr[i]);
#pragma unroll
    for (int i = 0; i < LD; ++i) {
        tile_data<B, T, KMAX, FUSE, MULTI, HELP>(a, chunk_at(i), qc, r, mr[i % NR], dr[i % NR], cm);
        wait_at(i, wr[i % NR]);
        if (NR + i < LM) meta_at(NR + i, mr[(NR + i) % NR]);
    }
    // slot row range of the next chunk whose metadata is due, read a step
    // ahead so that no step waits on the scalar cache
    int pre_lo = uniform_load(a.chunk_row, chunk_at(LM));
    int pre_hi = uniform_load(a.chunk_row, chunk_at(LM) + 1);
    int wchunk = 0;                                          // ring position of the chunk computed next
    // whole turns of the ring; steps past the tile's end load clamped
    // chunks and compute nothing
    for (int i0 = 0; i0 < nch; i0 += NR) {
#pragma unroll
        for (int p = 0; p < NR; ++p) {
            const int i = i0 + p;
            tile_meta<B, KMAX>(a, chunk_at(i + LM), pre_lo, pre_hi - pre_lo, qc, mr[(p + LM) % NR]);
            pre_lo = uniform_load(a.chunk_row, chunk_at(i + LM + 1));
            pre_hi = uniform_load(a.chunk_row, chunk_at(i + LM + 1) + 1);
            tile_data<B, T, KMAX, FUSE, MULTI, HELP>(a, chunk_at(i + LD), qc, r, mr[(p + LD) % NR], dr[(p + LD) % NR],
                                                     cm);
            wait_at(i + LD, wr[(p + LD) % NR]);
            const HelpView hv{hprog, ring, i < nch ? i : nch - 1};
            tile_compute<B, T, KMAX, FUSE, MULTI, GROUPED, HELP>(a, lo, qc, r, lane_ok && i < nch, lds_base, tile_vals,
                                                                 dr[p], wr[p], prog, cm,
                                                                 a.ring > 0 ? wchunk * RPC : -1, hv
#ifdef BILU_TRACE
                                                           , (a.trace && i < nch) ? a.trace + 4 * (c0 + i) : nullptr
#endif
            );
            wchunk = wchunk + 1 == a.ring ? 0 : wchunk + 1;
#ifdef BILU_TRACE
            if (a.trace && lane == 0 && i < nch) a.trace[4 * (c0 + i)] = wall_clock64();
#endif
            // one wavefront: its LDS accesses complete in issue order, so
            // only the compiler must keep this chunk's writes before the
            // next chunk's reads (and before the progress count)
            __builtin_amdgcn_wave_barrier();
            asm volatile("" ::: "memory");
            if (GROUPED && i < nch && lane == 0)
                __hip_atomic_store(prog + member, i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
}

// The helper wavefront of one member tile: for each chunk in the member's
// order, the values of other tiles its lanes need (the same slots, lanes and
// columns as the member's), read with device-coherent loads and polled until
// none shows kNotReady, then written to the member's LDS ring once the
// member has finished the chunk that entry held, and the delivered count
// published after them (one wavefront: its LDS operations take effect in
// issue order).  The dependency codes of the next chunk are loaded while
// the current chunk's values are awaited.
template <int B, int KMAX, bool MULTI>
__device__ __forceinline__ void run_helper(const TiledArgs& a, int t, const ColMap<MULTI>& cm, double* ring,
                                           int* hprog, const int* prog)
{
    constexpr int RPC = 64 / B;
    const int lane = lane_id();
    const int q = lane / B;
    const int qc = q < RPC ? q : RPC - 1;
    const int c0 = uniform_load(a.tile_chunk_ptr, t);
    const int nch = uniform_load(a.tile_chunk_ptr, t + 1) - c0;
    if (nch <= 0) return;
    auto meta_at = [&](int i, TileMeta<KMAX>& m) {
        const int ch = c0 + (i < nch ? i : nch - 1);
        const int sr = uniform_load(a.chunk_row, ch);
        tile_meta<B, KMAX>(a, ch, sr, uniform_load(a.chunk_row, ch + 1) - sr, qc, m);
    };
    TileMeta<KMAX> cur, nxt;
    meta_at(0, cur);
    for (int i = 0; i < nch; ++i) {
        double v[KMAX * B];
        // a chunk whose dependencies all lie in the group needs no load
        bool any = false;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) any |= cur.code[k] >= 0;
        const bool wave_any = __any(any ? 1 : 0) != 0;
        if (wave_any) {
#pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const uint32_t xb = cur.code[k] >= 0 ? static_cast<uint32_t>(cur.code[k]) : 0u;
#pragma unroll
                for (int c = 0; c < B; ++c)
                    v[k * B + c] = coherent_load(reinterpret_cast<const double*>(
                        reinterpret_cast<const char*>(a.out) + cm.at(xb, c)));
            }
        } else {
#pragma unroll
            for (int j = 0; j < KMAX * B; ++j) v[j] = 0.0;
        }
        meta_at(i + 1, nxt);
        if (wave_any) await_tile<KMAX, B, MULTI>(v, cur.code, a.out, cm, a.spin_limit, a.status);
        // the entry's previous chunk, i - kHelpRing, is finished
        await_count(prog, i - kHelpRing + 1, a.spin_limit, a.status);
        double* dst = ring + (i % kHelpRing) * (KMAX * B * 64) + lane;
#pragma unroll
        for (int j = 0; j < KMAX * B; ++j) dst[j * 64] = v[j];
        __builtin_amdgcn_wave_barrier();
        asm volatile("" ::: "memory");
        if (lane == 0) __hip_atomic_store(hprog, i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        cur = nxt;
    }
}

// MULTI: R right-hand sides swept side by side, one wavefront per (tile,
// column); tickets run tile by tile, the columns of a tile together, so
// every dependency of a ticket (same column, earlier tile) has a smaller one.
template <int B, typename T, bool FUSE, int KMAX, bool MULTI>
__global__ __launch_bounds__(64) void k_sweep_tiled(TiledArgs a)
{
    extern __shared__ double tile_vals[];                    // [tile rows + 1][B]
    if (gated_off(a.gate)) return;
    // LDS row tile_rows stays zero: padding slots read it
    if (lane_id() < B) tile_vals[a.tile_rows * B + lane_id()] = 0.0;
    const int nticket = MULTI ? a.ntiles * a.R : a.ntiles;
    for (int tk = __builtin_amdgcn_readfirstlane(grab_ticket(a.ticket)); tk < nticket;
         tk = __builtin_amdgcn_readfirstlane(grab_ticket(a.ticket))) {
        const int t = MULTI ? tk / a.R : tk;
        ColMap<MULTI> cm;
        cm.R = static_cast<uint32_t>(a.R);
        cm.j8 = MULTI ? static_cast<uint32_t>(tk - t * a.R) * 8u : 0u;
        run_tile<B, T, FUSE, KMAX, MULTI, false>(a, t, cm, tile_vals, tile_vals, nullptr, 0);
    }
    finish_persistent(a.ticket, a.done, a.total_waves);
}

// ---------------------------------------------------------------------------
// Two right-hand sides per wavefront (k_sweep_tiled_pairs, single tiles):
// columns j0 and j0 + 1 (j0 even) of the (n x R) row-major vectors, R even,
// lie next to each other, so every vector access of the one-column walk
// (right-hand side, values of other tiles, the published row, its reset,
// LDS) becomes one 16-byte access, while each factor block, dependency code
// and D^{-1} value is loaded once for both columns.  Each column is formed
// with the operations of the one-column sweep in the same order, so both
// give the same bits.  LDS keeps both columns of a row: (tile rows + 1) *
// B * 16 bytes, the dependency codes' LDS byte offsets doubled.
// ---------------------------------------------------------------------------
template <int B, typename T, int KMAX, bool FUSE>
struct TileDataP {
    int64_t off;
    int w;
    int row;
    int code[KMAX];
    T f[KMAX][B];
    double2 x[KMAX][B];      // values read from other tiles (may show kNotReady)
    double2 h[FUSE ? B : 1];
    T d[FUSE ? B : 1];
};

__device__ __forceinline__ bool pair_not_ready(const double2& v) { return is_not_ready(v.x) || is_not_ready(v.y); }

template <int B, typename T, int KMAX, bool FUSE>
__device__ __forceinline__ void tile_data_p(const TiledArgs& a, int chunk, int qc, int r, const TileMeta<KMAX>& m,
                                            TileDataP<B, T, KMAX, FUSE>& s, const ColMap<true>& cm)
{
    constexpr int RPC = 64 / B;
    constexpr int BB = B * B;
    const int lane_off = r * RPC + qc;
    s.off = m.off;
    s.w = m.w;
    s.row = m.row;
    const T* vp = static_cast<const T*>(a.vals) + m.off * BB;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        s.code[k] = m.code[k];
#pragma unroll
        for (int c = 0; c < B; ++c) s.f[k][c] = vp[k * RPC * BB + c * B * RPC + lane_off];
    }
    const uint32_t rowc_b = static_cast<uint32_t>(m.row >= 0 ? m.row : 0) * (B * 8u);
    const double2* rhs2 = reinterpret_cast<const double2*>(a.rhs);
    if (FUSE) {
        const T* dp = static_cast<const T*>(a.dinv) + static_cast<int64_t>(chunk) * RPC * BB;
#pragma unroll
        for (int c = 0; c < B; ++c) {
            s.h[c] = load_at(rhs2, cm.at(rowc_b, c));
            s.d[c] = dp[c * B * RPC + lane_off];
        }
    } else {
        s.h[0] = load_at(rhs2, cm.at(rowc_b, r));
    }
    const double2* out2 = reinterpret_cast<const double2*>(a.out);
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const uint32_t xb = s.code[k] >= 0 ? static_cast<uint32_t>(s.code[k]) : 0u;
#pragma unroll
        for (int c = 0; c < B; ++c) s.x[k][c] = load_at(out2, cm.at(xb, c));
    }
}

// await_tile for column pairs: each column of a pair is polled on its own
// (the two are published by two stores).
template <int K, int B>
__device__ __forceinline__ void await_tile_p(double2 (&v)[K * B], const int (&code)[K], const double* out,
                                             const ColMap<true>& cm, unsigned int limit, int* status)
{
    bool pending = false;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < B; ++c) pending |= (code[k] >= 0) & pair_not_ready(v[k * B + c]);
    unsigned int spins = 0;
    while (pending) {
        if (++spins > limit) {
            atomicOr(status, 1);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
        pending = false;
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < B; ++c)
                if (code[k] >= 0 && pair_not_ready(v[k * B + c])) {
                    const double* p = reinterpret_cast<const double*>(reinterpret_cast<const char*>(out) +
                                                                      cm.at(static_cast<uint32_t>(code[k]), c));
                    if (is_not_ready(v[k * B + c].x)) v[k * B + c].x = coherent_load(p);
                    if (is_not_ready(v[k * B + c].y)) v[k * B + c].y = coherent_load(p + 1);
                }
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < B; ++c) pending |= (code[k] >= 0) & pair_not_ready(v[k * B + c]);
    }
}

template <int B, typename T, int KMAX, bool FUSE>
__device__ __forceinline__ void tile_compute_p(const TiledArgs& a, int lo, int qc, int r, bool active,
                                               double2* tile_vals, const TileDataP<B, T, KMAX, FUSE>& s,
                                               const ColMap<true>& cm, int wbase)
{
    constexpr int RPC = 64 / B;
    constexpr int BB = B * B;
    // take delivery of the whole batch (see tile_compute)
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
#pragma unroll
        for (int c = 0; c < B; ++c) asm volatile("" ::"v"(s.f[k][c]), "v"(s.x[k][c].x), "v"(s.x[k][c].y));
    }
#pragma unroll
    for (int c = 0; c < (FUSE ? B : 1); ++c) asm volatile("" ::"v"(s.h[c].x), "v"(s.h[c].y), "v"(s.d[c]));
    double2 xg[KMAX * B];
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
#pragma unroll
        for (int c = 0; c < B; ++c) xg[k * B + c] = s.x[k][c];
    await_tile_p<KMAX, B>(xg, s.code, a.out, cm, a.spin_limit, a.status);
    if (!active || s.row < 0) return;
    double acc0, acc1;
    if (FUSE) {
        acc0 = 0.0;
        acc1 = 0.0;
#pragma unroll
        for (int c = 0; c < B; ++c) {
            acc0 += widen(s.d[c]) * s.h[c].x;
            acc1 += widen(s.d[c]) * s.h[c].y;
        }
    } else {
        acc0 = s.h[0].x;
        acc1 = s.h[0].y;
    }
    const char* lds = reinterpret_cast<const char*>(tile_vals);
    double2 lv[KMAX * B];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const uint32_t lb = s.code[k] < 0 ? 2u * (static_cast<uint32_t>(s.code[k]) & 0x7fffffffu) : 0u;
#pragma unroll
        for (int c = 0; c < B; ++c) lv[k * B + c] = *reinterpret_cast<const double2*>(lds + lb + c * 16u);
    }
#pragma unroll
    for (int i = 0; i < KMAX * B; ++i) asm volatile("" : "+v"(lv[i].x), "+v"(lv[i].y));
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const bool local = s.code[k] < 0;
#pragma unroll
        for (int c = 0; c < B; ++c) {
            const double f = widen(s.f[k][c]);
            acc0 -= f * (local ? lv[k * B + c].x : xg[k * B + c].x);
            acc1 -= f * (local ? lv[k * B + c].y : xg[k * B + c].y);
        }
    }
    if (s.w > KMAX) {
        // slots past the first KMAX, XB at a time, as in tile_compute
        constexpr int XB = B == 1 ? 16 : B == 2 ? 8 : (16 / B > 2 ? 16 / B : 2);
        const T* __restrict__ vals = static_cast<const T*>(a.vals);
        const char* ob = reinterpret_cast<const char*>(a.out);
        for (int k0 = KMAX; k0 < s.w; k0 += XB) {
            int code[XB];
#pragma unroll
            for (int j = 0; j < XB; ++j)
                code[j] = k0 + j < s.w ? a.deps[s.off + static_cast<int64_t>(k0 + j) * RPC + qc] : INT_MIN;
            double2 xv[XB * B];
            T fv[XB][B];
#pragma unroll
            for (int j = 0; j < XB; ++j) {
                const int k = k0 + j < s.w ? k0 + j : k0;
                const int64_t vbase = (s.off + static_cast<int64_t>(k) * RPC) * BB + r * RPC + qc;
                const uint32_t lb = code[j] < 0 ? 2u * (static_cast<uint32_t>(code[j]) & 0x7fffffffu) : 0u;
                const uint32_t gb = code[j] >= 0 ? static_cast<uint32_t>(code[j]) : 0u;
#pragma unroll
                for (int c = 0; c < B; ++c) {
                    fv[j][c] = vals[vbase + c * B * RPC];
                    const double2 lx = *reinterpret_cast<const double2*>(lds + lb + c * 16u);
                    const double2 gx = *reinterpret_cast<const double2*>(ob + cm.at(gb, c));
                    xv[j * B + c] = code[j] < 0 ? lx : gx;
                }
            }
            await_tile_p<XB, B>(xv, code, a.out, cm, a.spin_limit, a.status);
#pragma unroll
            for (int j = 0; j < XB; ++j)
                if (k0 + j < s.w)
#pragma unroll
                    for (int c = 0; c < B; ++c) {
                        acc0 -= widen(fv[j][c]) * xv[j * B + c].x;
                        acc1 -= widen(fv[j][c]) * xv[j * B + c].y;
                    }
        }
    }
    const double v0 = publishable(acc0);
    const double v1 = publishable(acc1);
    const uint32_t ob = cm.at(static_cast<uint32_t>(s.row) * (B * 8u), r);
    if (a.reset)
        *reinterpret_cast<double2*>(reinterpret_cast<char*>(a.reset) + ob) = make_double2(not_ready(), not_ready());
    double* dst = reinterpret_cast<double*>(reinterpret_cast<char*>(a.out) + ob);
    coherent_store(dst, v0);
    coherent_store(dst + 1, v1);
    tile_vals[(wbase >= 0 ? wbase + qc : s.row - lo) * B + r] = make_double2(v0, v1);
}

// Ring depth of the column-pair walk (as TiledRing for single tiles, with
// two values per vector element).
template <int B, typename T, bool FUSE, int KMAX>
struct TiledRingP {
    static constexpr int w = sizeof(T) == 8 ? 2 : 1;
    static constexpr int state = KMAX * B * (4 + w) + KMAX + (FUSE ? B * (4 + w) : 4) + 4 + KMAX + 3;
    static constexpr int value = 3 * state + 40 <= 240 ? 3 : 2;
};

// One tile, one column pair (run_tile without groups or helpers).
template <int B, typename T, bool FUSE, int KMAX>
__device__ __forceinline__ void run_tile_p(const TiledArgs& a, int t, const ColMap<true>& cm, double2* tile_vals)
{
    constexpr int RPC = 64 / B;
    constexpr int NR = TiledRingP<B, T, FUSE, KMAX>::value;
    constexpr int LD = NR - 1;
    constexpr int LM = 2 * LD;
    const int lane = lane_id();
    const int q = lane / B;
    const int r = lane - q * B;
    const bool lane_ok = q < RPC;
    const int qc = lane_ok ? q : RPC - 1;
    TileMeta<KMAX> mr[NR];
    TileDataP<B, T, KMAX, FUSE> dr[NR];
    const int lo = uniform_load(a.tile_lo, t);
    const int c0 = uniform_load(a.tile_chunk_ptr, t);
    const int nch = uniform_load(a.tile_chunk_ptr, t + 1) - c0;
    if (nch <= 0) return;
    const int clast = c0 + nch - 1;
    auto chunk_at = [&](int i) { return min(c0 + i, clast); };
    auto meta_at = [&](int i, TileMeta<KMAX>& m) {
        const int ch = chunk_at(i);
        const int sr = uniform_load(a.chunk_row, ch);
        tile_meta<B, KMAX>(a, ch, sr, uniform_load(a.chunk_row, ch + 1) - sr, qc, m);
    };
#pragma unroll
    for (int i = 0; i < NR; ++i) meta_at(i, mr[i]);
#pragma unroll
    for (int i = 0; i < LD; ++i) {
        tile_data_p<B, T, KMAX, FUSE>(a, chunk_at(i), qc, r, mr[i % NR], dr[i % NR], cm);
        if (NR + i < LM) meta_at(NR + i, mr[(NR + i) % NR]);
    }
    int pre_lo = uniform_load(a.chunk_row, chunk_at(LM));
    int pre_hi = uniform_load(a.chunk_row, chunk_at(LM) + 1);
    int wchunk = 0;
    for (int i0 = 0; i0 < nch; i0 += NR) {
#pragma unroll
        for (int p = 0; p < NR; ++p) {
            const int i = i0 + p;
            tile_meta<B, KMAX>(a, chunk_at(i + LM), pre_lo, pre_hi - pre_lo, qc, mr[(p + LM) % NR]);
            pre_lo = uniform_load(a.chunk_row, chunk_at(i + LM + 1));
            pre_hi = uniform_load(a.chunk_row, chunk_at(i + LM + 1) + 1);
            tile_data_p<B, T, KMAX, FUSE>(a, chunk_at(i + LD), qc, r, mr[(p + LD) % NR], dr[(p + LD) % NR], cm);
            tile_compute_p<B, T, KMAX, FUSE>(a, lo, qc, r, lane_ok && i < nch, tile_vals, dr[p], cm,
                                             a.ring > 0 ? wchunk * RPC : -1);
            wchunk = wchunk + 1 == a.ring ? 0 : wchunk + 1;
            __builtin_amdgcn_wave_barrier();
            asm volatile("" ::: "memory");
        }
    }
}

// Tickets: tiles times column pairs, the pairs of a tile together (every
// dependency of a ticket -- same columns, earlier tile -- has a smaller one).
template <int B, typename T, bool FUSE, int KMAX>
__global__ __launch_bounds__(64) void k_sweep_tiled_pairs(TiledArgs a)
{
    extern __shared__ double2 pair_vals[];                   // [tile rows + 1][B]
    if (gated_off(a.gate)) return;
    if (lane_id() < B) pair_vals[a.tile_rows * B + lane_id()] = make_double2(0.0, 0.0);
    const int npairs = a.R / 2;
    const int nticket = a.ntiles * npairs;
    for (int tk = __builtin_amdgcn_readfirstlane(grab_ticket(a.ticket)); tk < nticket;
         tk = __builtin_amdgcn_readfirstlane(grab_ticket(a.ticket))) {
        const int t = tk / npairs;
        ColMap<true> cm;
        cm.R = static_cast<uint32_t>(a.R);
        cm.j8 = static_cast<uint32_t>(tk - t * npairs) * 16u;
        run_tile_p<B, T, FUSE, KMAX>(a, t, cm, pair_vals);
    }
    finish_persistent(a.ticket, a.done, a.total_waves);
}

// Tile groups: one workgroup of a.group wavefronts per ticket (a group, or
// with MULTI a (group, column) pair); member m sweeps the group's m-th tile
// into its part of the shared LDS and reads rows of earlier members there
// once their progress counts cover them.  Tickets run in group order, and
// every row a group reads from outside lies in a group with a smaller
// ticket, so the persistent launch drains.
// HELP: a.group helper wavefronts follow the a.group members (workgroup of
// 2 * a.group wavefronts, a.group <= kHelpGroupMax; a.group may then be 1,
// with a.ngroups the number of tiles); LDS after the progress counts:
// kGroupMax delivered counts, then the members' rings.  At most four
// wavefronts per workgroup keep each wavefront's full register budget (one
// per SIMD), which the members' prefetch rings need.
template <int B, typename T, bool FUSE, int KMAX, bool MULTI, bool HELP>
__global__ __launch_bounds__(HELP ? 128 * kHelpGroupMax : 64 * kGroupMax) void k_sweep_grouped(TiledArgs a)
{
    extern __shared__ double group_vals[];   // [group*tile_rows + 1][B], then kGroupMax progress counts
    __shared__ int s_ticket;
    if (gated_off(a.gate)) return;
    const int G = a.group;
    // wave-uniform (the compiler cannot see that on its own): the member's
    // tile and chunk indices then stay scalar
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
    const bool helper = HELP && wave >= G;
    const int member = helper ? wave - G : wave;
    const int zrow = G * a.tile_rows;
    int* prog = reinterpret_cast<int*>(group_vals + static_cast<int64_t>(zrow + 1) * B);
    int* hprog = prog + kGroupMax;
    double* rings = reinterpret_cast<double*>(hprog + kGroupMax);
    double* ring = rings + static_cast<int64_t>(member) * (kHelpRing * KMAX * B * 64);
    if (static_cast<int>(threadIdx.x) < B) group_vals[zrow * B + threadIdx.x] = 0.0;
    const int nticket = MULTI ? a.ngroups * a.R : a.ngroups;
    for (;;) {
        // the previous group is finished by every member (barrier below)
        if (threadIdx.x < (HELP ? 2 : 1) * kGroupMax) prog[threadIdx.x] = 0;
        if (threadIdx.x == 0) {
            const unsigned long long tk = atomicAdd(a.ticket, 1ULL);
            s_ticket = tk > 0x3fffffffULL ? 0x3fffffff : static_cast<int>(tk);
        }
        __syncthreads();
        const int tk = __builtin_amdgcn_readfirstlane(s_ticket);
        if (tk >= nticket) break;
        const int g = MULTI ? tk / a.R : tk;
        const int t = member >= G ? -1 : G == 1 ? g : uniform_load(a.group_tiles, g * G + member);
        ColMap<MULTI> cm;
        cm.R = static_cast<uint32_t>(a.R);
        cm.j8 = MULTI ? static_cast<uint32_t>(tk - g * a.R) * 8u : 0u;
        if (t >= 0) {
            if (helper)
                run_helper<B, KMAX, MULTI>(a, t, cm, ring, hprog + member, prog + member);
            else
                run_tile<B, T, FUSE, KMAX, MULTI, true, HELP>(a, t, cm, group_vals,
                                                              group_vals + static_cast<int64_t>(member) * a.tile_rows * B,
                                                              prog, member, hprog + member, ring);
        }
        __syncthreads();
    }
    if (wave == 0) finish_persistent(a.ticket, a.done, a.total_waves);
}

// ---------------------------------------------------------------------------
// Line sweep: the sweep of a pattern in natural grid order (block rows in
// lines of nx along x, ny lines per plane, nz planes) whose rows depend only
// on their x-, y- and z-neighbour before them in the sweep (ILU(0) on a
// 7-point stencil).  In sweep coordinates (x~, y~, z~: the grid coordinates
// for a forward sweep, mirrored for a backward one) a row depends on
// (x~-1), (y~-1) and (z~-1).  A wavefront owns a block of WY x WZ lines
// (lane (q, r): component r of line q = yl + WY*zl) and at step s computes
// the row x~ = s - yl - zl of every line: the rows of one step are
// independent, the x~- and in-block y~/z~-neighbours were computed by the
// wavefront one step earlier and are exchanged through a small LDS area,
// and neighbours in the blocks before (y~ or z~ side) are read from the
// output vector, prefetched and polled with the data-carried readiness of
// the tiled sweeps.  Factor values arrive in the chunk format of the tiled
// layouts (chunk = block*nsteps + step, row slot q = line, slot k = the
// neighbour in the k-th dimension of the ascending column order: z~, y~, x~
// for L, x~, y~, z~ for U' with D^{-1} fused); row indices are computed, not
// loaded.  Every row is formed with the same operations in the same order as
// by the other sweeps.
// ---------------------------------------------------------------------------
struct LineArgs {
    const void* vals;
    const void* dinv;
    const double* rhs;
    double* out;
    double* reset;
    unsigned long long* ticket;
    unsigned int* done;
    int* status;
    const int* gate;
    int nx, ny, nz;
    int WY, WZ;               // lines per block along y~ and z~
    int NYb, nblocks;         // blocks along y~, blocks in all (ticket t: block t)
    int nsteps;               // nx + WY + WZ - 2
    int forward;
    unsigned int total_waves;
    unsigned int spin_limit;
#ifdef BILU_TRACE
    long long* trace;         // [nblocks*nsteps][4]: finish, wait begin, wait end, polls
#endif
};

template <int B, typename T, bool FUSE>
struct LineStage {
    T f[3][B];               // factor row r of the three neighbour blocks, as stored
    double h[FUSE ? B : 1];  // right-hand side (the whole row when D^{-1} is fused)
    T d[FUSE ? B : 1];       // row r of D^{-1}
    double ext[2][B];        // neighbour rows in earlier blocks (y~ side, z~ side)
};

template <int B, typename T, bool FUSE>
__device__ __forceinline__ void line_stage_load(const LineArgs& a, int chunk, int lane_off, int64_t rowc_b,
                                                int64_t ext_y_b, int64_t ext_z_b, LineStage<B, T, FUSE>& g)
{
    constexpr int RPC = 64 / B;
    constexpr int BB = B * B;
    const T* vp = static_cast<const T*>(a.vals) + static_cast<int64_t>(chunk) * 3 * RPC * BB;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < B; ++c) g.f[k][c] = vp[k * RPC * BB + c * B * RPC + lane_off];
    const char* rb = reinterpret_cast<const char*>(a.rhs);
    if (FUSE) {
        const T* dp = static_cast<const T*>(a.dinv) + static_cast<int64_t>(chunk) * RPC * BB;
#pragma unroll
        for (int c = 0; c < B; ++c) {
            g.h[c] = *reinterpret_cast<const double*>(rb + rowc_b + 8 * c);
            g.d[c] = dp[c * B * RPC + lane_off];
        }
    } else {
        g.h[0] = *reinterpret_cast<const double*>(rb + rowc_b + 8 * (lane_off / RPC));
    }
    const char* ob = reinterpret_cast<const char*>(a.out);
    // device-coherent: a cached copy of a line read before its neighbours
    // were published would show kNotReady for them
#pragma unroll
    for (int c = 0; c < B; ++c) {
        g.ext[0][c] = coherent_load(reinterpret_cast<const double*>(ob + ext_y_b + 8 * c));
        g.ext[1][c] = coherent_load(reinterpret_cast<const double*>(ob + ext_z_b + 8 * c));
    }
}

template <int B, typename T, bool FUSE>
__global__ __launch_bounds__(64) void k_sweep_lines(LineArgs a)
{
    constexpr int RPC = 64 / B;
    constexpr int NR = 3;                   // stages in flight
    __shared__ double xch[2][64];           // outputs of the last step, by lane
    if (gated_off(a.gate)) return;
    const int lane = lane_id();
    const int q = lane / B;
    const int r = lane - q * B;
    const int nlines = a.WY * a.WZ;
    const bool lane_ok = q < nlines && q < RPC;
    const int qc = lane_ok ? q : 0;
    const int yl = qc % a.WY;
    const int zl = qc / a.WY;
    const int lane_off = r * RPC + qc;
    const int nxy = a.nx * a.ny;
    const int sgn = a.forward ? 1 : -1;
    for (int tk = __builtin_amdgcn_readfirstlane(grab_ticket(a.ticket)); tk < a.nblocks;
         tk = __builtin_amdgcn_readfirstlane(grab_ticket(a.ticket))) {
        const int Yb = tk % a.NYb, Zb = tk / a.NYb;
        const int ys = Yb * a.WY + yl, zs = Zb * a.WZ + zl;    // sweep coordinates
        const bool line_ok = lane_ok && ys < a.ny && zs < a.nz;
        const int y = a.forward ? ys : a.ny - 1 - ys;
        const int z = a.forward ? zs : a.nz - 1 - zs;
        const int64_t line_row0 = a.forward ? static_cast<int64_t>(a.nx) * (y + static_cast<int64_t>(a.ny) * z)
                                            : static_cast<int64_t>(a.nx) * (y + static_cast<int64_t>(a.ny) * z) + a.nx - 1;
        // neighbours outside the block read from the output vector
        const bool ext_y = line_ok && yl == 0 && ys > 0;
        const bool ext_z = line_ok && zl == 0 && zs > 0;
        const int c0 = static_cast<int>(tk) * a.nsteps;
#ifdef BILU_TRACE
        if (a.trace && lane == 0) a.trace[4 * static_cast<int64_t>(a.nblocks) * a.nsteps + tk] = wall_clock64();
#endif
        auto row_at = [&](int s) -> int64_t {   // row of this line at step s (any x~, clamped)
            int xs = s - yl - zl;
            xs = xs < 0 ? 0 : (xs >= a.nx ? a.nx - 1 : xs);
            return line_row0 + sgn * static_cast<int64_t>(xs);
        };
        auto stage = [&](int s, LineStage<B, T, FUSE>& g) {
            const int sc = s < a.nsteps ? s : a.nsteps - 1;
            const int64_t row = line_ok ? row_at(sc) : 0;
            const int64_t rowc_b = row * (B * 8);
            const int64_t ey = ext_y ? (row - sgn * static_cast<int64_t>(a.nx)) * (B * 8) : 0;
            const int64_t ez = ext_z ? (row - sgn * static_cast<int64_t>(nxy)) * (B * 8) : 0;
            line_stage_load<B, T, FUSE>(a, c0 + sc, lane_off, rowc_b, ey, ez, g);
        };
        LineStage<B, T, FUSE> ring[NR];
#pragma unroll
        for (int i = 0; i < NR - 1; ++i) stage(i, ring[i]);
        double cur = 0.0;                   // this lane's output of the previous step
        xch[1][lane] = 0.0;
        for (int s0 = 0; s0 < a.nsteps; s0 += NR) {
#pragma unroll
            for (int p = 0; p < NR; ++p) {
                const int s = s0 + p;
                LineStage<B, T, FUSE>& g = ring[p];
                // every lane takes delivery of the stage (see tile_compute)
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int c = 0; c < B; ++c) asm volatile("" ::"v"(g.f[k][c]));
                const int xs = s - yl - zl;
                const bool act = line_ok && s < a.nsteps && xs >= 0 && xs < a.nx;
                // neighbours in earlier blocks: polled until published
                double ev[2 * B];
#pragma unroll
                for (int c = 0; c < B; ++c) {
                    ev[c] = g.ext[0][c];
                    ev[B + c] = g.ext[1][c];
                }
                {
                    const int64_t row = line_ok ? row_at(s < a.nsteps ? s : a.nsteps - 1) : 0;
                    const int code_y = act && ext_y ? static_cast<int>((row - sgn * static_cast<int64_t>(a.nx)) * (B * 8)) : -1;
                    const int code_z = act && ext_z ? static_cast<int>((row - sgn * static_cast<int64_t>(nxy)) * (B * 8)) : -1;
                    const int codes[2] = {code_y, code_z};
                    ColMap<false> cm;
                    cm.R = 1;
                    cm.j8 = 0;
#ifdef BILU_TRACE
                    long long* trc = (a.trace && s < a.nsteps) ? a.trace + 4 * (static_cast<int64_t>(c0) + s) : nullptr;
                    if (trc && lane == 0) trc[1] = wall_clock64();
                    const unsigned int sp_ = await_tile<2, B, false>(ev, codes, a.out, cm, a.spin_limit, a.status);
                    if (trc && lane == 0) { trc[2] = wall_clock64(); trc[3] = sp_; }
#else
                    await_tile<2, B, false>(ev, codes, a.out, cm, a.spin_limit, a.status);
#endif
                }
                // values of the last step: this line (x~), the line before
                // along y~ and along z~ inside the block
                const double* xb = xch[(s + 1) & 1];
                double nv[3][B];
                const int qy = qc - 1, qz = qc - a.WY;
#pragma unroll
                for (int c = 0; c < B; ++c) {
                    nv[0][c] = xb[qc * B + c];
                    nv[1][c] = xb[(qy >= 0 ? qy : 0) * B + c];
                    nv[2][c] = xb[(qz >= 0 ? qz : 0) * B + c];
                }
#pragma unroll
                for (int c = 0; c < B; ++c) {
                    if (yl == 0) nv[1][c] = ext_y ? ev[c] : 0.0;
                    if (zl == 0) nv[2][c] = ext_z ? ev[B + c] : 0.0;
                    if (xs <= 0) nv[0][c] = 0.0;
                }
                double acc;
                if (FUSE) {
                    acc = 0.0;
#pragma unroll
                    for (int c = 0; c < B; ++c) acc += widen(g.d[c]) * g.h[c];
                } else {
                    acc = g.h[0];
                }
                // slots in ascending column order: L (forward) z~, y~, x~;
                // U' (backward, D^{-1} fused) x~, y~, z~
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    constexpr int kDimL[3] = {2, 1, 0}, kDimU[3] = {0, 1, 2};
                    const int d = FUSE ? kDimU[k] : kDimL[k];
#pragma unroll
                    for (int c = 0; c < B; ++c) acc -= widen(g.f[k][c]) * nv[d][c];
                }
                const double v = publishable(acc);
                cur = act ? v : 0.0;
                if (act) {
                    const int64_t o = row_at(s) * B + r;
                    if (a.reset) a.reset[o] = not_ready();
                    coherent_store(a.out + o, v);
                }
                xch[s & 1][lane] = cur;
                // one wavefront: its LDS accesses complete in issue order
                __builtin_amdgcn_wave_barrier();
                asm volatile("" ::: "memory");
#ifdef BILU_TRACE
                if (a.trace && s < a.nsteps && lane == 0) a.trace[4 * (static_cast<int64_t>(c0) + s)] = wall_clock64();
#endif
                // the next stage is requested only now, so a poll above
                // never waits behind it (vector loads complete in order)
                stage(s + NR - 1, ring[(p + NR - 1) % NR]);
            }
        }
    }
    finish_persistent(a.ticket, a.done, a.total_waves);
}

// ---------------------------------------------------------------------------
// U' sweep fused with y = A x on its output x: one persistent launch whose
// tickets are the sweep's tiles and then the blocks of 64/B rows of A,
// ordered by the tile that finishes the lowest row each reads (host-built
// order, so every item depends only on earlier tickets, and every tile has
// a wavefront before any wavefront waits in an SpMV block).  An SpMV block
// requests A's values and the x values (device-coherent) of a group of
// blocks of a row together, polls any x value still showing kNotReady, then
// forms its rows exactly as k_spmv does (same operations, same order).
// ---------------------------------------------------------------------------
struct FusedSpmvArgs {
    const int32_t* sched;        // >= 0 tile, < 0 SpMV block -(1 + b)
    int nsched;
    int nb;
    const int32_t* Ap;
    const int32_t* Aj;
    const double* Ax;
    double* y;
};

template <int B>
__device__ __forceinline__ void spmv_block_ready(const FusedSpmvArgs& m, int64_t row0, const double* x,
                                                 unsigned int limit, int* status)
{
    constexpr int RPC = 64 / B;
    constexpr int BB = B * B;
    constexpr int EG = B <= 4 ? 8 : 4;          // blocks of a row read together
    const int lane = lane_id();
    const int q = lane / B;
    const int r = lane - q * B;
    const int64_t row = row0 + q;
    if (q >= RPC || row >= m.nb) return;
    const int e0 = m.Ap[row], e1 = m.Ap[row + 1];
    double acc = 0.0;
    for (int g = e0; g < e1; g += EG) {
        int j[EG];
#pragma unroll
        for (int k = 0; k < EG; ++k) j[k] = g + k < e1 ? m.Aj[g + k] : -1;
        // A's values and x's values requested together (the x values with
        // device-coherent loads: cached copies would be stale)
        double av[EG * B], xv[EG * B];
#pragma unroll
        for (int k = 0; k < EG; ++k)
#pragma unroll
            for (int c = 0; c < B; ++c) {
                const int64_t blk = g + k;
                av[k * B + c] = j[k] >= 0 ? m.Ax[blk * BB + c * B + r] : 0.0;
                xv[k * B + c] = j[k] >= 0 ? coherent_load(x + static_cast<int64_t>(j[k]) * B + c) : 0.0;
            }
        await_rows<EG, B, 1>(xv, j, x, 1, 0, limit, status);
#pragma unroll
        for (int k = 0; k < EG; ++k) {
            if (j[k] < 0) continue;
#pragma unroll
            for (int c = 0; c < B; ++c) acc += av[k * B + c] * xv[k * B + c];
        }
    }
    m.y[row * B + r] = acc;
}

template <int B, typename T, int KMAX>
__global__ __launch_bounds__(64) void k_sweep_tiled_spmv(TiledArgs a, FusedSpmvArgs m)
{
    extern __shared__ double tile_vals[];                    // [tile rows + 1][B]
    if (gated_off(a.gate)) return;
    if (lane_id() < B) tile_vals[a.tile_rows * B + lane_id()] = 0.0;
    for (int tk = __builtin_amdgcn_readfirstlane(grab_ticket(a.ticket)); tk < m.nsched;
         tk = __builtin_amdgcn_readfirstlane(grab_ticket(a.ticket))) {
        const int it = uniform_load(m.sched, tk);
        if (it >= 0) {
            ColMap<false> cm;
            cm.R = 1;
            cm.j8 = 0;
            run_tile<B, T, true, KMAX, false, false>(a, it, cm, tile_vals, tile_vals, nullptr, 0);
        } else {
            spmv_block_ready<B>(m, static_cast<int64_t>(-1 - it) * (64 / B), a.out, a.spin_limit, a.status);
        }
    }
    finish_persistent(a.ticket, a.done, a.total_waves);
}

// Rows [row0, row0 + 64/B) of y = A x (or A^T x through the transposed
// structure), by one wavefront; lane (q, r) owns component r of row q.
// Block values are read from Av at block (e - ebase): A itself (ebase 0), or
// the wavefront's LDS copy of its rows' blocks (ebase the first of them).
template <int B, int RT, bool TRANS>
__device__ __forceinline__ void spmv_rows(int64_t row0, int nb, const int32_t* __restrict__ rp,
                                          const int32_t* __restrict__ cj, const int64_t* __restrict__ srcpos,
                                          const double* __restrict__ Av, int64_t ebase,
                                          const double* __restrict__ x, double* __restrict__ y, int R)
{
    constexpr int RPC = 64 / B;
    constexpr int BB = B * B;
    const int lane = lane_id();
    const int q = lane / B;
    const int r = lane - q * B;
    const int64_t row = row0 + q;
    if (q >= RPC || row >= nb) return;
    const int e0 = rp[row], e1 = rp[row + 1];
    for (int c0 = 0; c0 < R; c0 += RT) {
        double acc[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[t] = 0.0;
        // unrolled: the column-index and x loads of several blocks in flight
        // (same accumulation order)
#pragma unroll 4
        for (int e = e0; e < e1; ++e) {
            const int j = cj[e];
            const int64_t blk = (TRANS ? srcpos[e] : e) - ebase;
#pragma unroll
            for (int c = 0; c < B; ++c) {
                const double v = TRANS ? Av[blk * BB + r * B + c] : Av[blk * BB + c * B + r];
                const double* xj = x + (static_cast<int64_t>(j) * B + c) * R + c0;
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    if (RT == 1 || c0 + t < R) acc[t] += v * xj[t];
            }
        }
        double* dst = y + (row * B + r) * R + c0;
#pragma unroll
        for (int t = 0; t < RT; ++t)
            if (RT == 1 || c0 + t < R) dst[t] = acc[t];
    }
}

// LDS per wavefront for its rows' blocks in k_spmv when each block serves a
// tile of right-hand sides (RT > 1): eight blocks per row on average (a
// 7-point stencil needs seven); 0 for block sizes whose rows already read
// whole cache lines.  With one right-hand side the copy did not pay (156 ->
// 159 us on 60x220x85, b = 3); with 8 and 32 it did (64^3 ILU(1) solves
// 162 -> 172 and 219 -> 233 per second).
template <int B>
struct SpmvStage {
    static constexpr int doubles = B <= 3 ? (64 / B) * 8 * B * B : 0;
};

template <int B, int RT, bool TRANS>
__global__ __launch_bounds__(kThreads) void k_spmv(int nb, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ cj,
                                                   const int64_t* __restrict__ srcpos,
                                                   const double* __restrict__ Ax,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y, int R, const int* gate, int stream_a)
{
    constexpr int RPC = 64 / B;
    constexpr int BB = B * B;
    constexpr int STAGE = TRANS || RT == 1 ? 0 : SpmvStage<B>::doubles;
    if (gated_off(gate)) return;
    // stream_a: workgroup b runs on XCD b % 8 (the grid is a multiple of 8),
    // so each XCD takes a contiguous eighth of the rows and its L2 keeps the
    // x entries its rows share
    const int64_t lb = stream_a ? static_cast<int64_t>(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8
                                : static_cast<int64_t>(blockIdx.x);
    const int64_t wave_global = lb * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t row0 = wave_global * RPC;
    if constexpr (STAGE > 0) {
        // The wavefront's rows own one contiguous run of blocks: copied to
        // LDS with whole-wavefront loads, then read as from A (same values,
        // same accumulation order).
        __shared__ double stage[kWavesPerBlock][STAGE];
        if (row0 < nb) {
            const int64_t rend = row0 + RPC < nb ? row0 + RPC : nb;
            const int32_t E0 = uniform_load(rp, row0);
            const int64_t n = static_cast<int64_t>(uniform_load(rp, rend) - E0) * BB;
            if (n <= STAGE) {
                constexpr int PER = (STAGE + 63) / 64;
                double* st = stage[threadIdx.x >> 6];
                const double* src = Ax + static_cast<int64_t>(E0) * BB;
                const int lane = lane_id();
                double v[PER];
#pragma unroll
                for (int k = 0; k < PER; ++k) v[k] = lane + 64 * k < n ? src[lane + 64 * k] : 0.0;
#pragma unroll
                for (int k = 0; k < PER; ++k)
                    if (lane + 64 * k < n) st[lane + 64 * k] = v[k];
                // one wavefront: its LDS accesses complete in issue order
                __builtin_amdgcn_wave_barrier();
                asm volatile("" ::: "memory");
                spmv_rows<B, RT, TRANS>(row0, nb, rp, cj, srcpos, st, E0, x, y, R);
                return;
            }
        }
    }
    if constexpr (!TRANS && RT == 1 && SpmvStage<B>::doubles > 0) {
        if (stream_a) {
            // One right-hand side on a large matrix: the wavefront's run of
            // A is copied to LDS (dynamic) with whole-wavefront nontemporal
            // loads, so every line of A is fetched once and does not evict
            // x from L2, then read from there in the same order.
            extern __shared__ double dyn_stage[];
            constexpr int ST = SpmvStage<B>::doubles;
            if (row0 < nb) {
                const int64_t rend = row0 + RPC < nb ? row0 + RPC : nb;
                const int32_t E0 = uniform_load(rp, row0);
                const int64_t n = static_cast<int64_t>(uniform_load(rp, rend) - E0) * BB;
                if (n <= ST) {
                    constexpr int PER = (ST + 63) / 64;
                    double* st = dyn_stage + (threadIdx.x >> 6) * ST;
                    const double* src = Ax + static_cast<int64_t>(E0) * BB;
                    const int lane = lane_id();
                    double v[PER];
#pragma unroll
                    for (int k = 0; k < PER; ++k)
                        v[k] = lane + 64 * k < n ? __builtin_nontemporal_load(src + lane + 64 * k) : 0.0;
#pragma unroll
                    for (int k = 0; k < PER; ++k)
                        if (lane + 64 * k < n) st[lane + 64 * k] = v[k];
                    __builtin_amdgcn_wave_barrier();
                    asm volatile("" ::: "memory");
                    spmv_rows<B, RT, TRANS>(row0, nb, rp, cj, srcpos, st, E0, x, y, R);
                    return;
                }
            }
        }
    }
    spmv_rows<B, RT, TRANS>(row0, nb, rp, cj, srcpos, Ax, 0, x, y, R);
}

// y = A x (or A^T x) for R >= 2 right-hand sides, lanes over columns: lane
// (s, j) of a wavefront computes column j of block row row0 + s, all B
// components of it in registers, with CW >= R lanes per row (a power of
// two) and 64/CW rows per wavefront.  A block's values are read by all CW
// lanes of its row at once (one cache line per row and load), and the x
// values of a block column (B unknowns, R columns each, row-major) by the
// row's lanes together, contiguous.  Per column, the products are summed in
// the order of spmv_rows (blocks in order, components in order), so each
// column equals the one-column result bit for bit.
template <int B, int CW, bool TRANS>
__global__ __launch_bounds__(kThreads) void k_spmv_cols(int nb, const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ cj,
                                                        const int64_t* __restrict__ srcpos,
                                                        const double* __restrict__ Ax,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ y, int R, const int* gate)
{
    constexpr int RPW = 64 / CW;
    constexpr int BB = B * B;
    if (gated_off(gate)) return;
    const int lane = lane_id();
    const int s = lane / CW;
    const int j = lane - s * CW;
    const int64_t wave = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t row = wave * RPW + s;
    if (row >= nb || j >= R) return;
    const int e0 = rp[row], e1 = rp[row + 1];
    double acc[B];
#pragma unroll
    for (int r = 0; r < B; ++r) acc[r] = 0.0;
#pragma unroll 2
    for (int e = e0; e < e1; ++e) {
        const int64_t col = cj[e];
        const double* av = Ax + (TRANS ? srcpos[e] : static_cast<int64_t>(e)) * BB;
        const double* xj = x + col * B * R + j;
        double xv[B];
#pragma unroll
        for (int c = 0; c < B; ++c) xv[c] = xj[c * R];
#pragma unroll
        for (int c = 0; c < B; ++c)
#pragma unroll
            for (int r = 0; r < B; ++r) acc[r] += (TRANS ? av[r * B + c] : av[c * B + r]) * xv[c];
    }
    double* dst = y + row * B * R + j;
#pragma unroll
    for (int r = 0; r < B; ++r) dst[r * R] = acc[r];
}

// ---------------------------------------------------------------------------
// Sweeps over the batch: one persistent launch per sweep on the members''
// row-tile layouts.  Items are (member, tile), merged tile index by tile
// index (tile t of every member before tile t + 1 of any), so each item
// depends only on items with smaller tickets, as in the single-system tiled
// sweep.  Members whose Krylov recurrence is frozen are skipped by both
// sweeps of an application alike, which keeps the kNotReady invariant of
// their buffers.
// ---------------------------------------------------------------------------
struct BatchTiled {               // one member's tiled layout of one sweep
    const int32_t* tile_chunk_ptr;
    const int32_t* tile_lo;
    const int32_t* chunk_row;
    const int32_t* rows;
    const int32_t* deps;
    const void* vals;
    const void* dinv;
    int64_t voff;                 // first unknown of the member in the batch vectors
    int tile_rows;
    int kmax;
    int bs;
    int pad;
};

struct BatchSweepArgs {
    const BatchTiled* mem;        // per member, this sweep
    const int2* items;            // (member, tile)
    int nitems;
    const double* rhs;
    double* out;
    double* reset;
    const int* active;            // per member, or null: every member
    const int* gate;              // nothing runs when given and *gate == 0
    unsigned long long* ticket;
    unsigned int* done;
    int* status;
    unsigned int total_waves;
    unsigned int spin_limit;
};

template <int B, typename T, bool FUSE, int KMAX>
__device__ __forceinline__ void batch_tile(const BatchSweepArgs& a, const BatchTiled& M, int tile, double* tile_vals)
{
    TiledArgs t{};
    t.tile_chunk_ptr = M.tile_chunk_ptr;
    t.tile_lo = M.tile_lo;
    t.chunk_row = M.chunk_row;
    t.rows = M.rows;
    t.deps = M.deps;
    t.vals = M.vals;
    t.dinv = M.dinv;
    t.rhs = a.rhs + M.voff;
    t.out = a.out + M.voff;
    t.reset = a.reset ? a.reset + M.voff : nullptr;
    t.status = a.status;
    t.tile_rows = M.tile_rows;
    t.ring = 0;                      // member layouts keep whole tiles
    t.R = 1;
    t.spin_limit = a.spin_limit;
    // this member's zero row (an earlier item may have used that LDS)
    if (lane_id() < B) tile_vals[M.tile_rows * B + lane_id()] = 0.0;
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
    ColMap<false> cm;
    cm.R = 1;
    cm.j8 = 0;
    run_tile<B, T, FUSE, KMAX, false, false>(t, tile, cm, tile_vals, tile_vals, nullptr, 0);
}

template <typename T, bool FUSE>
__global__ __launch_bounds__(64) void k_sweep_batch(BatchSweepArgs a)
{
    extern __shared__ double tile_vals[];
    // the gate is uniform over the grid: either every wavefront leaves here
    // (the ticket and done counters stay untouched) or none does
    if (gated_off(a.gate)) return;
    for (int tk = __builtin_amdgcn_readfirstlane(grab_ticket(a.ticket)); tk < a.nitems;
         tk = __builtin_amdgcn_readfirstlane(grab_ticket(a.ticket))) {
        const int2 it = uniform_record(a.items, tk);
        if (a.active && !uniform_load(a.active, it.x)) continue;
        const BatchTiled M = uniform_record(a.mem, it.x);
        switch (M.bs * 16 + M.kmax) {
#define BILU_BATCH_TILE(BS, K) \
    case BS * 16 + K: batch_tile<BS, T, FUSE, K>(a, M, it.y, tile_vals); break;
        BILU_BATCH_TILE(1, 3) BILU_BATCH_TILE(2, 3) BILU_BATCH_TILE(3, 3) BILU_BATCH_TILE(4, 3)
        BILU_BATCH_TILE(5, 3) BILU_BATCH_TILE(6, 3) BILU_BATCH_TILE(7, 3) BILU_BATCH_TILE(8, 3)
        BILU_BATCH_TILE(1, 6) BILU_BATCH_TILE(2, 6) BILU_BATCH_TILE(3, 6) BILU_BATCH_TILE(4, 6)
        BILU_BATCH_TILE(1, 9) BILU_BATCH_TILE(2, 9) BILU_BATCH_TILE(3, 9) BILU_BATCH_TILE(4, 9)
#undef BILU_BATCH_TILE
        default: break;
        }
    }
    finish_persistent(a.ticket, a.done, a.total_waves);
}

}  // namespace dev
}  // namespace bilu
