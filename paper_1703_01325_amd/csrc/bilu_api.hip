// C ABI of the block ILU(k) library: context, device storage, launches and
// the Krylov drivers.  See include/bilu.h for the contract of each call.
#include <hip/hip_runtime.h>
#include <mutex>
#include <cstdio>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "bilu.h"
#include "bilu_internal.h"
#include "kernels.h"
#include "kernels_batch.h"
#include "launch.h"

using namespace bilu;
using dev::KState;
using dev::SweepArgs;
using dev::TiledArgs;

#ifdef BILU_TRACE
#define CK(call)                                                                                   \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
            return BILU_ERR_HIP;                                                                   \
        }                                                                                          \
    } while (0)
#else
#define CK(call)                                       \
    do {                                               \
        if ((call) != hipSuccess) return BILU_ERR_HIP; \
    } while (0)
#endif

namespace {
constexpr int kFormLevel = 0;   // level-chunk layout (sweep modes 0 and 1)
constexpr int kFormTiled = 1;   // tiled layout (sweep mode 2)
constexpr int kFormLines = 2;   // line-sweep layout of L and U' (BILU_TUNE_LINE_SWEEP)
constexpr int kForms = 3;
constexpr int kMaxTileDoubles = 8192;   // LDS of one tiled wavefront: 64 KiB
}  // namespace

// Scratch of bilu_apply_noalloc, one copy per device for the life of the
// process: bytes [0, 8) ticket, [8, 12) done count and [12, 16) status of the
// persistent sweeps, from byte kScratchHeader the intermediate vector y of
// the application.  Host code uses the address hipGetSymbolAddress gives for
// the current device, never the symbol itself.
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr size_t kScratchHeader = 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_addr[kScratchDevices] = {};

// Device address of the scratch on `device` (the current device), looked up
// once per device.
bilu_status scratch_of_device(int device, unsigned char** out)
{
    if (device < 0 || device >= kScratchDevices) return BILU_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BILU_ERR_HIP;
        g_scratch_addr[device] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_addr[device];
    return BILU_OK;
}
}  // namespace

struct bilu_ctx {
    Host h;
    int device = -1;
    int num_cu = 0;
    bool dev_ready = false;
    bool factored = false;
    bool split_done = false;
    mutable bool f_ready = false; // d_F holds the split factors of the current factorisation
    int precision = BILU_FACTORS_FP64;
    int sweep_mode = 2;
    int tile_rows = 0;          // rows per tile of the tiled layouts (0: not chosen yet)
    int tile_group = 1;         // tiles per workgroup of the tiled layouts
    int tile_rows_req = 0;      // requested rows per tile (0: by schedule simulation)
    int tile_group_req = 0;     // requested tiles per group (0: by schedule simulation)
    int tile_block = 0;         // line-block tiles: ny + 256*nz (0: row-range tiles)
    int64_t lds_max = 65536;    // LDS bytes a workgroup may use (the device's, once known)
    int64_t layout_lds = 0;     // lds_max the tiled layouts were chosen for
    int blocks_override = 0;
    int rhs_tile = 0;           // columns per pass for several right-hand sides; 0: 8
    bool fuse_spmv = false;     // solvers run U' sweep + SpMV as one launch
    int helper = 0;             // helper wavefronts: 0 automatic, 1 always, 2 never
    dev::OmState* d_om = nullptr; // ORTHOMIN(k) state
    // point-granularity view (bilu_apply_point): the split factors expanded
    // to point rows and swept by a context of block size 1 whose values are
    // set, not factored (values_only: no factorisation plan)
    bool values_only = false;
    bilu_ctx* point = nullptr;
    int64_t* d_point_src = nullptr;   // per point entry: index into F, -1 the unit diagonal
    double* d_point_y = nullptr;      // D^{-1} y between the two point sweeps
    int64_t point_n = 0;              // point entries
    unsigned long factor_gen = 0;     // bumped by every bilu_factor_diag
    unsigned long point_gen = 0;      // factor_gen the point values were expanded from (0: none)
    unsigned int spin_limit = 1u << 24;

    int32_t *d_Ap = nullptr, *d_Aj = nullptr, *d_Arow = nullptr;
    int32_t *d_Pp = nullptr, *d_Pj = nullptr, *d_Prow = nullptr, *d_Pdiag = nullptr, *d_PtoA = nullptr;
    int32_t* d_Lrows = nullptr;
    // factorisation with rows in LDS: update lists and per L level the LDS
    // bytes of its largest row (0: that level takes k_factor_rows)
    int32_t *d_upd_ptr = nullptr, *d_upd_f = nullptr, *d_upd_g = nullptr;
    // per row of the L levels, in level order: {row, first entry, entries,
    // pivots, first update pair, update pairs, 0, 0}
    int32_t* d_frec = nullptr;
    std::vector<int32_t> fac_lds;
    // the whole factorisation in one persistent launch (k_factor_waves):
    // LDS bytes per wavefront (0: some row does not fit, one launch per
    // level instead), ticket and expired-wait words
    int fwave_lds = 0;
    int fwave_n = 16;                     // wavefronts (rows) per workgroup and ticket
    unsigned int* d_fticket = nullptr;
    int factor_mode = 0;                  // BILU_TUNE_FACTOR
    int spmv_stream = 0;                  // BILU_TUNE_SPMV_STREAM
    int rhs_pairs = 0;                    // BILU_TUNE_RHS_PAIRS
    int32_t *d_ATp = nullptr, *d_ATj = nullptr;
    int64_t* d_ATsrc = nullptr;
    double *d_P = nullptr, *d_F = nullptr, *d_Dinv = nullptr;
    DevSweep ds[kForms][4];     // [form][sweep]
    bool form_uploaded[kForms] = {false, false, false};
    int line_block = 0;         // line sweep of L and U' with blocks ny + 256*nz (0: off)
    bool layouts_checked = false;   // validate_layout passed on the layouts as built

    double* d_y = nullptr;      // intermediate of an application, kept at kNotReady
    size_t y_cap = 0;
    double* d_y2 = nullptr;     // D^{-1} y when the U' sweep runs unfused
    size_t y2_cap = 0;
    int split_dinv = 0;         // BILU_TUNE_SPLIT_DINV
    int* d_bad = nullptr;
    int* d_status = nullptr;
    unsigned int* d_done = nullptr;
    unsigned long long* d_ticket = nullptr;

    double* d_kv = nullptr;
    size_t kv_cap = 0;
    double* d_part = nullptr;
    double* d_gmh = nullptr;    // GMRES Hessenberg matrix, coefficient and y
    size_t gm_cap = 0;
    KState* d_state = nullptr;
    KState* h_state = nullptr;  // pinned host copy of the Krylov state, read at the end of a solve
    int* h_flags = nullptr;     // mapped pinned host flags written by the decide kernel (2 slots)
    int* d_flags = nullptr;     // their device address
    hipEvent_t step_ev[2] = {nullptr, nullptr};

    // HIP-event timing of kernel classes (bilu_timing)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> ev_marks;   // (class, index of start event)

    std::vector<void*> allocs;
};

namespace {

// Records the start event of a timed region; returns its slot or -1.
long timing_begin(bilu_ctx* c, int cls, hipStream_t s)
{
    if (!c->timing) return -1;
    if (c->ev_used + 2 > c->ev_pool.size()) {
        for (int k = 0; k < 64; ++k) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            c->ev_pool.push_back(e);
        }
    }
    const size_t i = c->ev_used;
    c->ev_used += 2;
    if (hipEventRecord(c->ev_pool[i], s) != hipSuccess) return -1;
    c->ev_marks.emplace_back(cls, i);
    return static_cast<long>(i);
}

void timing_end(bilu_ctx* c, long slot, hipStream_t s)
{
    if (slot < 0) return;
    (void)hipEventRecord(c->ev_pool[static_cast<size_t>(slot) + 1], s);
}

// Device allocations are owned by a context or a batch (anything with an
// `allocs` list) and freed with it.
template <typename O, typename T>
bilu_status dalloc(O* c, T** p, size_t count)
{
    void* q = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) return BILU_ERR_ALLOC;
    c->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return BILU_OK;
}

template <typename O>
void dfree(O* c, void* p)
{
    if (!p) return;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it != c->allocs.end()) {
        (void)hipFree(p);
        c->allocs.erase(it);
    }
}

template <typename O, typename T>
bilu_status upload(O* c, T** d, const std::vector<T>& h)
{
    bilu_status st = dalloc(c, d, h.size());
    if (st != BILU_OK) return st;
    if (!h.empty() && hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return BILU_ERR_HIP;
    return BILU_OK;
}

int grid_for(int64_t work, int threads = 256, int cap = 65536)
{
    int64_t g = (work + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<int>(g);
}

bool fused_sweep(int w) { return w == BILU_SWEEP_U || w == BILU_SWEEP_LT; }

// Right-hand-side columns per pass of the level-chunk sweeps and the SpMV.
int rhs_tile(const bilu_ctx* c, int R)
{
    if (R == 1) return 1;
    return c->rhs_tile > 0 ? c->rhs_tile : 8;
}
// The SpMV's columns per pass: by default (rhs_tile 0) one pass with lanes
// over all columns (0); an explicit rhs_tile keeps the per-row kernel.
int spmv_tile(const bilu_ctx* c, int R)
{
    if (R == 1) return 1;
    return c->rhs_tile > 0 ? c->rhs_tile : 0;
}

// Whether A x with R columns stages A through LDS with nontemporal loads in
// XCD-contiguous row ranges (BILU_TUNE_SPMV_STREAM; automatic: one column,
// b <= 3, at least 2^19 block rows -- measured on MI355X: 60x220x85, b = 3,
// 155-159 -> 145 us with 29% fewer fetched bytes; 64^3, b = 3, 32 -> 39 us,
// where the lower occupancy of the staged kernel costs more than it saves).
bool spmv_streams_a(const bilu_ctx* c, int R)
{
    if (R != 1 || c->h.bs > 3 || c->spmv_stream == 2) return false;
    return c->spmv_stream == 1 || c->h.nb >= (1 << 19);
}

bool transposed_sweep(int w) { return w == BILU_SWEEP_UT || w == BILU_SWEEP_LT; }

// Helper wavefronts for a tiled sweep of R columns.  Automatic: for single
// tiles whose rows load six or more dependency slots ahead (ILU(1) and
// beyond on a 7-point grid), where the member's deeper prefetch ring pays:
// measured on MI355X, 64^3 ILU(1) L/U' sweeps 682/707 -> 517/532 us and
// 60x220x85 ILU(1) U' 1587 -> 1491 us, while ILU(0) tiles (three slots,
// already a three-state ring) and tile groups ran slower with helpers
// (60x220x85 ILU(0), groups of 3: 483/499 -> 505/550 us).
bool use_helper(const bilu_ctx* c, const HostTiled& ht, int R)
{
    if (R != 1 || c->helper == 2 || ht.group > kHelpGroupMax) return false;
    if (c->helper == 1) return true;
    return ht.group == 1 && ht.kmax >= 6;
}

// Several right-hand sides on single tiles run two columns per wavefront
// (k_sweep_tiled_pairs) where R is even, the doubled LDS fits and the
// register ring of the pair walk fits without spilling (b <= 5 and at most
// 18 dependency values per lane in registers: gfx950 ISA of the build);
// automatically from 16 columns up (BILU_TUNE_RHS_PAIRS).  Measured on
// MI355X, 64^3 ILU(1): 32 columns, L / U' sweeps 2900 / 2994 -> 2059 / 2095
// us; 8 columns, 969 / 997 -> 1087 / 1086 us (half as many wavefronts on a
// front that is already short of them).
bool use_pairs(const bilu_ctx* c, const HostTiled& ht, int R, size_t lds)
{
    if (c->rhs_pairs == 1 || R < 2 || R % 2 != 0 || (c->rhs_pairs == 0 && R < 16)) return false;
    return ht.group == 1 && c->h.bs <= 5 && ht.kmax * c->h.bs <= 18 && static_cast<int64_t>(2 * lds) <= c->lds_max;
}

// ----- templated launch helpers ---------------------------------------------
#define BILU_SWITCH_B(bs, CALL)     \
    switch (bs) {                   \
    case 1: { constexpr int B = 1; CALL; return true; } \
    case 2: { constexpr int B = 2; CALL; return true; } \
    case 3: { constexpr int B = 3; CALL; return true; } \
    case 4: { constexpr int B = 4; CALL; return true; } \
    case 5: { constexpr int B = 5; CALL; return true; } \
    case 6: { constexpr int B = 6; CALL; return true; } \
    case 7: { constexpr int B = 7; CALL; return true; } \
    case 8: { constexpr int B = 8; CALL; return true; } \
    }                               \
    return false;

// rt: right-hand-side columns per pass (1, 4 or 8)
bool launch_sweep(int bs, int prec, int rt, int blocks, hipStream_t s, const SweepArgs& a)
{
    BILU_SWITCH_B(bs, if (!launch::sweep<B>(prec, rt, blocks, s, a)) return false)
}

// One wavefront per tile (a.group == 1) or per member tile of a group.
bool launch_tiled(int bs, int kmax, int prec, bool fuse, bool multi, int blocks, size_t lds, hipStream_t s,
                  const TiledArgs& a)
{
    BILU_SWITCH_B(bs, if (!launch::tiled<B>(kmax, prec, fuse, multi, blocks, lds, s, a)) return false)
}

bool launch_pairs(int bs, int kmax, int prec, bool fuse, int blocks, size_t lds, hipStream_t s, const TiledArgs& a)
{
    BILU_SWITCH_B(bs, if (!launch::pairs<B>(kmax, prec, fuse, blocks, lds, s, a)) return false)
}

bool launch_helped(int bs, int kmax, int prec, bool fuse, int blocks, size_t lds, hipStream_t s, const TiledArgs& a)
{
    BILU_SWITCH_B(bs, if (!launch::helped<B>(kmax, prec, fuse, blocks, lds, s, a)) return false)
}

bool launch_lines(int bs, int prec, bool fuse, int blocks, hipStream_t s, const dev::LineArgs& a)
{
    BILU_SWITCH_B(bs, if (!launch::lines<B>(prec, fuse, blocks, s, a)) return false)
}

bool launch_fused(int bs, int kmax, int prec, int blocks, size_t lds, hipStream_t s, const TiledArgs& a,
                  const dev::FusedSpmvArgs& m)
{
    BILU_SWITCH_B(bs, if (!launch::fused<B>(kmax, prec, blocks, lds, s, a, m)) return false)
}

bool launch_spmv(int bs, int rt, bool tr, int nb, const int32_t* rp, const int32_t* cj, const int64_t* src,
                 const double* Ax, const double* x, double* y, int R, hipStream_t s, const int* gate = nullptr,
                 bool stream_a = false)
{
    if (bs > kMaxKernelBs) {
        if (R != 1) return false;
        hipLaunchKernelGGL(dev::k_spmv_gen, dim3(grid_for(static_cast<int64_t>(nb) * bs)), dim3(256), 0, s, nb, bs,
                           rp, cj, tr ? src : nullptr, Ax, x, y, gate);
        return true;
    }
    BILU_SWITCH_B(bs, if (!launch::spmv<B>(rt, tr, nb, rp, cj, src, Ax, x, y, R, s, gate, stream_a)) return false)
}

// Rows [first, first + nrows) of the L level order.
bool launch_factor(int bs, int64_t first, int nrows, int lds, bilu_ctx* c, hipStream_t s)
{
    const int32_t* rows = c->d_Lrows + first;
    if (lds > 0) {
        const int4* rec = reinterpret_cast<const int4*>(c->d_frec + 8 * first);
        BILU_SWITCH_B(bs, hipLaunchKernelGGL((dev::k_factor_rows_lds<B>), dim3(nrows), dim3(64), lds, s, rec, nrows,
                                             c->d_Pj, c->d_upd_ptr, c->d_upd_f, c->d_upd_g, c->d_P, c->d_Dinv,
                                             c->d_bad))
    }
    if (bs > kMaxKernelBs) {
        const size_t glds = (3 * static_cast<size_t>(bs) * bs + bs) * sizeof(double);
        hipLaunchKernelGGL(dev::k_factor_rows_gen, dim3(nrows), dim3(256), glds, s, bs, rows, nrows, c->d_Pp,
                           c->d_Pj, c->d_Pdiag, c->d_upd_ptr, c->d_upd_f, c->d_upd_g, c->d_P, c->d_Dinv, c->d_bad);
        return true;
    }
    BILU_SWITCH_B(bs, hipLaunchKernelGGL((dev::k_factor_rows<B>), dim3(nrows), dim3(64), 0, s, rows, nrows,
                                         c->d_Pp, c->d_Pj, c->d_Pdiag, c->d_upd_ptr, c->d_upd_f, c->d_upd_g, c->d_P,
                                         c->d_Dinv, c->d_bad))
}

// Backfill with a compile-time block size (false: no kernel for bs).
bool launch_backfill(int bs, int64_t nP, const int32_t* PtoA, const double* Ax, double* P, hipStream_t s)
{
    BILU_SWITCH_B(bs, hipLaunchKernelGGL((dev::k_backfill_b<B>), dim3(grid_for(nP * B * B)), dim3(256), 0, s, nP,
                                         PtoA, Ax, P))
}

// Update lists of Algorithm 4 for k_factor_rows_lds and k_factor_rows: for each pivot entry
// e = (i, p) of P (in entry order), the pairs (f, g) of entries (i, j), f > e,
// and (p, j), g > diagonal of p, with the same column (f as a block index in
// row i); and per L level the LDS bytes of its largest row.
bilu_status factor_plan(bilu_ctx* c)
{
    constexpr int kCap = 48 * 1024;            // LDS per workgroup for the row
    const Host& h = c->h;
    const int nb = h.nb;
    const int64_t nP = static_cast<int64_t>(h.Pj.size());
    const int64_t bb8 = static_cast<int64_t>(h.bs) * h.bs * 8;
    std::vector<int32_t> uptr(static_cast<size_t>(nP) + 1, 0), uf, ug;
    std::vector<int64_t> row_bytes(static_cast<size_t>(nb), 0);
    int64_t row_min = 0;      // largest LDS a row needs with one pivot's pairs at a time
    for (int32_t i = 0; i < nb; ++i) {
        const int32_t e0 = h.Pp[i], e1 = h.Pp[i + 1], d = h.Pdiag[i];
        for (int32_t e = e0; e < e1; ++e) {
            if (e < d) {
                const int32_t p = h.Pj[e];
                int32_t f = e + 1, g = h.Pdiag[p] + 1;
                const int32_t gEnd = h.Pp[p + 1];
                while (f < e1 && g < gEnd) {
                    if (h.Pj[f] == h.Pj[g]) {
                        uf.push_back(f - e0);
                        ug.push_back(g);
                        ++f;
                        ++g;
                    } else if (h.Pj[f] < h.Pj[g]) {
                        ++f;
                    } else {
                        ++g;
                    }
                }
                if (uf.size() > static_cast<size_t>(INT32_MAX)) return BILU_ERR_ALLOC;   // lists beyond int32 indices
            }
            uptr[e + 1] = static_cast<int32_t>(uf.size());
        }
        const int64_t nrow = e1 - e0, dk = d - e0, npair = uptr[d] - uptr[e0];
        const int64_t lists = ((2 * dk + 1 + 2 * npair) * 4 + 7) / 8 * 8;
        row_bytes[i] = (nrow + dk + npair) * bb8 + lists;
        int64_t maxpp = 0;
        for (int32_t e = e0; e < d; ++e) maxpp = std::max<int64_t>(maxpp, uptr[e + 1] - uptr[e]);
        row_min = std::max(row_min, (nrow + dk + maxpp) * bb8 + lists);
    }
    const HostSweep& L = h.sweep[BILU_SWEEP_L];
    c->fac_lds.assign(static_cast<size_t>(L.nlev), 0);
    std::vector<int32_t> rec(static_cast<size_t>(L.level_ptr[L.nlev]) * 8, 0);
    for (int l = 0; l < L.nlev; ++l) {
        int64_t m = 0;
        for (int32_t x = L.level_ptr[l]; x < L.level_ptr[l + 1]; ++x) {
            const int32_t i = L.level_rows[x];
            m = std::max(m, row_bytes[i]);
            const int32_t e0 = h.Pp[i], d = h.Pdiag[i];
            int32_t* q = &rec[static_cast<size_t>(x) * 8];
            q[0] = i;
            q[1] = e0;
            q[2] = h.Pp[i + 1] - e0;
            q[3] = d - e0;
            q[4] = uptr[e0];
            q[5] = uptr[d] - uptr[e0];
        }
        c->fac_lds[l] = m <= kCap && h.bs <= kMaxKernelBs ? static_cast<int32_t>(m) : 0;
    }
    // the persistent factorisation: as many wavefronts per workgroup (16, 8,
    // 4, 2 or 1) as fit 96 KiB of LDS with the largest row of the pattern; a
    // row larger than 96 KiB stages the A_pj blocks of its pivots a run of
    // pivots at a time, which takes one wavefront per workgroup and every
    // row's blocks, pivot inverses, lists and one pivot's A_pj within 96 KiB
    constexpr int64_t kWaveCap = 96 * 1024;
    int64_t mrow = 0;
    for (int32_t i = 0; i < nb; ++i) mrow = std::max(mrow, row_bytes[i]);
    mrow = std::min<int64_t>((mrow + 7) / 8 * 8, kWaveCap);
    c->fwave_n = 16;
    while (c->fwave_n > 1 && mrow * c->fwave_n > kWaveCap) c->fwave_n /= 2;
    c->fwave_lds = L.nlev > 0 && h.bs <= kMaxKernelBs && row_min <= kWaveCap ? static_cast<int>(mrow) : 0;
    bilu_status st;
    if ((st = upload(c, &c->d_upd_ptr, uptr)) || (st = upload(c, &c->d_upd_f, uf)) || (st = upload(c, &c->d_upd_g, ug)) ||
        (st = upload(c, &c->d_frec, rec)) || (st = dalloc(c, &c->d_fticket, 2)))
        return st;
    return BILU_OK;
}

// The whole factorisation in one persistent launch (k_factor_waves); false
// when there is no kernel for bs.
bool launch_factor_waves(bilu_ctx* c, const double* Ax, hipStream_t s)
{
    dev::FactorWaveArgs a{};
    a.rec = reinterpret_cast<const int4*>(c->d_frec);
    a.Pj = c->d_Pj;
    a.PtoA = c->d_PtoA;
    a.Ax = Ax;
    a.upd_ptr = c->d_upd_ptr;
    a.upd_f = c->d_upd_f;
    a.upd_g = c->d_upd_g;
    a.P = c->d_P;
    a.Dinv = c->d_Dinv;
    a.bad_row = c->d_bad;
    a.ticket = c->d_fticket;
    a.status = reinterpret_cast<int*>(c->d_fticket + 1);
    const HostSweep& L = c->h.sweep[BILU_SWEEP_L];
    a.nrows = L.level_ptr[L.nlev];
    a.lds_per_wave = c->fwave_lds;
    a.spin_limit = c->spin_limit;
    // wavefronts per workgroup: 8 where the LDS allows (measured on MI355X,
    // 60x220x85: ILU(0) 2.40 ms with 16, 2.05 with 8, 3.54 with 4 -- four rows
    // per ticket make the ticket counter the bottleneck; ILU(1) 4.60 / 4.38 /
    // 4.73), fewer for larger rows; BILU_TUNE_FACTOR 2: 16 where the LDS
    // allows, 3: at most 4
    const int nw = c->factor_mode == 2 ? c->fwave_n : std::min(c->fwave_n, c->factor_mode == 3 ? 4 : 8);
    const int groups = (a.nrows + nw - 1) / nw;
    const int blocks = std::max(1, std::min(groups, (32 / nw) * std::max(1, c->num_cu)));
    const size_t lds = static_cast<size_t>(c->fwave_lds) * nw;
    if (nw == 16) {
        BILU_SWITCH_B(c->h.bs, hipLaunchKernelGGL((dev::k_factor_waves<B, 16>), dim3(blocks), dim3(64 * 16), lds, s, a))
    }
    if (nw == 8) {
        BILU_SWITCH_B(c->h.bs, hipLaunchKernelGGL((dev::k_factor_waves<B, 8>), dim3(blocks), dim3(64 * 8), lds, s, a))
    }
    if (nw == 4) {
        BILU_SWITCH_B(c->h.bs, hipLaunchKernelGGL((dev::k_factor_waves<B, 4>), dim3(blocks), dim3(64 * 4), lds, s, a))
    }
    if (nw == 2) {
        BILU_SWITCH_B(c->h.bs, hipLaunchKernelGGL((dev::k_factor_waves<B, 2>), dim3(blocks), dim3(64 * 2), lds, s, a))
    }
    BILU_SWITCH_B(c->h.bs, hipLaunchKernelGGL((dev::k_factor_waves<B, 1>), dim3(blocks), dim3(64), lds, s, a))
}

bool launch_split(const bilu_ctx* c, hipStream_t s)
{
    const int64_t nP = static_cast<int64_t>(c->h.Pj.size());
    if (c->h.bs > kMaxKernelBs) {
        const int bs = c->h.bs;
        hipLaunchKernelGGL(dev::k_split_gen, dim3(grid_for(nP * bs * bs)), dim3(256), 0, s, nP, bs, c->d_Prow, c->d_Pj,
                           c->d_P, c->d_Dinv, c->d_F);
        return true;
    }
    BILU_SWITCH_B(c->h.bs, hipLaunchKernelGGL((dev::k_split<B>), dim3(grid_for(nP * B * B)), dim3(256), 0, s, nP,
                                              c->d_Prow, c->d_Pj, c->d_P, c->d_Dinv, c->d_F))
}

// Sweep layouts with a compile-time block size (k_layout_b, k_layout_dinv_b;
// dinv: the fused sweep's D^{-1} rows, or null).
template <typename T>
void layout_b_t(int bs, int64_t nslots, int64_t nrs, const int64_t* src, const int32_t* rows, const int32_t* Prow,
                const double* P, const double* Dinv, int up, int tr, void* vals, void* dinv, hipStream_t s, bool& ok)
{
    ok = true;
    switch (bs) {
#define BILU_LAYOUT_CASE(BV)                                                                                         \
    case BV:                                                                                                       \
        hipLaunchKernelGGL((dev::k_layout_b<BV, T>), dim3(grid_for(nslots * BV * BV)), dim3(256), 0, s, nslots, src, \
                           Prow, P, Dinv, up, tr, static_cast<T*>(vals));                                          \
        if (dinv)                                                                                                  \
            hipLaunchKernelGGL((dev::k_layout_dinv_b<BV, T>), dim3(grid_for(nrs * BV * BV)), dim3(256), 0, s, nrs,   \
                               rows, Dinv, tr, static_cast<T*>(dinv));                                             \
        return;
        BILU_LAYOUT_CASE(1)
        BILU_LAYOUT_CASE(2)
        BILU_LAYOUT_CASE(3)
        BILU_LAYOUT_CASE(4)
        BILU_LAYOUT_CASE(5)
        BILU_LAYOUT_CASE(6)
        BILU_LAYOUT_CASE(7)
        BILU_LAYOUT_CASE(8)
#undef BILU_LAYOUT_CASE
    }
    ok = false;
}

bool launch_layout_b(int bs, bool fp32, int64_t nslots, int64_t nrs, const int64_t* src, const int32_t* rows,
                     const int32_t* Prow, const double* P, const double* Dinv, int up, int tr, void* vals, void* dinv,
                     hipStream_t s)
{
    bool ok = false;
    if (fp32)
        layout_b_t<float>(bs, nslots, nrs, src, rows, Prow, P, Dinv, up, tr, vals, dinv, s, ok);
    else
        layout_b_t<double>(bs, nslots, nrs, src, rows, Prow, P, Dinv, up, tr, vals, dinv, s, ok);
    return ok;
}

void free_form(bilu_ctx* c, int form);

// Tile size and group size of the tiled layouts from the requests (0: the
// host simulation's choice), for the device's LDS.
void choose_layout(bilu_ctx* c)
{
    if (c->tile_rows_req > 0 && c->tile_group_req > 0) {
        // both given: no simulation (a tile's rows stay within 64 KiB of LDS)
        const int64_t cap = std::min<int64_t>(c->lds_max, 65536) / (8LL * c->h.bs) - 1;
        c->tile_rows = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>({c->tile_rows_req, c->h.nb, cap})));
        c->tile_group = std::min(c->tile_group_req, kGroupMax);
    } else {
        const TileChoice best =
            rank_tile_layouts(c->h, c->h.rpc, c->lds_max, c->tile_rows_req, c->tile_group_req).front();
        c->tile_rows = std::max(1, std::min(best.tile_rows, c->h.nb));
        c->tile_group = best.group;
    }
    c->layout_lds = c->lds_max;
}

// Tiled layout of sweep w as requested: line blocks where asked for and
// possible, else row-range tiles of the chosen size and group.
void build_tiled_layout(bilu_ctx* c, int w)
{
    HostTiled& ht = c->h.tiled[w];
    ht.built = false;
    if (c->tile_block > 0) build_tiled_blocks(c->h, w, c->h.rpc, c->tile_block & 255, c->tile_block >> 8, ht);
    if (!ht.built) build_tiled(c->h, w, c->h.rpc, c->tile_rows, c->tile_group, c->lds_max, true, ht);
}

// Group size the tiled layouts were built with (they fall back to smaller
// groups where a larger one cannot be used).
int built_group(const bilu_ctx* c)
{
    const HostTiled& ht = c->h.tiled[BILU_SWEEP_L];
    return ht.built ? ht.group : c->tile_group;
}

// New layout requests: the tiled layouts are rebuilt (host) if the choice
// changes, and uploaded again on their next use.
bilu_status set_layout(bilu_ctx* c, int tile_rows_req, int tile_group_req)
{
    const int rows0 = c->tile_rows, group0 = c->tile_group;
    c->tile_rows_req = tile_rows_req;
    c->tile_group_req = tile_group_req;
    choose_layout(c);
    if (c->tile_rows == rows0 && c->tile_group == group0) return BILU_OK;
    free_form(c, kFormTiled);
    c->layouts_checked = false;
    for (int w = 0; w < 4; ++w)
        if (c->h.sweep[w].built) build_tiled_layout(c, w);
    return BILU_OK;
}

// ----- device setup --------------------------------------------------------
bilu_status upload_form(bilu_ctx* c, int form)
{
    Host& h = c->h;
    bilu_status st;
    for (int w = 0; w < 4; ++w) {
        DevSweep& d = c->ds[form][w];
        if (form == kFormLevel) {
            const HostSweep& hs = h.sweep[w];
            if (!hs.built) continue;
            if ((st = upload(c, &d.chunk_off, hs.chunk_off)) || (st = upload(c, &d.rows, hs.rows)) ||
                (st = upload(c, &d.cols, hs.cols)) || (st = upload(c, &d.src, hs.src)))
                return st;
        } else if (form == kFormLines) {
            const HostTiled& hl = h.lines[w];
            if (!hl.built) continue;
            if ((st = upload(c, &d.rows, hl.rows)) || (st = upload(c, &d.src, hl.src))) return st;
        } else {
            if (!h.sweep[w].built) continue;
            if (c->tile_rows <= 0 || c->layout_lds != c->lds_max) choose_layout(c);
            HostTiled& ht = h.tiled[w];
            if (!ht.built || (!ht.block_ny && (ht.tile_rows != c->tile_rows || ht.group_req != c->tile_group))) {
                build_tiled_layout(c, w);
                c->layouts_checked = false;
            }
            std::vector<int32_t> crow(ht.chunk_off.size());
            for (size_t i = 0; i < crow.size(); ++i) {
                if (ht.chunk_off[i] % h.rpc != 0 || ht.chunk_off[i] / h.rpc > INT32_MAX) return BILU_ERR_STATE;
                crow[i] = static_cast<int32_t>(ht.chunk_off[i] / h.rpc);
            }
            if ((st = upload(c, &d.chunk_off, ht.chunk_off)) || (st = upload(c, &d.rows, ht.rows)) ||
                (st = upload(c, &d.cols, ht.deps)) || (st = upload(c, &d.src, ht.src)) ||
                (st = upload(c, &d.tile_chunk_ptr, ht.tile_chunk_ptr)) || (st = upload(c, &d.tile_lo, ht.tile_lo)) ||
                (st = upload(c, &d.chunk_row, crow)) || (st = upload(c, &d.group_tiles, ht.group_tiles)) ||
                (st = upload(c, &d.chunk_wait, ht.chunk_wait)))
                return st;
        }
        d.vals_precision = -1;
    }
    // no kernel ever runs on a layout that fails the host self-check
    if (!c->layouts_checked) {
        if (validate_layout(h) != BILU_OK) return BILU_ERR_STATE;
        c->layouts_checked = true;
    }
    c->form_uploaded[form] = true;
    return BILU_OK;
}

void free_form(bilu_ctx* c, int form)
{
    for (int w = 0; w < 4; ++w) {
        DevSweep& d = c->ds[form][w];
        for (void* p : {static_cast<void*>(d.chunk_off), static_cast<void*>(d.rows), static_cast<void*>(d.cols),
                        static_cast<void*>(d.src), static_cast<void*>(d.tile_chunk_ptr),
                        static_cast<void*>(d.tile_lo), static_cast<void*>(d.chunk_row), static_cast<void*>(d.fused),
                        static_cast<void*>(d.group_tiles), static_cast<void*>(d.chunk_wait), d.vals, d.dinv})
            dfree(c, p);
        d = DevSweep{};
    }
    c->form_uploaded[form] = false;
}

bilu_status ensure_device(bilu_ctx* c)
{
    if (c->dev_ready) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != c->device) return BILU_ERR_STATE;
        return BILU_OK;
    }
    CK(hipGetDevice(&c->device));
    hipDeviceProp_t prop;
    CK(hipGetDeviceProperties(&prop, c->device));
    c->num_cu = prop.multiProcessorCount;
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) == hipSuccess &&
            lds >= 65536)
            c->lds_max = lds;
    }
    Host& h = c->h;
    bilu_status st;
    const size_t bb = static_cast<size_t>(h.bs) * h.bs;
    if ((st = upload(c, &c->d_Ap, h.Ap)) || (st = upload(c, &c->d_Aj, h.Aj)) ||
        (st = upload(c, &c->d_Arow, h.Arow)) || (st = upload(c, &c->d_Pp, h.Pp)) ||
        (st = upload(c, &c->d_Pj, h.Pj)) || (st = upload(c, &c->d_Prow, h.Prow)) ||
        (st = upload(c, &c->d_Pdiag, h.Pdiag)) ||
        (st = upload(c, &c->d_Lrows, h.sweep[BILU_SWEEP_L].level_rows)))
        return st;
    {
        std::vector<int32_t> PtoA(h.Pj.size(), -1);
        for (size_t e = 0; e < h.AtoP.size(); ++e) PtoA[h.AtoP[e]] = static_cast<int32_t>(e);
        if ((st = upload(c, &c->d_PtoA, PtoA))) return st;
    }
    if (h.flags & BILU_WANT_TRANSPOSE) {
        if ((st = upload(c, &c->d_ATp, h.ATp)) || (st = upload(c, &c->d_ATj, h.ATj)) ||
            (st = upload(c, &c->d_ATsrc, h.ATsrc)))
            return st;
    }
    if ((st = dalloc(c, &c->d_P, h.Pj.size() * bb)) || (st = dalloc(c, &c->d_F, h.Pj.size() * bb)) ||
        (st = dalloc(c, &c->d_Dinv, static_cast<size_t>(h.nb) * bb)) || (st = dalloc(c, &c->d_bad, 1)) ||
        (st = dalloc(c, &c->d_status, 1)) || (st = dalloc(c, &c->d_done, 1)) ||
        (st = dalloc(c, &c->d_ticket, 1)))
        return st;
    CK(hipMemset(c->d_status, 0, sizeof(int)));
    CK(hipMemset(c->d_done, 0, sizeof(unsigned int)));
    CK(hipMemset(c->d_ticket, 0, sizeof(unsigned long long)));
    if (!c->values_only && (st = factor_plan(c))) return st;
    c->dev_ready = true;
    return BILU_OK;
}

// Layout form the sweeps use: row tiles in mode 2 (their vector accesses are
// 31-bit byte offsets, so the (n x R) vectors must stay below 2 GiB), level
// chunks otherwise.
// Sweep `which` of R columns runs as a line sweep.
bool use_lines(const bilu_ctx* c, int which, int R)
{
    return c->line_block > 0 && R == 1 && c->sweep_mode == 2 && c->h.lines[which].built;
}

int sweep_form(const bilu_ctx* c, int R)
{
    const bool fits = static_cast<int64_t>(c->h.nb) * c->h.bs * 8 * R <= static_cast<int64_t>(INT32_MAX);
    return c->sweep_mode == 2 && fits ? kFormTiled : kFormLevel;
}

// Factor values of one layout form in the current precision.
bilu_status layout_form(bilu_ctx* c, int form, hipStream_t s)
{
    Host& h = c->h;
    const int bb = h.bs * h.bs;
    const size_t esz = c->precision == BILU_FACTORS_FP32 ? sizeof(float) : sizeof(double);
    bilu_status st;
    if (!c->form_uploaded[form] && (st = upload_form(c, form))) return st;
    for (int w = 0; w < 4; ++w) {
        if (!h.sweep[w].built) continue;
        DevSweep& d = c->ds[form][w];
        if (d.vals_precision == c->precision) continue;
        if (form == kFormLines && !h.lines[w].built) continue;
        const int64_t nslots = form == kFormLevel ? h.sweep[w].nslots
                               : form == kFormTiled ? h.tiled[w].nslots : h.lines[w].nslots;
        const int nchunks = form == kFormLevel ? h.sweep[w].nchunks
                            : form == kFormTiled ? h.tiled[w].nchunks : h.lines[w].nchunks;
        const int rpc = h.rpc;
        // a new factorisation of the same layout reuses the arrays (no
        // allocation on the factorisation path); another size or precision
        // allocates them again
        const size_t vbytes = static_cast<size_t>(nslots) * bb * esz;
        const size_t dbytes = fused_sweep(w) ? static_cast<size_t>(nchunks) * rpc * bb * esz : 0;
        if (!d.vals || d.vals_bytes != vbytes || d.dinv_bytes != dbytes) {
            dfree(c, d.vals);
            dfree(c, d.dinv);
            d.vals = d.dinv = nullptr;
            d.vals_bytes = d.dinv_bytes = 0;
            char* p = nullptr;
            if ((st = dalloc(c, &p, vbytes))) return st;
            d.vals = p;
            d.vals_bytes = vbytes;
            if (dbytes) {
                if ((st = dalloc(c, &p, dbytes))) return st;
                d.dinv = p;
                d.dinv_bytes = dbytes;
            }
        }
        const int tr = transposed_sweep(w) ? 1 : 0;
        const int up = (w == BILU_SWEEP_U || w == BILU_SWEEP_UT) ? 1 : 0;
        const int64_t nrs = static_cast<int64_t>(nchunks) * rpc;
        if (rpc == kWave / h.bs && h.bs <= kMaxKernelBs && nslots % rpc == 0) {
            if (!launch_layout_b(h.bs, c->precision == BILU_FACTORS_FP32, nslots, nrs, d.src, d.rows, c->d_Prow,
                                 c->d_P, c->d_Dinv, up, tr, d.vals, d.dinv, s))
                return BILU_ERR_ARG;
        } else if (c->precision == BILU_FACTORS_FP32) {
            hipLaunchKernelGGL(dev::k_layout<float>, dim3(grid_for(nslots * bb)), dim3(256), 0, s, nslots, h.bs, rpc,
                               d.src, c->d_Prow, c->d_P, c->d_Dinv, up, tr, static_cast<float*>(d.vals));
            if (d.dinv)
                hipLaunchKernelGGL(dev::k_layout_dinv<float>, dim3(grid_for(nrs * bb)), dim3(256), 0, s, nrs, h.bs,
                                   rpc, d.rows, c->d_Dinv, tr, static_cast<float*>(d.dinv));
        } else {
            hipLaunchKernelGGL(dev::k_layout<double>, dim3(grid_for(nslots * bb)), dim3(256), 0, s, nslots, h.bs,
                               rpc, d.src, c->d_Prow, c->d_P, c->d_Dinv, up, tr, static_cast<double*>(d.vals));
            if (d.dinv)
                hipLaunchKernelGGL(dev::k_layout_dinv<double>, dim3(grid_for(nrs * bb)), dim3(256), 0, s, nrs, h.bs,
                                   rpc, d.rows, c->d_Dinv, tr, static_cast<double*>(d.dinv));
        }
        CK(hipGetLastError());
        d.vals_precision = c->precision;
    }
    return BILU_OK;
}

// D^{-1} y by blocks ahead of an unfused U' sweep instead of inside it
// (BILU_TUNE_SPLIT_DINV): one right-hand side, tiled U' layout;
// automatically where U' rows keep six or more dependency slots in
// registers (ILU(k >= 1) on a 7-point grid), whose fused sweep spends the
// most on the D^{-1} loads.  With FP32 factors the block pass multiplies
// by the FP32-rounded D^{-1}, as the fused sweep does.  Same bits either way.
bool use_split_dinv(const bilu_ctx* c, int R)
{
    if (c->split_dinv == 1 || R != 1) return false;
    if (sweep_form(c, 1) != kFormTiled || use_lines(c, BILU_SWEEP_U, 1)) return false;
    return c->split_dinv == 2 || c->h.tiled[BILU_SWEEP_U].kmax >= 6;
}

// Second intermediate of an application (D^{-1} y), one column.
bilu_status ensure_y2(bilu_ctx* c, hipStream_t s)
{
    (void)s;
    const size_t need = static_cast<size_t>(c->h.nb) * c->h.bs;
    if (c->y2_cap >= need) return BILU_OK;
    dfree(c, c->d_y2);
    c->d_y2 = nullptr;
    c->y2_cap = 0;
    bilu_status st = dalloc(c, &c->d_y2, need);
    if (st) return st;
    c->y2_cap = need;
    return BILU_OK;
}

bilu_status ensure_y(bilu_ctx* c, int R, hipStream_t s)
{
    const size_t need = static_cast<size_t>(c->h.nb) * c->h.bs * R;
    if (c->y_cap >= need) return BILU_OK;
    dfree(c, c->d_y);
    c->d_y = nullptr;
    c->y_cap = 0;
    bilu_status st = dalloc(c, &c->d_y, need);
    if (st) return st;
    c->y_cap = need;
    hipLaunchKernelGGL(dev::k_fill_not_ready, dim3(grid_for(static_cast<int64_t>(need))), dim3(256), 0, s,
                       static_cast<int64_t>(need), c->d_y);
    CK(hipGetLastError());
    return BILU_OK;
}

int persistent_blocks(bilu_ctx* c, int units, int units_per_block, int per_cu)
{
    const int want = std::max(1, (units + units_per_block - 1) / units_per_block);
    const int cap = c->blocks_override > 0 ? c->blocks_override : c->num_cu * per_cu;
    return std::max(1, std::min(want, cap));
}

#ifdef BILU_TRACE
long long* g_trace_buf[4] = {nullptr, nullptr, nullptr, nullptr};
size_t g_trace_n[4] = {0, 0, 0, 0};
#endif

// Ticket, done count and status of a persistent sweep launch.
struct SweepSync {
    unsigned long long* ticket;
    unsigned int* done;
    int* status;
};

// sync: counters to use instead of the context's (may be null); timed:
// recorded in bilu_timing's sweep classes.
static bool launch_block_dinv(int bs, int64_t nb, const double* Dinv, const double* x, double* y, hipStream_t s,
                              const int* gate, bool f32 = false);

// scaled (U' sweep only, tiled form): D^{-1} rhs is formed into scaled by
// blocks first (k_block_dinv, the fused sweep's products in its order) and
// the sweep runs unfused on it; both count as the sweep's time.
bilu_status run_sweep(bilu_ctx* c, int which, const double* rhs, double* out, double* reset, int R, hipStream_t s,
                      const int* gate = nullptr, const SweepSync* sync = nullptr, bool timed = true,
                      double* scaled = nullptr)
{
    const int form = sweep_form(c, R);
    const long tslot = timed ? timing_begin(c, BILU_K_SWEEP_L + which, s) : -1;
    if (scaled) {
        if (which != BILU_SWEEP_U || form != kFormTiled || R != 1 || use_lines(c, which, R)) return BILU_ERR_STATE;
        if (!launch_block_dinv(c->h.bs, c->h.nb, c->d_Dinv, rhs, scaled, s, gate,
                               c->precision == BILU_FACTORS_FP32))
            return BILU_ERR_ARG;
        rhs = scaled;
    }
    const SweepSync own{c->d_ticket, c->d_done, c->d_status};
    const SweepSync& sy = sync ? *sync : own;
    if (use_lines(c, which, R)) {
        const HostTiled& hl = c->h.lines[which];
        // the kernel's slot order: L z~, y~, x~ (forward); U' x~, y~, z~
        if (hl.line_dim[0] != (which == BILU_SWEEP_L ? 2 : 0) || hl.line_dim[1] != 1 ||
            hl.line_dim[2] != (which == BILU_SWEEP_L ? 0 : 2) || fused_sweep(which) != (which == BILU_SWEEP_U))
            return BILU_ERR_STATE;
        const DevSweep& d = c->ds[kFormLines][which];
        dev::LineArgs a{};
        a.vals = d.vals;
        a.dinv = d.dinv;
        a.rhs = rhs;
        a.out = out;
        a.reset = reset;
        a.ticket = sy.ticket;
        a.done = sy.done;
        a.status = sy.status;
        a.gate = gate;
        a.nx = hl.line_nx;
        a.ny = hl.line_ny;
        a.nz = hl.line_nz;
        a.WY = hl.block_ny;
        a.WZ = hl.block_nz;
        a.NYb = hl.line_NYb;
        a.nblocks = hl.ntiles;
        a.nsteps = hl.line_steps;
        a.forward = which == BILU_SWEEP_L ? 1 : 0;
        a.spin_limit = c->spin_limit;
        const int blocks = persistent_blocks(c, hl.ntiles, 1, 8);
        a.total_waves = static_cast<unsigned int>(blocks);
#ifdef BILU_TRACE
        {
            static long long* lbuf[4] = {nullptr, nullptr, nullptr, nullptr};
            static size_t lcap[4] = {0, 0, 0, 0};
            const size_t need = 4 * static_cast<size_t>(hl.nchunks) + hl.ntiles;
            if (lcap[which] < need) {
                if (lbuf[which]) (void)hipFree(lbuf[which]);
                if (hipMalloc(&lbuf[which], need * sizeof(long long)) != hipSuccess) return BILU_ERR_ALLOC;
                lcap[which] = need;
            }
            a.trace = lbuf[which];
            g_trace_buf[which] = lbuf[which];
            g_trace_n[which] = need;
        }
#endif
        if (!launch_lines(c->h.bs, c->precision, fused_sweep(which), blocks, s, a)) return BILU_ERR_ARG;
        timing_end(c, tslot, s);
        CK(hipGetLastError());
        return BILU_OK;
    }
    const int fuse = fused_sweep(which) && !scaled ? 1 : 0;
    if (form == kFormTiled) {
        const HostTiled& ht = c->h.tiled[which];
        const DevSweep& d = c->ds[kFormTiled][which];
        TiledArgs a{};
        a.tile_chunk_ptr = d.tile_chunk_ptr;
        a.tile_lo = d.tile_lo;
        a.chunk_row = d.chunk_row;
        a.rows = d.rows;
        a.deps = d.cols;
        a.vals = d.vals;
        a.dinv = d.dinv;
        a.rhs = rhs;
        a.out = out;
        a.reset = reset;
        a.ticket = sy.ticket;
        a.done = sy.done;
        a.status = sy.status;
        a.ntiles = ht.ntiles;
        a.R = R;
        a.spin_limit = c->spin_limit;
        a.group = ht.group;
        a.ngroups = ht.ngroups;
        a.group_tiles = d.group_tiles;
        a.chunk_wait = d.chunk_wait;
        a.gate = gate;
        // tickets: tiles (or groups of tiles) times right-hand sides
        const int blocks = ht.group > 1 ? persistent_blocks(c, ht.ngroups * R, 1, std::max(1, 8 / ht.group))
                                        : persistent_blocks(c, ht.ntiles * R, 1, 8);
        a.total_waves = static_cast<unsigned int>(blocks);
        a.ring = ht.ring;
        a.tile_rows = ht.ring > 0 ? ht.ring * c->h.rpc : ht.tile_rows;
        // the member tiles' rows (or the ring's), one row kept at zero
        // (padding slots read it) and the members' progress counts
        const size_t lds = static_cast<size_t>(tiled_lds_bytes(a.tile_rows, ht.group, c->h.bs));
        if (static_cast<int64_t>(lds) > c->lds_max) return BILU_ERR_STATE;
#ifdef BILU_TRACE
        {
            static long long* tbuf[4] = {nullptr, nullptr, nullptr, nullptr};
            static size_t tcap[4] = {0, 0, 0, 0};
            const size_t need = 4 * static_cast<size_t>(ht.nchunks) + ht.ntiles;
            if (tcap[which] < need) {
                if (tbuf[which]) (void)hipFree(tbuf[which]);
                if (hipMalloc(&tbuf[which], need * sizeof(long long)) != hipSuccess) return BILU_ERR_ALLOC;
                tcap[which] = need;
            }
            a.trace = tbuf[which];
            a.trace_nchunks = ht.nchunks;
            g_trace_buf[which] = tbuf[which];
            g_trace_n[which] = need;
        }
#endif
        const size_t hlds = static_cast<size_t>(helped_lds_bytes(a.tile_rows, ht.group, c->h.bs, ht.kmax));
        if (use_helper(c, ht, R) && static_cast<int64_t>(hlds) <= c->lds_max) {
            // one workgroup of 2 * group wavefronts per group (or tile)
            a.ngroups = ht.group > 1 ? ht.ngroups : ht.ntiles;
            const int hblocks = persistent_blocks(c, a.ngroups, 1, std::max(1, 4 / ht.group));
            a.total_waves = static_cast<unsigned int>(hblocks);
            if (!launch_helped(c->h.bs, ht.kmax, c->precision, fuse != 0, hblocks, hlds, s, a)) return BILU_ERR_ARG;
        } else if (use_pairs(c, ht, R, lds)) {
            // two right-hand sides per wavefront: tickets tiles times column pairs
            const int pblocks = persistent_blocks(c, ht.ntiles * (R / 2), 1, 8);
            a.total_waves = static_cast<unsigned int>(pblocks);
            if (!launch_pairs(c->h.bs, ht.kmax, c->precision, fuse != 0, pblocks, 2 * lds, s, a)) return BILU_ERR_ARG;
        } else if (!launch_tiled(c->h.bs, ht.kmax, c->precision, fuse != 0, R > 1, blocks, lds, s, a)) {
            return BILU_ERR_ARG;
        }
    } else {
        const HostSweep& hs = c->h.sweep[which];
        const DevSweep& d = c->ds[kFormLevel][which];
        SweepArgs a{};
        a.chunk_off = d.chunk_off;
        a.rows = d.rows;
        a.cols = d.cols;
        a.vals = d.vals;
        a.dinv = d.dinv;
        a.rhs = rhs;
        a.out = out;
        a.reset = reset;
        a.ticket = sy.ticket;
        a.done = sy.done;
        a.status = sy.status;
        a.nchunks = hs.nchunks;
        a.R = R;
        a.fuse = fuse;
        a.spin_limit = c->spin_limit;
        a.gate = gate;
        if (c->sweep_mode != 0) {
            a.persistent = 1;
            const int blocks = persistent_blocks(c, hs.nchunks, dev::kWavesPerBlock, 1);
            a.total_waves = static_cast<unsigned int>(blocks) * dev::kWavesPerBlock;
            if (!launch_sweep(c->h.bs, c->precision, rhs_tile(c, R), blocks, s, a)) return BILU_ERR_ARG;
        } else {
            a.persistent = 0;
            for (int l = 0; l < hs.nlev; ++l) {
                a.chunk_begin = hs.level_chunk_ptr[l];
                a.chunk_end = hs.level_chunk_ptr[l + 1];
                const int n = a.chunk_end - a.chunk_begin;
                if (n <= 0) continue;
                const int blocks = (n + dev::kWavesPerBlock - 1) / dev::kWavesPerBlock;
                if (!launch_sweep(c->h.bs, c->precision, rhs_tile(c, R), blocks, s, a)) return BILU_ERR_ARG;
            }
        }
    }
    timing_end(c, tslot, s);
    CK(hipGetLastError());
    return BILU_OK;
}

// Point rows of the split factors (block size b, pattern P): point row
// I*b + r holds, in ascending column order, the unit diagonal for the
// diagonal block (the diagonal blocks of L and U' are identities) and b
// entries per off-diagonal block (I, J), element (r, c) at column J*b + c.
static void expand_point_pattern(const Host& h, std::vector<int32_t>& Ap, std::vector<int32_t>& Aj,
                                 std::vector<int64_t>& src)
{
    const int b = h.bs;
    const int64_t bb = static_cast<int64_t>(b) * b;
    const int64_t n = static_cast<int64_t>(h.nb) * b;
    Ap.assign(static_cast<size_t>(n) + 1, 0);
    for (int32_t I = 0; I < h.nb; ++I) {
        const int32_t cnt = (h.Pp[I + 1] - h.Pp[I] - 1) * b + 1;
        for (int r = 0; r < b; ++r) Ap[static_cast<size_t>(I) * b + r + 1] = cnt;
    }
    for (int64_t i = 0; i < n; ++i) Ap[i + 1] += Ap[i];
    Aj.resize(static_cast<size_t>(Ap[n]));
    src.resize(static_cast<size_t>(Ap[n]));
    for (int32_t I = 0; I < h.nb; ++I)
        for (int r = 0; r < b; ++r) {
            int64_t q = Ap[static_cast<size_t>(I) * b + r];
            for (int32_t e = h.Pp[I]; e < h.Pp[I + 1]; ++e) {
                const int32_t J = h.Pj[e];
                if (J == I) {
                    Aj[q] = I * b + r;
                    src[q++] = -1;
                } else {
                    for (int c = 0; c < b; ++c) {
                        Aj[q] = J * b + c;
                        src[q++] = static_cast<int64_t>(e) * bb + static_cast<int64_t>(c) * b + r;
                    }
                }
            }
        }
}

// The point view of the current factors: its context (analysed once), then
// values expanded from F after every factorisation.
static bilu_status ensure_point(bilu_ctx* c, hipStream_t s)
{
    bilu_status st;
    const Host& h = c->h;
    const int64_t n = static_cast<int64_t>(h.nb) * h.bs;
    if (!c->point) {
        if (n > INT32_MAX) return BILU_ERR_ARG;
        std::vector<int32_t> Ap, Aj;
        std::vector<int64_t> src;
        try {
            expand_point_pattern(h, Ap, Aj, src);
        } catch (const std::bad_alloc&) {
            return BILU_ERR_ALLOC;
        }
        bilu_ctx* p = nullptr;
        if ((st = bilu_analyze(static_cast<int>(n), 1, Ap.data(), Aj.data(), 0, 0, &p))) return st;
        p->values_only = true;
        p->sweep_mode = c->sweep_mode;
        p->spin_limit = c->spin_limit;
        p->timing = c->timing;
        c->point = p;
        c->point_gen = 0;
        if ((st = ensure_device(p)) || (st = upload(c, &c->d_point_src, src)) ||
            (st = dalloc(c, &c->d_point_y, static_cast<size_t>(n))))
            return st;
        c->point_n = static_cast<int64_t>(src.size());
    }
    if (c->point_gen != c->factor_gen) {
        bilu_ctx* p = c->point;
        if (!c->f_ready) {
            if (!launch_split(c, s)) return BILU_ERR_ARG;
            c->f_ready = true;
        }
        hipLaunchKernelGGL(dev::k_expand_point, dim3(grid_for(c->point_n)), dim3(256), 0, s, c->point_n,
                           c->d_point_src, c->d_F, p->d_P);
        hipLaunchKernelGGL(dev::k_fill_f64, dim3(grid_for(n)), dim3(256), 0, s, n, p->d_Dinv, 1.0);
        CK(hipGetLastError());
        p->factored = true;
        if ((st = bilu_factor_diag(p, BILU_FACTORS_FP64, s))) return st;
        c->point_gen = c->factor_gen;
    }
    return BILU_OK;
}

static bool launch_block_dinv(int bs, int64_t nb, const double* Dinv, const double* x, double* y, hipStream_t s,
                              const int* gate, bool f32)
{
    if (bs > kMaxKernelBs) {
        if (f32) return false;
        hipLaunchKernelGGL(dev::k_block_dinv_gen, dim3(grid_for(nb * bs)), dim3(256), 0, s, nb, bs, Dinv, x, y, gate);
        return true;
    }
    if (f32) {
        BILU_SWITCH_B(bs, hipLaunchKernelGGL((dev::k_block_dinv<B, true>), dim3(grid_for(nb * B)), dim3(256), 0, s,
                                             nb, Dinv, x, y, gate))
    }
    BILU_SWITCH_B(bs, hipLaunchKernelGGL((dev::k_block_dinv<B>), dim3(grid_for(nb * B)), dim3(256), 0, s, nb, Dinv,
                                         x, y, gate))
}

// Reads and clears the expired-wait flag of the point view's sweeps (1 if
// set); the caller's own flag is read where the caller reads it.
static int point_sweep_error(bilu_ctx* c, hipStream_t s)
{
    if (!c->point || !c->point->dev_ready) return 0;
    int v = 0;
    if (hipMemcpyAsync(&v, c->point->d_status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return 1;
    if (v) {
        (void)hipMemsetAsync(c->point->d_status, 0, sizeof(int), s);
        (void)hipStreamSynchronize(s);
    }
    return v ? 1 : 0;
}

// z = M^{-1} r at point granularity (one right-hand side): L sweep on the
// point rows (resets z), D^{-1} by blocks, U' sweep on the point rows with
// the unit D^{-1} of the point context (resets y); nothing runs when gate
// is given and *gate == 0.
static bilu_status do_apply_point(bilu_ctx* c, const double* r, double* z, hipStream_t s, const int* gate)
{
    bilu_status st = ensure_point(c, s);
    if (st) return st;
    bilu_ctx* p = c->point;
    if ((st = layout_form(p, sweep_form(p, 1), s)) || (st = ensure_y(p, 1, s))) return st;
    if ((st = run_sweep(p, BILU_SWEEP_L, r, p->d_y, z, 1, s, gate))) return st;
    if (!launch_block_dinv(c->h.bs, c->h.nb, c->d_Dinv, p->d_y, c->d_point_y, s, gate)) return BILU_ERR_ARG;
    CK(hipGetLastError());
    return run_sweep(p, BILU_SWEEP_U, c->d_point_y, z, p->d_y, 1, s, gate);
}

// z = M^{-1} r: first sweep r -> y (resets z), second y -> z (resets y).
bilu_status do_apply(bilu_ctx* c, const double* r, double* z, int R, bool transpose, hipStream_t s,
                     const int* gate = nullptr)
{
    if (!c || !r || !z || R < 1 || R > dev::kMaxRhs || r == z) return BILU_ERR_ARG;
    if (!c->split_done) return BILU_ERR_STATE;
    if (c->h.bs > kMaxKernelBs) {
        // block sizes without block-row sweep kernels: point granularity
        if (R != 1 || transpose) return BILU_ERR_ARG;
        return do_apply_point(c, r, z, s, gate);
    }
    const int first = transpose ? BILU_SWEEP_UT : BILU_SWEEP_L;
    const int second = transpose ? BILU_SWEEP_LT : BILU_SWEEP_U;
    if (!c->h.sweep[first].built || !c->h.sweep[second].built) return BILU_ERR_STATE;
    bilu_status st;
    const int form = sweep_form(c, R);
    if ((st = layout_form(c, form, s))) return st;
    if ((use_lines(c, first, R) || use_lines(c, second, R)) && (st = layout_form(c, kFormLines, s))) return st;
    if ((st = ensure_y(c, R, s))) return st;
    if ((st = run_sweep(c, first, r, c->d_y, z, R, s, gate))) return st;
    if (!transpose && use_split_dinv(c, R)) {
        if ((st = ensure_y2(c, s))) return st;
        return run_sweep(c, second, c->d_y, z, c->d_y, R, s, gate, nullptr, true, c->d_y2);
    }
    return run_sweep(c, second, c->d_y, z, c->d_y, R, s, gate);
}

// timed: counted in the SpMV class of bilu_timing (the solvers' gated
// true-residual SpMV, mostly gated off, is not)
bilu_status do_spmv(bilu_ctx* c, const double* Ax, const double* x, double* y, int R, int transpose,
                    hipStream_t s, const int* gate = nullptr, bool timed = true)
{
    if (!c || !Ax || !x || !y || R < 1 || R > dev::kMaxRhs || x == y) return BILU_ERR_ARG;
    bilu_status st = ensure_device(c);
    if (st) return st;
    const Host& h = c->h;
    bool ok;
    const long tslot = timed ? timing_begin(c, BILU_K_SPMV, s) : -1;
    if (transpose) {
        if (!(h.flags & BILU_WANT_TRANSPOSE)) return BILU_ERR_STATE;
        ok = launch_spmv(h.bs, spmv_tile(c, R), true, h.nb, c->d_ATp, c->d_ATj, c->d_ATsrc, Ax, x, y, R, s, gate);
    } else {
        ok = launch_spmv(h.bs, spmv_tile(c, R), false, h.nb, c->d_Ap, c->d_Aj, nullptr, Ax, x, y, R, s, gate,
                         spmv_streams_a(c, R));
    }
    timing_end(c, tslot, s);
    if (!ok) return BILU_ERR_ARG;
    CK(hipGetLastError());
    return BILU_OK;
}

// z = M^{-1} r and y = A z for one right-hand side: the L sweep, then the
// U' sweep and the SpMV in one launch (tiles and SpMV blocks share its
// ticket order).  Falls back to the separate calls where the fused launch
// does not apply (other sweep forms, transposes, several columns).
bilu_status do_apply_spmv(bilu_ctx* c, const double* Ax, const double* r, double* z, double* y, int R,
                          bool transpose, hipStream_t s, const int* gate = nullptr)
{
    if (transpose || R != 1 || sweep_form(c, 1) != kFormTiled || !c->fuse_spmv) {
        bilu_status st = do_apply(c, r, z, R, transpose, s, gate);
        return st ? st : do_spmv(c, Ax, z, y, R, transpose ? 1 : 0, s, gate);
    }
    if (!c || !Ax || !r || !z || !y || r == z || y == z) return BILU_ERR_ARG;
    if (!c->split_done) return BILU_ERR_STATE;
    bilu_status st;
    if ((st = layout_form(c, kFormTiled, s))) return st;
    if (c->h.tiled[BILU_SWEEP_U].group > 1 || c->h.tiled[BILU_SWEEP_U].block_ny) {
        // the fused ticket order is for single row-range tiles
        st = do_apply(c, r, z, R, false, s, gate);
        return st ? st : do_spmv(c, Ax, z, y, R, 0, s, gate);
    }
    if ((st = ensure_y(c, 1, s))) return st;
    HostTiled& hu = c->h.tiled[BILU_SWEEP_U];
    DevSweep& du = c->ds[kFormTiled][BILU_SWEEP_U];
    if (!du.fused) {
        if (build_fused_schedule(c->h, hu, hu.fused) != BILU_OK) return BILU_ERR_STATE;
        if ((st = upload(c, &du.fused, hu.fused))) return st;
    }
    if ((st = run_sweep(c, BILU_SWEEP_L, r, c->d_y, z, 1, s, gate))) return st;
    // U' sweep + SpMV
    const long tslot = timing_begin(c, BILU_K_SWEEP_U_SPMV, s);
    TiledArgs a{};
    a.tile_chunk_ptr = du.tile_chunk_ptr;
    a.tile_lo = du.tile_lo;
    a.chunk_row = du.chunk_row;
    a.rows = du.rows;
    a.deps = du.cols;
    a.vals = du.vals;
    a.dinv = du.dinv;
    a.rhs = c->d_y;
    a.out = z;
    a.reset = c->d_y;
    a.ticket = c->d_ticket;
    a.done = c->d_done;
    a.status = c->d_status;
    a.ntiles = hu.ntiles;
    a.ring = hu.ring;
    a.tile_rows = hu.ring > 0 ? hu.ring * c->h.rpc : hu.tile_rows;
    a.R = 1;
    a.spin_limit = c->spin_limit;
    a.gate = gate;
    dev::FusedSpmvArgs m{};
    m.sched = du.fused;
    m.nsched = static_cast<int>(hu.fused.size());
    m.nb = c->h.nb;
    m.Ap = c->d_Ap;
    m.Aj = c->d_Aj;
    m.Ax = Ax;
    m.y = y;
    // one wavefront per tile plus one per compute unit: SpMV blocks mostly
    // run on wavefronts whose tile is done, few wait and poll
    const int blocks = persistent_blocks(c, std::min(m.nsched, hu.ntiles + c->num_cu), 1, 8);
    a.total_waves = static_cast<unsigned int>(blocks);
    const size_t lds = static_cast<size_t>(a.tile_rows + 1) * c->h.bs * sizeof(double);
    const bool ok = launch_fused(c->h.bs, hu.kmax, c->precision, blocks, lds, s, a, m);
    timing_end(c, tslot, s);
    if (!ok) return BILU_ERR_ARG;
    CK(hipGetLastError());
    return BILU_OK;
}

}  // namespace

// ===========================================================================
// ABI
// ===========================================================================
extern "C" {

#ifdef BILU_TRACE
// trace of the last tiled launch of sweep `which`: chunk finish times, then
// tile start times (device wall clock); also the tile -> chunk map
int64_t bilu_trace_get(bilu_ctx* c, int which, long long* host, int64_t cap, int32_t* tile_ptr, int32_t* group_tiles,
                       int64_t cap2)
{
    if (!g_trace_buf[which]) return -1;
    (void)hipDeviceSynchronize();
    const int64_t n = std::min<int64_t>(cap, g_trace_n[which]);
    (void)hipMemcpy(host, g_trace_buf[which], n * sizeof(long long), hipMemcpyDeviceToHost);
    const HostTiled& ht = use_lines(c, which, 1) ? c->h.lines[which] : c->h.tiled[which];
    for (int64_t i = 0; i < std::min<int64_t>(cap2, ht.tile_chunk_ptr.size()); ++i) tile_ptr[i] = ht.tile_chunk_ptr[i];
    for (int64_t i = 0; i < std::min<int64_t>(cap2, ht.group_tiles.size()); ++i) group_tiles[i] = ht.group_tiles[i];
    return n;
}
#endif

bilu_status bilu_analyze(int nb, int bs, const int32_t* Ap, const int32_t* Aj, int k, int flags,
                         bilu_ctx** out)
{
    if (!out) return BILU_ERR_ARG;
    *out = nullptr;
    bilu_ctx* c = new (std::nothrow) bilu_ctx();
    if (!c) return BILU_ERR_ALLOC;
    int st;
    try {
        st = analyze_host(c->h, nb, bs, Ap, Aj, k, flags);
    } catch (const std::bad_alloc&) {
        st = BILU_ERR_ALLOC;
    }
    if (st != BILU_OK) {
        delete c;
        return static_cast<bilu_status>(st);
    }
    *out = c;
    return BILU_OK;
}

bilu_status bilu_get_pattern(const bilu_ctx* c, int64_t* nnzb, const int32_t** Pp, const int32_t** Pj,
                             const int32_t** lev)
{
    if (!c) return BILU_ERR_ARG;
    if (nnzb) *nnzb = static_cast<int64_t>(c->h.Pj.size());
    if (Pp) *Pp = c->h.Pp.data();
    if (Pj) *Pj = c->h.Pj.data();
    if (lev) *lev = c->h.Plev.data();
    return BILU_OK;
}

bilu_status bilu_get_levels(const bilu_ctx* c, int sweep, int* nlev, const int32_t** level_ptr,
                            const int32_t** level_rows)
{
    if (!c || sweep < 0 || sweep > 3) return BILU_ERR_ARG;
    const HostSweep& hs = c->h.sweep[sweep];
    if (!hs.built) return BILU_ERR_STATE;
    if (nlev) *nlev = hs.nlev;
    if (level_ptr) *level_ptr = hs.level_ptr.data();
    if (level_rows) *level_rows = hs.level_rows.data();
    return BILU_OK;
}

bilu_status bilu_get_info(const bilu_ctx* c, bilu_info* info)
{
    if (!c || !info) return BILU_ERR_ARG;
    const Host& h = c->h;
    std::memset(info, 0, sizeof(*info));
    info->nb = h.nb;
    info->bs = h.bs;
    info->k = h.k;
    info->nnzb_A = static_cast<int64_t>(h.Aj.size());
    info->nnzb_P = static_cast<int64_t>(h.Pj.size());
    for (int i = 0; i < h.nb; ++i)
        for (int32_t e = h.Pp[i]; e < h.Pp[i + 1]; ++e) {
            if (h.Pj[e] < i) info->nnzb_L++;
            if (h.Pj[e] > i) info->nnzb_U++;
        }
    info->rows_per_chunk = h.rpc;
    info->tile_rows = c->tile_rows;
    info->tile_group = built_group(c);
    for (int w = 0; w < 4; ++w) {
        info->nlev[w] = h.sweep[w].built ? h.sweep[w].nlev : 0;
        info->sweep_slots[w] = h.sweep[w].built ? h.sweep[w].nslots : 0;
        info->lds_ring[w] = h.tiled[w].built ? h.tiled[w].ring : 0;
        info->tile_block[w] = h.tiled[w].built && h.tiled[w].block_ny ? h.tiled[w].block_ny + 256 * h.tiled[w].block_nz : 0;
    }
    for (int w = 0; w < 2; ++w)
        info->line_sweep[w] = use_lines(c, w, 1) ? h.lines[w].block_ny + 256 * h.lines[w].block_nz : 0;
    return BILU_OK;
}

bilu_status bilu_validate(const bilu_ctx* c)
{
    if (!c) return BILU_ERR_ARG;
    return static_cast<bilu_status>(validate_layout(c->h));
}

bilu_status bilu_factor_numeric(bilu_ctx* c, const double* Ax, hipStream_t s, int* bad_row)
{
    if (bad_row) *bad_row = -1;
    if (!c || !Ax) return BILU_ERR_ARG;
    bilu_status st = ensure_device(c);
    if (st) return st;
    Host& h = c->h;
    const int bb = h.bs * h.bs;
    const int64_t nP = static_cast<int64_t>(h.Pj.size());
    c->factored = false;
    c->split_done = false;
    c->f_ready = false;
    const long tslot = timing_begin(c, BILU_K_FACTOR, s);
    hipLaunchKernelGGL(dev::k_fill_i32, dim3(1), dim3(64), 0, s, int64_t(1), c->d_bad, INT_MAX);
    const bool waves = c->factor_mode != 1 && c->fwave_lds > 0 && !c->values_only;
    if (waves) {
        // P and D^{-1} start at kNotReady (rows read A directly); the ticket
        // and the expired-wait word at zero
        hipLaunchKernelGGL(dev::k_fill_not_ready, dim3(grid_for(nP * bb)), dim3(256), 0, s, nP * bb, c->d_P);
        hipLaunchKernelGGL(dev::k_fill_not_ready, dim3(grid_for(static_cast<int64_t>(h.nb) * bb)), dim3(256), 0, s,
                           static_cast<int64_t>(h.nb) * bb, c->d_Dinv);
        hipLaunchKernelGGL(dev::k_fill_i32, dim3(1), dim3(64), 0, s, int64_t(2),
                           reinterpret_cast<int32_t*>(c->d_fticket), 0);
        if (!launch_factor_waves(c, Ax, s)) return BILU_ERR_ARG;
    } else {
        if (!launch_backfill(h.bs, nP, c->d_PtoA, Ax, c->d_P, s))
            hipLaunchKernelGGL(dev::k_backfill, dim3(grid_for(nP * bb)), dim3(256), 0, s, nP, bb, c->d_PtoA, Ax,
                               c->d_P);
        const HostSweep& L = h.sweep[BILU_SWEEP_L];
        for (int l = 0; l < L.nlev; ++l) {
            const int n = L.level_ptr[l + 1] - L.level_ptr[l];
            const int lds = l < static_cast<int>(c->fac_lds.size()) ? c->fac_lds[l] : 0;
            if (!launch_factor(h.bs, L.level_ptr[l], n, lds, c, s)) return BILU_ERR_ARG;
        }
    }
    timing_end(c, tslot, s);
    CK(hipGetLastError());
    int bad = INT_MAX;
    int expired = 0;
    CK(hipMemcpyAsync(&bad, c->d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    if (waves) CK(hipMemcpyAsync(&expired, c->d_fticket + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (expired) return BILU_ERR_TIMEOUT;
    c->factored = true;
    if (bad != INT_MAX) {
        if (bad_row) *bad_row = bad;
        return BILU_SINGULAR_PIVOT;
    }
    return BILU_OK;
}

bilu_status bilu_factor_diag(bilu_ctx* c, int precision, hipStream_t s)
{
    if (!c || (precision != BILU_FACTORS_FP64 && precision != BILU_FACTORS_FP32)) return BILU_ERR_ARG;
    if (!c->factored) return BILU_ERR_STATE;
    if (c->h.bs > kMaxKernelBs) {
        // no block-row sweep layouts: the point view is formed from F when an
        // application first needs it
        if (precision != BILU_FACTORS_FP64) return BILU_ERR_ARG;
        c->f_ready = false;
        c->precision = precision;
        c->split_done = true;
        ++c->factor_gen;
        return BILU_OK;
    }
    const long tslot = timing_begin(c, BILU_K_SPLIT, s);
    c->f_ready = false;                       // F is formed when a caller asks for it
    c->precision = precision;
    for (int f = 0; f < kForms; ++f)
        for (int w = 0; w < 4; ++w) c->ds[f][w].vals_precision = -1;
    bilu_status st = layout_form(c, sweep_form(c, 1), s);
    if (st) return st;
    if (use_lines(c, BILU_SWEEP_L, 1) || use_lines(c, BILU_SWEEP_U, 1)) {
        if ((st = layout_form(c, kFormLines, s))) return st;
    }
    timing_end(c, tslot, s);
    CK(hipGetLastError());
    c->split_done = true;
    ++c->factor_gen;
    return BILU_OK;
}

bilu_status bilu_get_factors(const bilu_ctx* c, double* F, double* Dinv, hipStream_t s)
{
    if (!c) return BILU_ERR_ARG;
    if (!c->split_done) return BILU_ERR_STATE;
    const size_t bb = static_cast<size_t>(c->h.bs) * c->h.bs;
    if (F && !c->f_ready) {
        if (!launch_split(c, s)) return BILU_ERR_ARG;
        c->f_ready = true;
    }
    if (F) CK(hipMemcpyAsync(F, c->d_F, c->h.Pj.size() * bb * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (Dinv)
        CK(hipMemcpyAsync(Dinv, c->d_Dinv, static_cast<size_t>(c->h.nb) * bb * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
    return BILU_OK;
}

bilu_status bilu_get_factors_f32(bilu_ctx* c, float* F, float* Dinv, hipStream_t s)
{
    if (!c) return BILU_ERR_ARG;
    if (!c->split_done || c->precision != BILU_FACTORS_FP32) return BILU_ERR_STATE;
    bilu_status st = layout_form(c, kFormLevel, s);
    if (st) return st;
    const Host& h = c->h;
    const int bb = h.bs * h.bs;
    if (F) {
        for (int w : {BILU_SWEEP_L, BILU_SWEEP_U}) {
            const HostSweep& hs = h.sweep[w];
            hipLaunchKernelGGL(dev::k_unlayout_f32, dim3(grid_for(hs.nslots * bb)), dim3(256), 0, s, hs.nslots, h.bs,
                               hs.rpc, c->ds[kFormLevel][w].src, static_cast<const float*>(c->ds[kFormLevel][w].vals),
                               F);
        }
        hipLaunchKernelGGL(dev::k_identity_f32, dim3(grid_for(static_cast<int64_t>(h.nb) * bb)), dim3(256), 0, s,
                           h.nb, h.bs, c->d_Pdiag, F);
    }
    if (Dinv) {
        const HostSweep& hs = h.sweep[BILU_SWEEP_U];
        const int64_t nrs = static_cast<int64_t>(hs.nchunks) * hs.rpc;
        hipLaunchKernelGGL(dev::k_unlayout_dinv_f32, dim3(grid_for(nrs * bb)), dim3(256), 0, s, nrs, h.bs, hs.rpc,
                           c->ds[kFormLevel][BILU_SWEEP_U].rows,
                           static_cast<const float*>(c->ds[kFormLevel][BILU_SWEEP_U].dinv), Dinv);
    }
    CK(hipGetLastError());
    return BILU_OK;
}

bilu_status bilu_apply(bilu_ctx* c, const double* r, double* z, int nrhs, hipStream_t s)
{
    return do_apply(c, r, z, nrhs, false, s);
}

bilu_status bilu_apply_noalloc(bilu_ctx* c, const double* r, double* z, int nrhs, hipStream_t s)
{
    if (!c || !r || !z || nrhs < 1 || nrhs > dev::kMaxRhs || r == z || c->h.bs > kMaxKernelBs) return BILU_ERR_ARG;
    const int64_t ny = static_cast<int64_t>(c->h.nb) * c->h.bs * nrhs;
    if (static_cast<size_t>(ny) * sizeof(double) > kScratchBytes - kScratchHeader) return BILU_ERR_ARG;
    if (!c->dev_ready || !c->split_done) return BILU_ERR_STATE;
    // the layouts of this form must already hold the current factors: laying
    // them out would allocate
    const int form = sweep_form(c, nrhs);
    for (int w : {static_cast<int>(BILU_SWEEP_L), static_cast<int>(BILU_SWEEP_U)}) {
        const int f = use_lines(c, w, nrhs) ? kFormLines : form;
        if (!c->form_uploaded[f] || !c->h.sweep[w].built || c->ds[f][w].vals_precision != c->precision)
            return BILU_ERR_STATE;
    }
    int device = -1;
    CK(hipGetDevice(&device));
    if (device != c->device) return BILU_ERR_STATE;
    unsigned char* base = nullptr;
    bilu_status st = scratch_of_device(device, &base);
    if (st) return st;
    const SweepSync sync{reinterpret_cast<unsigned long long*>(base), reinterpret_cast<unsigned int*>(base + 8),
                         reinterpret_cast<int*>(base + 12)};
    double* y = reinterpret_cast<double*>(base + kScratchHeader);
    // the scratch keeps the last call's contents: counters cleared and y set
    // to kNotReady by fill kernels on every call
    hipLaunchKernelGGL(dev::k_fill_i32, dim3(1), dim3(64), 0, s, int64_t(4), reinterpret_cast<int32_t*>(base), 0);
    hipLaunchKernelGGL(dev::k_fill_not_ready, dim3(grid_for(ny)), dim3(256), 0, s, ny, y);
    CK(hipGetLastError());
    if ((st = run_sweep(c, BILU_SWEEP_L, r, y, z, nrhs, s, nullptr, &sync, false))) return st;
    if ((st = run_sweep(c, BILU_SWEEP_U, y, z, y, nrhs, s, nullptr, &sync, false))) return st;
    // a bounded wait that expired shows in bilu_check and the solvers, as for
    // bilu_apply
    hipLaunchKernelGGL(dev::k_merge_status, dim3(1), dim3(64), 0, s, sync.status, c->d_status);
    CK(hipGetLastError());
    return BILU_OK;
}

bilu_status bilu_apply_point(bilu_ctx* c, const double* r, double* z, hipStream_t s)
{
    if (!c || !r || !z || r == z) return BILU_ERR_ARG;
    if (!c->split_done) return BILU_ERR_STATE;
    return do_apply_point(c, r, z, s, nullptr);
}

bilu_status bilu_apply_transpose(bilu_ctx* c, const double* r, double* z, int nrhs, hipStream_t s)
{
    return do_apply(c, r, z, nrhs, true, s);
}

bilu_status bilu_spmv(bilu_ctx* c, const double* Ax, const double* x, double* y, int nrhs, int transpose,
                      hipStream_t s)
{
    return do_spmv(c, Ax, x, y, nrhs, transpose, s);
}

bilu_status bilu_grad_A(bilu_ctx* c, const double* lam, const double* x, double* dA, hipStream_t s)
{
    if (!c || !lam || !x || !dA) return BILU_ERR_ARG;
    bilu_status st = ensure_device(c);
    if (st) return st;
    const int64_t nA = static_cast<int64_t>(c->h.Aj.size());
    const int bb = c->h.bs * c->h.bs;
    hipLaunchKernelGGL(dev::k_grad_A, dim3(grid_for(nA * bb)), dim3(256), 0, s, nA, c->h.bs, c->d_Arow, c->d_Aj,
                       lam, x, dA);
    CK(hipGetLastError());
    return BILU_OK;
}

bilu_status bilu_tune(bilu_ctx* c, int param, int value)
{
    if (!c) return BILU_ERR_ARG;
    switch (param) {
    case BILU_TUNE_SWEEP_MODE:
        if (value < 0 || value > 2) return BILU_ERR_ARG;
        c->sweep_mode = value;
        return BILU_OK;
    case BILU_TUNE_TILE_ROWS:
        if (value < 0) return BILU_ERR_ARG;
        return set_layout(c, value, c->tile_group_req);
    case BILU_TUNE_TILE_GROUP:
        if (value < 0 || value > kGroupMax) return BILU_ERR_ARG;
        return set_layout(c, c->tile_rows_req, value);
    case BILU_TUNE_BLOCKS:
        if (value < 0 || value > (1 << 20)) return BILU_ERR_ARG;
        c->blocks_override = value;
        return BILU_OK;
    case BILU_TUNE_RHS_TILE:
        if (value != 0 && value != 1 && value != 4 && value != 8) return BILU_ERR_ARG;
        c->rhs_tile = value;
        return BILU_OK;
    case BILU_TUNE_FUSE_SPMV:
        if (value != 0 && value != 1) return BILU_ERR_ARG;
        c->fuse_spmv = value != 0;
        return BILU_OK;
    case BILU_TUNE_HELPER:
        if (value < 0 || value > 2) return BILU_ERR_ARG;
        c->helper = value;
        return BILU_OK;
    case BILU_TUNE_FACTOR:
        if (value < 0 || value > 3) return BILU_ERR_ARG;
        c->factor_mode = value;
        return BILU_OK;
    case BILU_TUNE_SPIN_LIMIT:
        if (value < 0) return BILU_ERR_ARG;
        c->spin_limit = value == 0 ? 1u << 24 : static_cast<unsigned int>(value);
        return BILU_OK;
    case BILU_TUNE_SPLIT_DINV:
        if (value < 0 || value > 2) return BILU_ERR_ARG;
        c->split_dinv = value;
        return BILU_OK;
    case BILU_TUNE_RHS_PAIRS:
        if (value < 0 || value > 2) return BILU_ERR_ARG;
        c->rhs_pairs = value;
        return BILU_OK;
    case BILU_TUNE_SPMV_STREAM:
        if (value < 0 || value > 2) return BILU_ERR_ARG;
        c->spmv_stream = value;
        return BILU_OK;
    case BILU_TUNE_LINE_SWEEP: {
        const int ny = value & 255, nz = value >> 8;
        if (value < 0 || (value != 0 && (ny < 1 || nz < 1 || nz > 255))) return BILU_ERR_ARG;
        if (value == c->line_block) return BILU_OK;
        c->line_block = value;
        free_form(c, kFormLines);
        c->layouts_checked = false;
        for (int w : {static_cast<int>(BILU_SWEEP_L), static_cast<int>(BILU_SWEEP_U)}) {
            if (value > 0 && c->h.sweep[w].built) build_line_layout(c->h, w, c->h.rpc, ny, nz, c->h.lines[w]);
            else c->h.lines[w] = HostTiled{};
        }
        return BILU_OK;
    }
    case BILU_TUNE_TILE_BLOCK: {
        const int ny = value & 255, nz = value >> 8;
        if (value < 0 || (value != 0 && (ny < 1 || nz < 1 || nz > 255))) return BILU_ERR_ARG;
        if (value == c->tile_block) return BILU_OK;
        c->tile_block = value;
        free_form(c, kFormTiled);
        c->layouts_checked = false;
        if (c->tile_rows <= 0) choose_layout(c);
        for (int w = 0; w < 4; ++w)
            if (c->h.sweep[w].built) build_tiled_layout(c, w);
        return BILU_OK;
    }
    }
    return BILU_ERR_ARG;
}

// Times one configuration: median of `reps` applications (after warm-ups).
static bilu_status time_apply(bilu_ctx* c, const double* r, double* z, int R, hipStream_t s, double* us)
{
    constexpr int warm = 2, reps = 5;
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return BILU_ERR_HIP;
    }
    bilu_status st = BILU_OK;
    std::vector<double> t;
    for (int i = 0; i < warm + reps && st == BILU_OK; ++i) {
        if (hipEventRecord(e0, s) != hipSuccess) { st = BILU_ERR_HIP; break; }
        st = do_apply(c, r, z, R, false, s);
        if (st) break;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = BILU_ERR_HIP;
            break;
        }
        if (i >= warm) t.push_back(1e3 * ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    std::sort(t.begin(), t.end());
    *us = t[t.size() / 2];
    return BILU_OK;
}

bilu_status bilu_autotune(bilu_ctx* c, int nrhs, hipStream_t s, bilu_tune_result* out)
{
    if (!c || !out || nrhs < 1 || nrhs > dev::kMaxRhs || c->h.bs > kMaxKernelBs) return BILU_ERR_ARG;
    if (!c->split_done) return BILU_ERR_STATE;
    std::memset(out, 0, sizeof(*out));
    // tile_rows / group: the layout requests (0: by schedule simulation)
    struct Cand {
        int mode, tile_rows, group, rhs_tile, helper;
    };
    std::vector<Cand> cands;
    const Cand before{c->sweep_mode, c->tile_rows_req, c->tile_group_req, c->rhs_tile, c->helper};
    if (nrhs == 1) {
        // the preferred layouts, every group size of the best tile size, and
        // the next single-tile sizes, each with and without helper
        // wavefronts
        auto add = [&](int rows, int group) {
            for (const Cand& k : cands)
                if (k.mode == 2 && k.tile_rows == rows && k.group == group) return;
            cands.push_back({2, rows, group, 0, 2});
            cands.push_back({2, rows, group, 0, 1});
        };
        const auto ranked = rank_tile_layouts(c->h, c->h.rpc, c->lds_max, 0, 0);
        for (size_t i = 0; i < ranked.size() && i < 4; ++i) add(ranked[i].tile_rows, ranked[i].group);
        const int best_rows = ranked.front().tile_rows;
        for (int g = 1; g <= kGroupMax; ++g)
            if (tiled_lds_bytes(best_rows, g, c->h.bs) <= c->lds_max) add(best_rows, g);
        cands.push_back({1, before.tile_rows, before.group, 0, before.helper});
    } else {
        cands.push_back({2, 0, 0, 0, before.helper});
        cands.push_back({2, 0, 1, 0, before.helper});
        for (int rt : {1, 4, 8}) cands.push_back({1, before.tile_rows, before.group, rt, before.helper});
    }
    const size_t n = static_cast<size_t>(c->h.nb) * c->h.bs * nrhs;
    double* r = nullptr;
    double* z = nullptr;
    bilu_status st;
    if ((st = dalloc(c, &r, n)) || (st = dalloc(c, &z, n))) {
        dfree(c, r);
        return st;
    }
    hipLaunchKernelGGL(dev::k_fill_f64, dim3(grid_for(static_cast<int64_t>(n))), dim3(256), 0, s,
                       static_cast<int64_t>(n), r, 1.0);
    auto set = [&](const Cand& k) -> bilu_status {
        bilu_status e;
        if ((e = bilu_tune(c, BILU_TUNE_SWEEP_MODE, k.mode)) || (e = bilu_tune(c, BILU_TUNE_RHS_TILE, k.rhs_tile)) ||
            (e = bilu_tune(c, BILU_TUNE_HELPER, k.helper)))
            return e;
        return k.mode == 2 ? set_layout(c, k.tile_rows, k.group) : BILU_OK;
    };
    double best_us = 1e300;
    Cand best = before;
    // the configuration in force first, as the reference
    double ref_us = 0.0;
    st = time_apply(c, r, z, nrhs, s, &ref_us);
    for (size_t i = 0; i < cands.size() && st == BILU_OK; ++i) {
        double us = 0.0;
        if ((st = set(cands[i])) || (st = time_apply(c, r, z, nrhs, s, &us))) break;
        ++out->candidates;
        if (us < best_us) {
            best_us = us;
            best = cands[i];
        }
    }
    if (st == BILU_OK && ref_us <= best_us) {
        best = before;
        best_us = ref_us;
    }
    const bilu_status st2 = set(best);
    dfree(c, r);
    dfree(c, z);
    if (st) return st;
    if (st2) return st2;
    out->sweep_mode = c->sweep_mode;
    out->tile_rows = c->tile_rows;
    out->tile_group = built_group(c);
    out->rhs_tile = rhs_tile(c, nrhs);
    out->apply_us = best_us;
    out->default_us = ref_us;
    return bilu_check(c, s);
}

bilu_status bilu_timing(bilu_ctx* c, int enable)
{
    if (!c) return BILU_ERR_ARG;
    if (enable) {
        c->ev_used = 0;
        c->ev_marks.clear();
    }
    c->timing = enable != 0;
    // the point view's sweeps are timed with the caller's
    if (c->point) bilu_timing(c->point, enable);
    return BILU_OK;
}

bilu_status bilu_timing_read(bilu_ctx* c, hipStream_t s, bilu_kernel_time* out)
{
    if (!c || !out) return BILU_ERR_ARG;
    for (int k = 0; k < BILU_K_COUNT; ++k) out[k] = bilu_kernel_time{0, 0.0};
    CK(hipStreamSynchronize(s));
    for (const bilu_ctx* t : {static_cast<const bilu_ctx*>(c), static_cast<const bilu_ctx*>(c->point)}) {
        if (!t) continue;
        for (const auto& m : t->ev_marks) {
            float ms = 0.f;
            CK(hipEventElapsedTime(&ms, t->ev_pool[m.second], t->ev_pool[m.second + 1]));
            out[m.first].launches += 1;
            out[m.first].total_ms += ms;
        }
    }
    return BILU_OK;
}

bilu_status bilu_check(bilu_ctx* c, hipStream_t s)
{
    if (!c) return BILU_ERR_ARG;
    if (!c->dev_ready) return BILU_OK;
    if (point_sweep_error(c, s)) return BILU_ERR_TIMEOUT;
    int v = 0;
    CK(hipMemcpyAsync(&v, c->d_status, sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (v) {
        CK(hipMemsetAsync(c->d_status, 0, sizeof(int), s));
        CK(hipStreamSynchronize(s));
        return BILU_ERR_TIMEOUT;
    }
    return BILU_OK;
}

// ----- Krylov ---------------------------------------------------------------
static bilu_status ensure_krylov(bilu_ctx* c, int R, int nvec)
{
    const size_t need = static_cast<size_t>(c->h.nb) * c->h.bs * R * nvec;
    bilu_status st;
    if (c->kv_cap < need) {
        dfree(c, c->d_kv);
        c->d_kv = nullptr;
        c->kv_cap = 0;
        if ((st = dalloc(c, &c->d_kv, need))) return st;
        c->kv_cap = need;
    }
    if (!c->d_part) {
        if ((st = dalloc(c, &c->d_part, static_cast<size_t>(dev::kSlots + 64) * dev::kMaxRhs * dev::kRedBlocks)))
            return st;
        if ((st = dalloc(c, &c->d_state, 1))) return st;
    }
    return BILU_OK;
}

// Host side of the solvers' step loop: pinned state, mapped flags and the
// two events of the one-step-behind exit test.
static bilu_status ensure_step_host(bilu_ctx* c)
{
    if (!c->h_state) {
        void* hp = nullptr;
        if (hipHostMalloc(&hp, sizeof(KState), hipHostMallocDefault) != hipSuccess) return BILU_ERR_ALLOC;
        c->h_state = static_cast<KState*>(hp);
    }
    if (!c->h_flags) {
        void* hp = nullptr;
        if (hipHostMalloc(&hp, 2 * sizeof(int), hipHostMallocMapped) != hipSuccess) return BILU_ERR_ALLOC;
        c->h_flags = static_cast<int*>(hp);
        void* dp = nullptr;
        if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess) return BILU_ERR_HIP;
        c->d_flags = static_cast<int*>(dp);
    }
    for (hipEvent_t& e : c->step_ev)
        if (!e) CK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return BILU_OK;
}

// Right-preconditioned BiCGSTAB on R columns at once, each with its own
// recurrence.  Every decision is taken on the device: the scalar kernels
// freeze a column that breaks down, k_bicg_s_end marks a column whose
// recurrence residual passes for the true-residual test, a gated SpMV
// computes b - A x only when some column is marked, and k_bicg_decide
// either stops the column (true residual passes) or restarts it from the
// true residual.  The host queues steps without waiting: after queuing step
// it, it waits only for step it - 1 and reads the flag that step wrote to
// mapped host memory, so one step is always queued ahead; a step queued
// after every column had stopped is gated off and costs only its launches.
static bilu_status bicgstab(bilu_ctx* c, const double* Ax, const double* b, double* x, int R,
                            const bilu_solve_opts* o, bilu_rhs_info* info, int tr, hipStream_t s)
{
    const int64_t n = static_cast<int64_t>(c->h.nb) * c->h.bs;
    const size_t vb = static_cast<size_t>(n) * R * sizeof(double);
    bilu_status st = ensure_krylov(c, R, 9);
    if (st) return st;
    if ((st = ensure_step_host(c))) return st;
    double* kv = c->d_kv;
    const size_t stride = static_cast<size_t>(n) * R;
    double *r = kv, *rh = kv + stride, *p = kv + 2 * stride, *v = kv + 3 * stride, *ph = kv + 4 * stride;
    double *sv = kv + 5 * stride, *sh = kv + 6 * stride, *t = kv + 7 * stride, *w = kv + 8 * stride;
    double* part = c->d_part;
    KState* S = c->d_state;
    const int* g_active = &S->any_active;
    const int* g_check = &S->any_check;
    const int eg = grid_for(n * R);
    const dim3 rb(dev::kRedBlocks), rt(dev::kThreads);

    CK(hipMemcpyAsync(r, b, vb, hipMemcpyDeviceToDevice, s));
    CK(hipMemcpyAsync(rh, b, vb, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(dev::k_fill_f64, dim3(eg), dim3(256), 0, s, n * R, x, 0.0);
    hipLaunchKernelGGL(dev::k_fill_f64, dim3(eg), dim3(256), 0, s, n * R, p, 0.0);
    hipLaunchKernelGGL(dev::k_fill_f64, dim3(eg), dim3(256), 0, s, n * R, v, 0.0);
    hipLaunchKernelGGL(dev::k_dot, rb, rt, 0, s, n, R, b, b, part, dev::SL_BB, nullptr);
    hipLaunchKernelGGL(dev::k_bicg_init, dim3(R), dim3(64), 0, s, R, part, S, o->rtol);
    hipLaunchKernelGGL(dev::k_bicg_decide, dim3(1), dim3(64), 0, s, R, S, 0, c->d_flags);
    CK(hipGetLastError());
    CK(hipEventRecord(c->step_ev[0], s));

    int it = 0;
    while (it < o->maxit) {
        ++it;
        hipLaunchKernelGGL(dev::k_dot, rb, rt, 0, s, n, R, rh, r, part, dev::SL_RHO, g_active);
        hipLaunchKernelGGL(dev::k_bicg_s_rho, dim3(R), dim3(64), 0, s, R, part, S);
        hipLaunchKernelGGL(dev::k_bicg_p, dim3(eg), dim3(256), 0, s, n, R, r, v, p, S);
        if ((st = do_apply_spmv(c, Ax, p, ph, v, R, tr != 0, s, g_active))) return st;
        hipLaunchKernelGGL(dev::k_dot, rb, rt, 0, s, n, R, rh, v, part, dev::SL_RV, g_active);
        hipLaunchKernelGGL(dev::k_bicg_s_alpha, dim3(R), dim3(64), 0, s, R, part, S);
        hipLaunchKernelGGL(dev::k_bicg_s, rb, rt, 0, s, n, R, r, v, sv, S, part);
        hipLaunchKernelGGL(dev::k_bicg_s_snorm, dim3(R), dim3(64), 0, s, R, part, S);
        if ((st = do_apply_spmv(c, Ax, sv, sh, t, R, tr != 0, s, g_active))) return st;
        hipLaunchKernelGGL(dev::k_dot2, rb, rt, 0, s, n, R, t, sv, part, dev::SL_TS, dev::SL_TT, g_active);
        hipLaunchKernelGGL(dev::k_bicg_s_omega, dim3(R), dim3(64), 0, s, R, part, S);
        hipLaunchKernelGGL(dev::k_bicg_xr, rb, rt, 0, s, n, R, x, r, ph, sh, sv, t, S, part);
        hipLaunchKernelGGL(dev::k_bicg_s_end, dim3(R), dim3(64), 0, s, R, part, S);
        // true residual of the marked columns, then their verdict
        if ((st = do_spmv(c, Ax, x, w, R, tr, s, g_check, false))) return st;
        hipLaunchKernelGGL(dev::k_resid, rb, rt, 0, s, n, R, b, w, part, dev::SL_TRUE, g_check);
        hipLaunchKernelGGL(dev::k_s_true, dim3(R), dim3(64), 0, s, R, part, S, g_check);
        hipLaunchKernelGGL(dev::k_bicg_decide, dim3(1), dim3(64), 0, s, R, S, it, c->d_flags + (it & 1));
        hipLaunchKernelGGL(dev::k_bicg_restart, dim3(eg), dim3(256), 0, s, n, R, w, r, rh, S);
        CK(hipGetLastError());
        CK(hipEventRecord(c->step_ev[it & 1], s));
        // step it - 1 has written its flag once its event has completed
        CK(hipEventSynchronize(c->step_ev[(it - 1) & 1]));
        if (__hip_atomic_load(c->h_flags + ((it - 1) & 1), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) == 0) break;
    }
    // final true residuals for every column
    if ((st = do_spmv(c, Ax, x, w, R, tr, s))) return st;
    hipLaunchKernelGGL(dev::k_resid, rb, rt, 0, s, n, R, b, w, part, dev::SL_TRUE, nullptr);
    hipLaunchKernelGGL(dev::k_s_true, dim3(R), dim3(64), 0, s, R, part, S, nullptr);
    KState& hs = *c->h_state;
    CK(hipMemcpyAsync(&hs, S, sizeof(KState), hipMemcpyDeviceToHost, s));
    int sweep_err = 0;
    CK(hipMemcpyAsync(&sweep_err, c->d_status, sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    int worst = BILU_OK;
    for (int j = 0; j < R; ++j) {
        int stj = hs.status[j];
        if (hs.active[j]) stj = BILU_NOT_CONVERGED;
        info[j].status = stj;
        info[j].iters = hs.done_it[j] >= 0 ? hs.done_it[j] : it;
        info[j].relres = hs.bnorm2[j] > 0 ? std::sqrt(hs.tnorm2[j] / hs.bnorm2[j]) : 0.0;
        info[j].restarts = hs.nrestart[j];
        info[j].reserved = 0;
        if (stj > worst) worst = stj;
    }
    if (point_sweep_error(c, s)) sweep_err = 1;
    if (sweep_err) {
        CK(hipMemsetAsync(c->d_status, 0, sizeof(int), s));
        CK(hipStreamSynchronize(s));
        return BILU_ERR_TIMEOUT;
    }
    return static_cast<bilu_status>(worst);
}

// Restarted right-preconditioned GMRES(m), one right-hand side: Arnoldi with
// modified Gram-Schmidt, the Givens rotations and the small triangular
// solve all on the device, x += M^{-1} V y at the end of each cycle, exit on
// the true residual at the start of a cycle.  Inside a cycle the host
// queues Arnoldi step j and then waits only for step j - 1, whose flag
// (mapped host memory) says whether the cycle goes on; a step queued after
// the cycle stopped is gated off.  One host read per cycle (the true
// residual norm and the cycle's step count).  maxit bounds the Arnoldi
// steps.
static bilu_status gmres(bilu_ctx* c, const double* Ax, const double* b, double* x, const bilu_solve_opts* o,
                         bilu_rhs_info* info, int tr, hipStream_t s)
{
    const int64_t n = static_cast<int64_t>(c->h.nb) * c->h.bs;
    const int m = o->restart;
    bilu_status st = ensure_krylov(c, 1, m + 4);
    if (st) return st;
    if ((st = ensure_step_host(c))) return st;
    double* V = c->d_kv;                                   // (m+1) x n basis
    double* w = V + static_cast<size_t>(m + 1) * n;
    double* z = w + n;
    double* u = z + n;
    // kept in the context across solves: the (m+1) x m Hessenberg matrix
    // (column j contiguous), coef, y, the rotations, g and the cycle flags
    const size_t hneed = static_cast<size_t>(m + 1) * m + 1 + 3 * static_cast<size_t>(m) + (m + 1) + 2;
    if (c->gm_cap < hneed) {
        dfree(c, c->d_gmh);
        c->d_gmh = nullptr;
        c->gm_cap = 0;
        if ((st = dalloc(c, &c->d_gmh, hneed))) return st;
        c->gm_cap = hneed;
    }
    double* dH = c->d_gmh;
    double* coef = dH + static_cast<size_t>(m + 1) * m;
    dev::GmView gv;
    gv.H = dH;
    gv.y = coef + 1;
    gv.cs = gv.y + m;
    gv.sn = gv.cs + m;
    gv.g = gv.sn + m;
    gv.flags = reinterpret_cast<int*>(gv.g + m + 1);
    gv.m = m;
    const int* g_active = gv.flags + dev::GM_ACTIVE;
    double* part = c->d_part;
    const int eg = grid_for(n);
    const dim3 rb(dev::kRedBlocks), rt(dev::kThreads);
    const double tol_abs_factor = o->rtol;
    struct Cycle {
        double beta;
        int flags[dev::GM_NFLAGS];
    };
    Cycle* hc = reinterpret_cast<Cycle*>(c->h_state);      // pinned host memory (KState-sized)
    static_assert(sizeof(Cycle) <= sizeof(KState), "cycle readback fits the pinned state");
    auto fetch_cycle = [&]() -> bilu_status {
        CK(hipMemcpyAsync(&hc->beta, dH, sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipMemcpyAsync(hc->flags, gv.flags, sizeof(hc->flags), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        return BILU_OK;
    };

    hipLaunchKernelGGL(dev::k_fill_f64, dim3(eg), dim3(256), 0, s, n, x, 0.0);
    hipLaunchKernelGGL(dev::k_fill_i32, dim3(1), dim3(64), 0, s, int64_t(dev::GM_NFLAGS), gv.flags, 0);
    hipLaunchKernelGGL(dev::k_dot, rb, rt, 0, s, n, 1, b, b, part, dev::SL_BB, nullptr);
    hipLaunchKernelGGL(dev::k_gm_h, dim3(1), dim3(64), 0, s, part, dev::SL_BB, dH, coef, 1, nullptr);
    if ((st = fetch_cycle())) return st;
    const double bnorm = hc->beta;
    const double tol = tol_abs_factor * bnorm;
    int total = 0, cycles = 0, status = BILU_NOT_CONVERGED;
    double rres = bnorm;
    if (bnorm == 0.0) status = BILU_OK;
    while (status == BILU_NOT_CONVERGED) {
        if ((st = do_spmv(c, Ax, x, w, 1, tr, s))) break;
        hipLaunchKernelGGL(dev::k_resid, rb, rt, 0, s, n, 1, b, w, part, dev::SL_TRUE, nullptr);
        hipLaunchKernelGGL(dev::k_gm_h, dim3(1), dim3(64), 0, s, part, dev::SL_TRUE, dH, coef, 1, nullptr);
        if ((st = fetch_cycle())) break;
        const double beta = hc->beta;
        if (cycles > 0) total += hc->flags[dev::GM_STEPS];
        rres = beta;
        if (cycles > 0 && hc->flags[dev::GM_BREAKDOWN]) { status = BILU_BREAKDOWN; break; }
        if (!std::isfinite(beta)) { status = BILU_NONFINITE; break; }
        if (beta <= tol) { status = BILU_OK; break; }
        if (total >= o->maxit) break;
        const int steps = std::min(m, o->maxit - total);
        hipLaunchKernelGGL(dev::k_gm_scale, dim3(eg), dim3(256), 0, s, n, w, coef, V, nullptr);
        hipLaunchKernelGGL(dev::k_gm_begin, dim3(1), dim3(64), 0, s, gv, steps);
        for (int j = 0; j < steps; ++j) {
            double* vj = V + static_cast<size_t>(j) * n;
            double* hcol = dH + static_cast<size_t>(j) * (m + 1);
            if ((st = do_apply_spmv(c, Ax, vj, z, w, 1, tr != 0, s, g_active))) break;
            hipLaunchKernelGGL(dev::k_gm_mgs, rb, rt, 0, s, n, w, nullptr, coef, V, part, dev::SL_RHO, g_active);
            hipLaunchKernelGGL(dev::k_gm_h, dim3(1), dim3(64), 0, s, part, dev::SL_RHO, hcol, coef, 0, g_active);
            for (int i = 1; i <= j; ++i) {
                hipLaunchKernelGGL(dev::k_gm_mgs, rb, rt, 0, s, n, w, V + static_cast<size_t>(i - 1) * n, coef,
                                   V + static_cast<size_t>(i) * n, part, dev::SL_RHO, g_active);
                hipLaunchKernelGGL(dev::k_gm_h, dim3(1), dim3(64), 0, s, part, dev::SL_RHO, hcol + i, coef, 0,
                                   g_active);
            }
            hipLaunchKernelGGL(dev::k_gm_mgs, rb, rt, 0, s, n, w, vj, coef, nullptr, part, dev::SL_RHO, g_active);
            hipLaunchKernelGGL(dev::k_gm_h, dim3(1), dim3(64), 0, s, part, dev::SL_RHO, hcol + j + 1, coef, 1,
                               g_active);
            hipLaunchKernelGGL(dev::k_gm_scale, dim3(eg), dim3(256), 0, s, n, w, coef, vj + n, g_active);
            hipLaunchKernelGGL(dev::k_gm_givens, dim3(1), dim3(64), 0, s, gv, j, steps, tol, c->d_flags + (j & 1));
            if (hipGetLastError() != hipSuccess) { st = BILU_ERR_HIP; break; }
            if (hipEventRecord(c->step_ev[j & 1], s) != hipSuccess) { st = BILU_ERR_HIP; break; }
            if (j >= 1) {
                // step j - 1 has written its flag once its event has completed
                if (hipEventSynchronize(c->step_ev[(j - 1) & 1]) != hipSuccess) { st = BILU_ERR_HIP; break; }
                if (__hip_atomic_load(c->h_flags + ((j - 1) & 1), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) == 0)
                    break;
            }
        }
        if (st) break;
        hipLaunchKernelGGL(dev::k_gm_solve_y, dim3(1), dim3(64), 0, s, gv);
        hipLaunchKernelGGL(dev::k_gm_combine, dim3(eg), dim3(256), 0, s, n, m, V, gv.y, u,
                           gv.flags + dev::GM_JEND);
        if ((st = do_apply(c, u, z, 1, tr != 0, s))) break;
        hipLaunchKernelGGL(dev::k_axpy1, dim3(eg), dim3(256), 0, s, n, x, z);
        ++cycles;
    }
    int sweep_err = 0;
    if (!st) {
        if (hipMemcpyAsync(&sweep_err, c->d_status, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = BILU_ERR_HIP;
    }
    if (st) return st;
    info[0].status = status;
    info[0].iters = total;
    info[0].relres = bnorm > 0.0 ? rres / bnorm : 0.0;
    info[0].restarts = cycles;
    info[0].reserved = 0;
    if (point_sweep_error(c, s)) sweep_err = 1;
    if (sweep_err) {
        CK(hipMemsetAsync(c->d_status, 0, sizeof(int), s));
        CK(hipStreamSynchronize(s));
        return BILU_ERR_TIMEOUT;
    }
    return static_cast<bilu_status>(status);
}

// Right-preconditioned ORTHOMIN(k), one right-hand side: each iteration
// takes z = M^{-1} r as the new direction (ring slot (it-1) mod (k+1)) with
// q = A z, makes q orthogonal to the A-images of the last k directions
// (k_om_dots, k_om_beta, k_om_update), minimises the residual along it
// (k_om_alpha, k_om_xr) and marks the iteration for the true-residual test
// when the recurrence residual passes (k_om_end); the gated true-residual
// SpMV and k_om_decide stop or restart.  The host queues iteration it and
// waits only for iteration it - 1, as in BiCGSTAB.
static bilu_status orthomin(bilu_ctx* c, const double* Ax, const double* b, double* x, const bilu_solve_opts* o,
                            bilu_rhs_info* info, int tr, hipStream_t s)
{
    const int64_t n = static_cast<int64_t>(c->h.nb) * c->h.bs;
    const int k = o->restart;
    const int K1 = k + 1;
    bilu_status st = ensure_krylov(c, 1, 2 * K1 + 2);
    if (st) return st;
    if ((st = ensure_step_host(c))) return st;
    if (!c->d_om && (st = dalloc(c, &c->d_om, 1))) return st;
    double* P = c->d_kv;
    double* Q = P + static_cast<size_t>(K1) * n;
    double* r = Q + static_cast<size_t>(K1) * n;
    double* w = r + n;
    double* part = c->d_part;
    dev::OmState* S = c->d_om;
    const int* g_active = &S->active;
    const int* g_check = &S->check;
    const int eg = grid_for(n);
    const dim3 rb(dev::kRedBlocks), rt(dev::kThreads);

    CK(hipMemcpyAsync(r, b, static_cast<size_t>(n) * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(dev::k_fill_f64, dim3(eg), dim3(256), 0, s, n, x, 0.0);
    hipLaunchKernelGGL(dev::k_dot, rb, rt, 0, s, n, 1, b, b, part, dev::SL_BB, nullptr);
    hipLaunchKernelGGL(dev::k_om_init, dim3(1), dim3(64), 0, s, part, S, o->rtol);
    hipLaunchKernelGGL(dev::k_om_decide, dim3(1), dim3(64), 0, s, part, S, 0, c->d_flags);
    CK(hipGetLastError());
    CK(hipEventRecord(c->step_ev[0], s));
    int it = 0;
    while (it < o->maxit) {
        ++it;
        const int sl = (it - 1) % K1;
        double* p = P + static_cast<size_t>(sl) * n;
        double* q = Q + static_cast<size_t>(sl) * n;
        if ((st = do_apply(c, r, p, 1, tr != 0, s, g_active)) || (st = do_spmv(c, Ax, p, q, 1, tr, s, g_active)))
            return st;
        hipLaunchKernelGGL(dev::k_om_dots, rb, rt, 0, s, n, Q, sl, K1, S, part);
        hipLaunchKernelGGL(dev::k_om_beta, dim3(1), dim3(64), 0, s, part, S, sl, K1);
        hipLaunchKernelGGL(dev::k_om_update, rb, rt, 0, s, n, P, Q, r, sl, K1, S, part);
        hipLaunchKernelGGL(dev::k_om_alpha, dim3(1), dim3(64), 0, s, part, S, sl);
        hipLaunchKernelGGL(dev::k_om_xr, rb, rt, 0, s, n, x, r, P, Q, sl, S, part);
        hipLaunchKernelGGL(dev::k_om_end, dim3(1), dim3(64), 0, s, part, S, k);
        // true residual when the recurrence residual passes, then the verdict
        if ((st = do_spmv(c, Ax, x, w, 1, tr, s, g_check, false))) return st;
        hipLaunchKernelGGL(dev::k_resid, rb, rt, 0, s, n, 1, b, w, part, dev::SL_TRUE, g_check);
        hipLaunchKernelGGL(dev::k_om_decide, dim3(1), dim3(64), 0, s, part, S, it, c->d_flags + (it & 1));
        hipLaunchKernelGGL(dev::k_om_restart, dim3(eg), dim3(256), 0, s, n, w, r, S);
        CK(hipGetLastError());
        CK(hipEventRecord(c->step_ev[it & 1], s));
        CK(hipEventSynchronize(c->step_ev[(it - 1) & 1]));
        if (__hip_atomic_load(c->h_flags + ((it - 1) & 1), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) == 0) break;
    }
    // final true residual
    if ((st = do_spmv(c, Ax, x, w, 1, tr, s))) return st;
    hipLaunchKernelGGL(dev::k_resid, rb, rt, 0, s, n, 1, b, w, part, dev::SL_TRUE, nullptr);
    hipLaunchKernelGGL(dev::k_om_final, dim3(1), dim3(64), 0, s, part, S);
    static_assert(sizeof(dev::OmState) <= sizeof(KState), "ORTHOMIN state readback fits the pinned state");
    dev::OmState* hs = reinterpret_cast<dev::OmState*>(c->h_state);
    CK(hipMemcpyAsync(hs, S, sizeof(dev::OmState), hipMemcpyDeviceToHost, s));
    int sweep_err = 0;
    CK(hipMemcpyAsync(&sweep_err, c->d_status, sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    int stj = hs->status;
    if (hs->active) stj = BILU_NOT_CONVERGED;
    info[0].status = stj;
    info[0].iters = hs->done_it >= 0 ? hs->done_it : it;
    info[0].relres = hs->bnorm2 > 0 ? std::sqrt(hs->tnorm2 / hs->bnorm2) : 0.0;
    info[0].restarts = hs->nrestart;
    info[0].reserved = 0;
    if (point_sweep_error(c, s)) sweep_err = 1;
    if (sweep_err) {
        CK(hipMemsetAsync(c->d_status, 0, sizeof(int), s));
        CK(hipStreamSynchronize(s));
        return BILU_ERR_TIMEOUT;
    }
    return static_cast<bilu_status>(stj);
}

bilu_status bilu_solve(bilu_ctx* c, const double* Ax, const double* b, double* x, int nrhs,
                       const bilu_solve_opts* o, bilu_rhs_info* info, int transpose, hipStream_t s)
{
    if (!c || !Ax || !b || !x || !o || !info || nrhs < 1 || nrhs > dev::kMaxRhs || b == x) return BILU_ERR_ARG;
    if (!(o->rtol >= 0.0) || o->maxit < 1) return BILU_ERR_ARG;
    if (!c->split_done) return BILU_ERR_STATE;
    if (transpose && !(c->h.flags & BILU_WANT_TRANSPOSE)) return BILU_ERR_STATE;
    if (o->method == BILU_BICGSTAB) return bicgstab(c, Ax, b, x, nrhs, o, info, transpose, s);
    if (o->method == BILU_GMRES) {
        if (nrhs != 1 || o->restart < 1 || o->restart > 1000) return BILU_ERR_ARG;
        return gmres(c, Ax, b, x, o, info, transpose, s);
    }
    if (o->method == BILU_ORTHOMIN) {
        if (nrhs != 1 || o->restart < 0 || o->restart > dev::kOmMax) return BILU_ERR_ARG;
        return orthomin(c, Ax, b, x, o, info, transpose, s);
    }
    return BILU_ERR_ARG;
}

void bilu_destroy(bilu_ctx* c)
{
    if (!c) return;
    if (c->point) bilu_destroy(c->point);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->h_state) (void)hipHostFree(c->h_state);
    if (c->h_flags) (void)hipHostFree(c->h_flags);
    for (hipEvent_t e : c->step_ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

const char* bilu_status_string(int s)
{
    switch (s) {
    case BILU_OK: return "ok";
    case BILU_ERR_ARG: return "invalid argument";
    case BILU_ERR_ALLOC: return "allocation failed";
    case BILU_ERR_HIP: return "HIP runtime error";
    case BILU_ERR_MISSING_DIAG: return "a block row has no diagonal block";
    case BILU_ERR_PATTERN: return "unsorted, duplicate or out-of-range block columns";
    case BILU_ERR_TIMEOUT: return "a sweep's bounded wait expired";
    case BILU_ERR_STATE: return "call order violated";
    case BILU_SINGULAR_PIVOT: return "singular or non-finite pivot block";
    case BILU_NOT_CONVERGED: return "not converged";
    case BILU_BREAKDOWN: return "Krylov breakdown";
    case BILU_NONFINITE: return "non-finite value in the iteration";
    }
    return "unknown status";
}

}  // extern "C"

// Batches of independent systems: part of this translation unit.
#include "batch_api.inc"
