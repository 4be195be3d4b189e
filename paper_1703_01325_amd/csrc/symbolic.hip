// Symbolic phase on the device: the ILU(k) pattern P with the level of fill
// of every kept entry (Algorithm 3 with Eq 1-2) and the level sets of the
// four sweeps (Eq 4).  The results are the ones the host analysis computes.
//
// Pattern.  Eq 1-2 take the levels of row i from the finished rows p < i,
// one row after another.  The same levels have a per-row characterisation
// (the fill-path theorem of Hysom and Pothen, 2001): (i, j) is kept with
// level l exactly when the shortest path i -> ... -> j in the graph of A
// (edge u -> v for every stored block (u, v)) whose inner vertices are all
// below min(i, j) has l + 1 edges.  Every row is then independent of the
// others.  One wavefront takes a row and runs k + 1 rounds of a
// Bellman-Ford search in the (min, max) semiring: M(v) is the smallest
// possible largest inner vertex over the paths i -> v of at most L edges
// whose inner vertices lie below i; a round extends by one edge the paths
// ending in the vertices u < i whose M dropped in the round before
// (M(v) <- min(M(v), max(M(u), u))), and v is kept with level L - 1 in the
// first round where M(v) < min(i, v).  The visited vertices live in a hash
// table in LDS (kHash slots; a row that reaches more than kHashFill
// distinct vertices is refused).  A count pass sizes the rows, a scan gives
// the row pointers and a write pass repeats the search and emits each row in
// ascending column order (rank of each kept column among the row's).
//
// Level sets.  The level of a row is one more than the deepest row it reads
// (0 if none).  A persistent kernel takes 64 rows at a time, in sweep order,
// from a ticket; a lane polls the levels of the rows its row reads (-1 until
// published, read with device-coherent loads) and publishes its own once all
// are there.  Every row read lies earlier in sweep order, so the rows held
// by running wavefronts always include one that can finish and the launch
// drains.  The transposed sweeps read the columns of P, gathered into lists
// per column first.  level_rows is a stable radix sort of the rows by level
// (rows ascending inside a level), level_ptr the first position of each
// level.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "bilu.h"
#include "bilu_internal.h"

namespace {

constexpr int kHash = 1024;          // hash slots per row search
constexpr int kHashFill = 768;       // distinct vertices a row search may reach
constexpr unsigned short kKept = 0x8000u;
constexpr unsigned int kSpinLimit = 1u << 20;

// status bits of the symbolic kernels
constexpr int kStPattern = 1;        // unsorted / duplicate / out-of-range column
constexpr int kStDiag = 2;           // a row without its diagonal block
constexpr int kStTable = 4;          // a row search outgrew the hash table
constexpr int kStTimeout = 8;        // a level wait expired

__global__ void k_check_pattern(int nb, const int32_t* __restrict__ Ap, const int32_t* __restrict__ Aj,
                                int* status)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) {
        const int e0 = Ap[i], e1 = Ap[i + 1];
        if (e1 < e0) {
            atomicOr(status, kStPattern);
            continue;
        }
        bool diag = false;
        int prev = -1;
        for (int e = e0; e < e1; ++e) {
            const int j = Aj[e];
            if (j <= prev || j >= nb) {
                atomicOr(status, kStPattern);
                break;
            }
            diag |= (j == i);
            prev = j;
        }
        if (!diag) atomicOr(status, kStDiag);
    }
}

__global__ void k_check_ptr(int nb, const int32_t* __restrict__ Ap, int* status)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && Ap[0] != 0) atomicOr(status, kStPattern);
}

struct RowTable {
    int key[kHash];              // vertex, -1 empty
    int mval[kHash];             // M after the last round
    int mnext[kHash];            // running minimum of the candidates
    unsigned short info[kHash];  // kKept | level
    int list[kHash];             // frontier slots / kept slots
    int nlist;
    int nused;
    int over;
};

__device__ __forceinline__ int table_slot(RowTable& t, int v)
{
    unsigned int h = (static_cast<unsigned int>(v) * 2654435761u) >> 22;   // 10 bits: kHash
    for (int probe = 0; probe < kHash; ++probe) {
        const int old = atomicCAS(&t.key[h], -1, v);
        if (old == v) return static_cast<int>(h);
        if (old == -1) {
            if (atomicAdd(&t.nused, 1) >= kHashFill) t.over = 1;
            return static_cast<int>(h);
        }
        h = (h + 1) & (kHash - 1);
    }
    t.over = 1;
    return -1;
}

// One wavefront per row.  WRITE = false: cnt[i] = kept entries of row i;
// WRITE = true: row i written at Pp[i] in ascending columns.
template <bool WRITE>
__global__ __launch_bounds__(64) void k_sym_rows(int nb, const int32_t* __restrict__ Ap,
                                                 const int32_t* __restrict__ Aj, int k, int32_t* __restrict__ cnt,
                                                 const int32_t* __restrict__ Pp, int32_t* __restrict__ Pj,
                                                 int32_t* __restrict__ Plev, int* status)
{
    __shared__ RowTable t;
    const int lane = threadIdx.x;
    for (int i = blockIdx.x; i < nb; i += gridDim.x) {
        __syncthreads();
        for (int s = lane; s < kHash; s += 64) {
            t.key[s] = -1;
            t.mval[s] = INT_MAX;
            t.mnext[s] = INT_MAX;
            t.info[s] = 0;
        }
        if (lane == 0) {
            t.nlist = 0;
            t.nused = 0;
            t.over = 0;
        }
        __syncthreads();
        // row i of A: level 0, no inner vertex (M = -1)
        for (int e = Ap[i] + lane; e < Ap[i + 1]; e += 64) {
            const int v = Aj[e];
            const int s = table_slot(t, v);
            if (s < 0) continue;
            t.mval[s] = -1;
            t.mnext[s] = -1;
            t.info[s] = kKept;
            if (v < i) t.list[atomicAdd(&t.nlist, 1)] = s;
        }
        __syncthreads();
        for (int L = 2; L <= k + 1; ++L) {
            const int nf = t.nlist;
            if (nf == 0 || t.over) break;
            // extend the paths ending in the frontier by one edge of A
            for (int f = lane; f < nf; f += 64) {
                const int su = t.list[f];
                const int u = t.key[su];
                const int mu = max(t.mval[su], u);
                for (int e = Ap[u]; e < Ap[u + 1]; ++e) {
                    const int s = table_slot(t, Aj[e]);
                    if (s >= 0) atomicMin(&t.mnext[s], mu);
                }
            }
            __syncthreads();
            if (lane == 0) t.nlist = 0;
            __syncthreads();
            // fold the round in; the next frontier: vertices below i whose M dropped
            for (int s = lane; s < kHash; s += 64) {
                const int v = t.key[s];
                if (v >= 0 && t.mnext[s] < t.mval[s]) {
                    const int m = t.mnext[s];
                    t.mval[s] = m;
                    if (!(t.info[s] & kKept) && m < min(i, v)) t.info[s] = static_cast<unsigned short>(kKept | (L - 1));
                    if (v < i) t.list[atomicAdd(&t.nlist, 1)] = s;
                }
            }
            __syncthreads();
        }
        if (t.over) {
            if (lane == 0) atomicOr(status, kStTable);
            continue;
        }
        __syncthreads();
        if (lane == 0) t.nlist = 0;
        __syncthreads();
        // the kept entries: columns into mnext[], levels into mval[]
        for (int s = lane; s < kHash; s += 64) {
            if (t.key[s] >= 0 && (t.info[s] & kKept)) {
                const int q = atomicAdd(&t.nlist, 1);
                t.mnext[q] = t.key[s];
                t.mval[q] = t.info[s] & 0xff;
            }
        }
        __syncthreads();
        const int nk = t.nlist;
        if (!WRITE) {
            if (lane == 0) cnt[i] = nk;
            continue;
        }
        const int base = Pp[i];
        for (int q = lane; q < nk; q += 64) {
            const int col = t.mnext[q];
            int rank = 0;
            for (int f = 0; f < nk; ++f) rank += t.mnext[f] < col;
            Pj[base + rank] = col;
            Plev[base + rank] = t.mval[q];
        }
    }
}

__global__ void k_narrow_ptr(int n1, const int64_t* __restrict__ in, int32_t* __restrict__ out)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n1; i += gridDim.x * blockDim.x)
        out[i] = static_cast<int32_t>(in[i]);
}

__device__ __forceinline__ int coherent_load_i(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void coherent_store_i(int* p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Level of every row (Eq 4) for one sweep.  Row r reads the rows idx[e],
// e in [ptr[r], ptr[r+1]) that pass the filter: mode 0 below r, mode 1
// above r, mode 2 all.  forward: sweep order is ascending rows.  A lane
// keeps a cursor into its row's list and the deepest level seen so far, so
// a dependency found published is never read again; a dependency on a row
// of the same wavefront is read from LDS, where the wavefront keeps its
// rows' levels, so chains inside the wavefront advance without a round
// trip through memory.  Global polls sleep between rounds only when no lane
// of the wavefront made progress.
__global__ __launch_bounds__(256) void k_levels(int nb, const int32_t* __restrict__ ptr,
                                                const int32_t* __restrict__ idx, int mode, int forward, int* lvl,
                                                unsigned int* ticket, int* status)
{
    __shared__ int wl[4][64];
    const int lane = threadIdx.x & 63;
    int* mine = wl[threadIdx.x >> 6];
    for (;;) {
        unsigned int tk = 0;
        if (lane == 0) tk = atomicAdd(ticket, 1u);
        tk = __shfl(tk, 0);
        if (static_cast<int64_t>(tk) * 64 >= nb) break;
        const int pos0 = static_cast<int>(tk) * 64;
        const int pos = pos0 + lane;
        const int row = pos < nb ? (forward ? pos : nb - 1 - pos) : -1;
        bool done = row < 0;
        mine[lane] = -1;
        __builtin_amdgcn_wave_barrier();
        int e = done ? 0 : ptr[row];
        const int e1 = done ? 0 : ptr[row + 1];
        int best = -1;
        // Advances the lane's cursor past every dependency found published;
        // with allow_global false only rows of this wavefront are read (LDS)
        // and a dependency on another wavefront's row stops the cursor.
        auto advance = [&](bool allow_global) {
            bool moved = false;
            if (done) return false;
            bool blocked = false;
            while (!blocked && e < e1) {
                int lv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = e + u < e1 ? idx[e + u] : row;
                    const bool use = mode == 2 ? (e + u < e1) : mode == 0 ? (j < row) : (j > row);
                    const int pj = forward ? j : nb - 1 - j;
                    const bool local = pj >= pos0 && pj < pos0 + 64;
                    lv[u] = !use ? INT_MIN : local ? mine[pj - pos0] : allow_global ? coherent_load_i(lvl + j) : -1;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (!blocked && e < e1) {
                        if (lv[u] == -1) {
                            blocked = true;
                        } else {
                            best = max(best, lv[u]);
                            ++e;
                            moved = true;
                        }
                    }
                }
            }
            if (!blocked) {
                mine[lane] = best + 1;
                coherent_store_i(lvl + row, best + 1);
                done = true;
                moved = true;
            }
            return moved;
        };
        unsigned int spins = 0;
        while (!__all(done)) {
            bool moved = advance(true);
            // chains inside the wavefront: LDS only, until nothing moves
            for (;;) {
                __builtin_amdgcn_wave_barrier();
                asm volatile("" ::: "memory");
                if (!__any(advance(false))) break;
                moved = true;
            }
            if (!__any(moved) && !__all(done)) {
                if (++spins > kSpinLimit) {
                    atomicOr(status, kStTimeout);
                    return;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
    }
}

// Column lists of the transposed sweeps: entry (i, j) of P with j > i
// (upper = 1: U'^T, row j reads row i) or j < i (upper = 0: L^T, row j
// reads row i) adds i to the list of j.
__global__ void k_col_count(int nb, const int32_t* __restrict__ Pp, const int32_t* __restrict__ Pj, int upper,
                            int32_t* cnt)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x)
        for (int e = Pp[i]; e < Pp[i + 1]; ++e) {
            const int j = Pj[e];
            if (upper ? j > i : j < i) atomicAdd(cnt + j, 1);
        }
}

__global__ void k_col_fill(int nb, const int32_t* __restrict__ Pp, const int32_t* __restrict__ Pj, int upper,
                           int32_t* cursor, int32_t* __restrict__ cidx)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x)
        for (int e = Pp[i]; e < Pp[i + 1]; ++e) {
            const int j = Pj[e];
            if (upper ? j > i : j < i) cidx[atomicAdd(cursor + j, 1)] = i;
        }
}

__global__ void k_iota_max(int nb, const int32_t* __restrict__ lvl, int32_t* __restrict__ rows, int* nlev)
{
    int m = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) {
        rows[i] = i;
        m = max(m, lvl[i] + 1);
    }
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) atomicMax(nlev, m);
}

// level_ptr[l] = first position of the sorted keys with key >= l.
__global__ void k_level_ptr(int nb, const int32_t* __restrict__ keys, int nlev, int32_t* __restrict__ level_ptr)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p <= nb; p += gridDim.x * blockDim.x) {
        const int lo = p == 0 ? -1 : keys[p - 1];
        const int hi = p == nb ? nlev : keys[p];
        for (int l = lo + 1; l <= hi && l <= nlev; ++l) level_ptr[l] = p;
    }
}

// Device scratch released on every exit path.
struct Scratch {
    std::vector<void*> ptrs;
    ~Scratch()
    {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    T* get(size_t n)
    {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return static_cast<T*>(p);
    }
};

int grid_for(int64_t n, int threads, int cap = 4096)
{
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((n + threads - 1) / threads, cap)));
}

int rows_grid(int nb) { return std::min(nb, 65536); }

bilu_status status_to_error(int st)
{
    if (st & kStTimeout) return BILU_ERR_TIMEOUT;
    if (st & kStPattern) return BILU_ERR_PATTERN;
    if (st & kStDiag) return BILU_ERR_MISSING_DIAG;
    if (st & kStTable) return BILU_ERR_ALLOC;
    return BILU_OK;
}

#define CKH(call)                                       \
    do {                                                \
        if ((call) != hipSuccess) return BILU_ERR_HIP; \
    } while (0)

// Checks the pattern, sizes the rows and writes the row pointers; *nnzb
// receives the entry count.
bilu_status sym_count(int nb, const int32_t* Ap, const int32_t* Aj, int k, int32_t* Pp, int64_t* nnzb, hipStream_t s)
{
    Scratch sc;
    int* d_status = sc.get<int>(1);
    int32_t* cnt = sc.get<int32_t>(static_cast<size_t>(nb) + 1);
    int64_t* ptr64 = sc.get<int64_t>(static_cast<size_t>(nb) + 1);
    if (!d_status || !cnt || !ptr64) return BILU_ERR_ALLOC;
    CKH(hipMemsetAsync(d_status, 0, sizeof(int), s));
    CKH(hipMemsetAsync(cnt + nb, 0, sizeof(int32_t), s));
    k_check_ptr<<<1, 64, 0, s>>>(nb, Ap, d_status);
    k_check_pattern<<<grid_for(nb, 256), 256, 0, s>>>(nb, Ap, Aj, d_status);
    int h_status = 0;
    CKH(hipMemcpyAsync(&h_status, d_status, sizeof(int), hipMemcpyDeviceToHost, s));
    CKH(hipStreamSynchronize(s));
    if (h_status) return status_to_error(h_status);
    k_sym_rows<false><<<rows_grid(nb), 64, 0, s>>>(nb, Ap, Aj, k, cnt, nullptr, nullptr, nullptr, d_status);
    size_t tmp_bytes = 0;
    if (rocprim::exclusive_scan(nullptr, tmp_bytes, cnt, ptr64, int64_t(0), static_cast<size_t>(nb) + 1,
                                rocprim::plus<int64_t>(), s) != hipSuccess)
        return BILU_ERR_HIP;
    void* tmp = sc.get<unsigned char>(tmp_bytes);
    if (!tmp) return BILU_ERR_ALLOC;
    if (rocprim::exclusive_scan(tmp, tmp_bytes, cnt, ptr64, int64_t(0), static_cast<size_t>(nb) + 1,
                                rocprim::plus<int64_t>(), s) != hipSuccess)
        return BILU_ERR_HIP;
    int64_t total = 0;
    CKH(hipMemcpyAsync(&total, ptr64 + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CKH(hipMemcpyAsync(&h_status, d_status, sizeof(int), hipMemcpyDeviceToHost, s));
    CKH(hipStreamSynchronize(s));
    if (h_status) return status_to_error(h_status);
    if (total > INT32_MAX) return BILU_ERR_ALLOC;
    k_narrow_ptr<<<grid_for(nb + 1, 256), 256, 0, s>>>(nb + 1, ptr64, Pp);
    CKH(hipStreamSynchronize(s));
    *nnzb = total;
    return BILU_OK;
}

// Writes the rows at the pointers sym_count produced.
bilu_status sym_write(int nb, const int32_t* Ap, const int32_t* Aj, int k, const int32_t* Pp, int32_t* Pj,
                      int32_t* Plev, hipStream_t s)
{
    Scratch sc;
    int* d_status = sc.get<int>(1);
    if (!d_status) return BILU_ERR_ALLOC;
    CKH(hipMemsetAsync(d_status, 0, sizeof(int), s));
    k_sym_rows<true><<<rows_grid(nb), 64, 0, s>>>(nb, Ap, Aj, k, nullptr, Pp, Pj, Plev, d_status);
    int h_status = 0;
    CKH(hipMemcpyAsync(&h_status, d_status, sizeof(int), hipMemcpyDeviceToHost, s));
    CKH(hipStreamSynchronize(s));
    return status_to_error(h_status);
}

bilu_status levels_impl(int nb, const int32_t* Pp, const int32_t* Pj, int sweep, int32_t* lvl, int32_t* level_ptr,
                        int32_t* level_rows, int* nlev, hipStream_t s)
{
    Scratch sc;
    int* d_small = sc.get<int>(4);   // status, nlev, ticket
    if (!d_small) return BILU_ERR_ALLOC;
    CKH(hipMemsetAsync(d_small, 0, 4 * sizeof(int), s));
    CKH(hipMemsetAsync(lvl, 0xff, static_cast<size_t>(nb) * sizeof(int32_t), s));
    const int32_t* ptr = Pp;
    const int32_t* idx = Pj;
    int mode = 0;
    const bool forward = (sweep == BILU_SWEEP_L || sweep == BILU_SWEEP_UT);
    if (sweep == BILU_SWEEP_U) {
        mode = 1;
    } else if (sweep == BILU_SWEEP_UT || sweep == BILU_SWEEP_LT) {
        const int upper = sweep == BILU_SWEEP_UT;
        int32_t* ccnt = sc.get<int32_t>(static_cast<size_t>(nb) + 1);
        int64_t* cptr64 = sc.get<int64_t>(static_cast<size_t>(nb) + 1);
        int32_t* cptr = sc.get<int32_t>(static_cast<size_t>(nb) + 1);
        int32_t* cursor = sc.get<int32_t>(static_cast<size_t>(nb) + 1);
        if (!ccnt || !cptr64 || !cptr || !cursor) return BILU_ERR_ALLOC;
        CKH(hipMemsetAsync(ccnt, 0, (static_cast<size_t>(nb) + 1) * sizeof(int32_t), s));
        k_col_count<<<grid_for(nb, 256), 256, 0, s>>>(nb, Pp, Pj, upper, ccnt);
        size_t tmp_bytes = 0;
        if (rocprim::exclusive_scan(nullptr, tmp_bytes, ccnt, cptr64, int64_t(0), static_cast<size_t>(nb) + 1,
                                    rocprim::plus<int64_t>(), s) != hipSuccess)
            return BILU_ERR_HIP;
        void* tmp = sc.get<unsigned char>(tmp_bytes);
        if (!tmp) return BILU_ERR_ALLOC;
        if (rocprim::exclusive_scan(tmp, tmp_bytes, ccnt, cptr64, int64_t(0), static_cast<size_t>(nb) + 1,
                                    rocprim::plus<int64_t>(), s) != hipSuccess)
            return BILU_ERR_HIP;
        int64_t total = 0;
        CKH(hipMemcpyAsync(&total, cptr64 + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
        CKH(hipStreamSynchronize(s));
        int32_t* cidx = sc.get<int32_t>(static_cast<size_t>(total));
        if (!cidx) return BILU_ERR_ALLOC;
        k_narrow_ptr<<<grid_for(nb + 1, 256), 256, 0, s>>>(nb + 1, cptr64, cptr);
        CKH(hipMemcpyAsync(cursor, cptr, (static_cast<size_t>(nb) + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        k_col_fill<<<grid_for(nb, 256), 256, 0, s>>>(nb, Pp, Pj, upper, cursor, cidx);
        ptr = cptr;
        idx = cidx;
        mode = 2;
    }
    // persistent: at most as many wavefronts as there are row groups
    const int groups = static_cast<int>((static_cast<int64_t>(nb) + 63) / 64);
    const int wg = std::max(1, std::min((groups + 3) / 4, 512));
    k_levels<<<wg, 256, 0, s>>>(nb, ptr, idx, mode, forward ? 1 : 0, lvl,
                                reinterpret_cast<unsigned int*>(d_small + 2), d_small);
    int32_t* rows_in = sc.get<int32_t>(static_cast<size_t>(nb));
    int32_t* keys_out = sc.get<int32_t>(static_cast<size_t>(nb));
    if (!rows_in || !keys_out) return BILU_ERR_ALLOC;
    k_iota_max<<<grid_for(nb, 256, 1024), 256, 0, s>>>(nb, lvl, rows_in, d_small + 1);
    int h_small[2] = {0, 0};
    CKH(hipMemcpyAsync(h_small, d_small, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    CKH(hipStreamSynchronize(s));
    if (h_small[0]) return status_to_error(h_small[0]);
    const int nl = h_small[1];
    int bits = 1;
    while (bits < 31 && (1 << bits) < nl) ++bits;
    size_t tmp_bytes = 0;
    const unsigned int* kin = reinterpret_cast<const unsigned int*>(lvl);
    unsigned int* kout = reinterpret_cast<unsigned int*>(keys_out);
    if (rocprim::radix_sort_pairs(nullptr, tmp_bytes, kin, kout, rows_in, level_rows, static_cast<unsigned int>(nb),
                                  0, bits, s) != hipSuccess)
        return BILU_ERR_HIP;
    void* tmp = sc.get<unsigned char>(tmp_bytes);
    if (!tmp) return BILU_ERR_ALLOC;
    if (rocprim::radix_sort_pairs(tmp, tmp_bytes, kin, kout, rows_in, level_rows, static_cast<unsigned int>(nb), 0,
                                  bits, s) != hipSuccess)
        return BILU_ERR_HIP;
    k_level_ptr<<<grid_for(nb + 1, 256), 256, 0, s>>>(nb, keys_out, nl, level_ptr);
    CKH(hipStreamSynchronize(s));
    *nlev = nl;
    return BILU_OK;
}

}  // namespace

namespace bilu {

// Host-vector form used by bilu_analyze with BILU_DEVICE_SYMBOLIC: copies the
// pattern to the current device, runs the symbolic phase and the requested
// level sets there and copies the results back.
int device_analysis(int nb, const int32_t* Ap, const int32_t* Aj, int k, int nsweeps, std::vector<int32_t>& Pp,
                    std::vector<int32_t>& Pj, std::vector<int32_t>& Plev, std::vector<int32_t> (&lvl)[4])
{
    Scratch sc;
    hipStream_t s = nullptr;
    const int64_t nA = Ap[nb];
    int32_t* dAp = sc.get<int32_t>(static_cast<size_t>(nb) + 1);
    int32_t* dAj = sc.get<int32_t>(static_cast<size_t>(nA));
    int32_t* dPp = sc.get<int32_t>(static_cast<size_t>(nb) + 1);
    if (!dAp || !dAj || !dPp) return BILU_ERR_ALLOC;
    CKH(hipMemcpy(dAp, Ap, (static_cast<size_t>(nb) + 1) * sizeof(int32_t), hipMemcpyHostToDevice));
    CKH(hipMemcpy(dAj, Aj, static_cast<size_t>(nA) * sizeof(int32_t), hipMemcpyHostToDevice));
    int64_t nnz = 0;
    bilu_status st = sym_count(nb, dAp, dAj, k, dPp, &nnz, s);
    if (st != BILU_OK) return st;
    int32_t* dPj = sc.get<int32_t>(static_cast<size_t>(nnz));
    int32_t* dPl = sc.get<int32_t>(static_cast<size_t>(nnz));
    if (!dPj || !dPl) return BILU_ERR_ALLOC;
    st = sym_write(nb, dAp, dAj, k, dPp, dPj, dPl, s);
    if (st != BILU_OK) return st;
    Pp.resize(static_cast<size_t>(nb) + 1);
    Pj.resize(static_cast<size_t>(nnz));
    Plev.resize(static_cast<size_t>(nnz));
    CKH(hipMemcpy(Pp.data(), dPp, Pp.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    CKH(hipMemcpy(Pj.data(), dPj, Pj.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    CKH(hipMemcpy(Plev.data(), dPl, Plev.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    int32_t* dl = sc.get<int32_t>(static_cast<size_t>(nb));
    int32_t* dptr = sc.get<int32_t>(static_cast<size_t>(nb) + 1);
    int32_t* drows = sc.get<int32_t>(static_cast<size_t>(nb));
    if (!dl || !dptr || !drows) return BILU_ERR_ALLOC;
    for (int w = 0; w < 4; ++w) {
        lvl[w].clear();
        if (w >= nsweeps) continue;
        int nl = 0;
        st = levels_impl(nb, dPp, dPj, w, dl, dptr, drows, &nl, s);
        if (st != BILU_OK) return st;
        lvl[w].resize(static_cast<size_t>(nb));
        CKH(hipMemcpy(lvl[w].data(), dl, static_cast<size_t>(nb) * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    return BILU_OK;
}

}  // namespace bilu

extern "C" {

bilu_status bilu_symbolic_device(int nb, const int32_t* Ap, const int32_t* Aj, int k, int32_t* Pp, int32_t* Pj,
                                 int32_t* lev, int64_t cap, int64_t* nnzb, void* stream)
{
    if (nb < 1 || k < 0 || k > 250 || !Ap || !Aj || !Pp || !nnzb || cap < 0) return BILU_ERR_ARG;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const bilu_status st = sym_count(nb, Ap, Aj, k, Pp, nnzb, s);
    if (st != BILU_OK) return st;
    if (!Pj && !lev && cap == 0) return BILU_OK;   // size query
    if (!Pj || !lev || cap < *nnzb) return BILU_ERR_ARG;
    return sym_write(nb, Ap, Aj, k, Pp, Pj, lev, s);
}

bilu_status bilu_levels_device(int nb, const int32_t* Pp, const int32_t* Pj, int sweep, int32_t* lvl,
                               int32_t* level_ptr, int32_t* level_rows, int* nlev, void* stream)
{
    if (nb < 1 || !Pp || !Pj || !lvl || !level_ptr || !level_rows || !nlev || sweep < 0 || sweep > 3)
        return BILU_ERR_ARG;
    return levels_impl(nb, Pp, Pj, sweep, lvl, level_ptr, level_rows, nlev, static_cast<hipStream_t>(stream));
}

}  // extern "C"
