// Host analysis: pattern validation, symbolic ILU(k), level sets and the
// chunked sweep layouts the GPU kernels stream.  Integer work only.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <numeric>

#include "bilu_internal.h"

namespace bilu {

int validate_pattern(int nb, const int32_t* Ap, const int32_t* Aj)
{
    if (Ap[0] != 0) return BILU_ERR_PATTERN;
    for (int i = 0; i < nb; ++i) {
        if (Ap[i + 1] < Ap[i]) return BILU_ERR_PATTERN;
        bool diag = false;
        for (int32_t e = Ap[i]; e < Ap[i + 1]; ++e) {
            int32_t j = Aj[e];
            if (j < 0 || j >= nb) return BILU_ERR_PATTERN;
            if (e > Ap[i] && j <= Aj[e - 1]) return BILU_ERR_PATTERN;
            diag |= (j == i);
        }
        if (!diag) return BILU_ERR_MISSING_DIAG;
    }
    return BILU_OK;
}

// Symbolic ILU(k) (Algorithm 3 with the level rule of Eq 1-2) on the
// point-wise view of the block pattern: Ap/Aj serve directly as the
// structure of the abstract point matrix (Section 2.3).
//
// Row i is held as a sorted singly linked list threaded through next[]
// (node nb is the head), with the current level of each listed column in
// lev[].  The list is walked in column order; at every column p < i whose
// level is <= k the strictly upper part of the finished row p (columns
// j > p, each with its own level) is merged into the list with level
// lev(i,p) + lev(p,j) + 1, keeping the minimum for columns already listed.
// Candidates above k are never inserted: they could not be used as pivots
// and, by the min rule, a later candidate <= k gives the same final level.
int symbolic_iluk(int nb, const int32_t* Ap, const int32_t* Aj, int k, std::vector<int32_t>& Pp,
                  std::vector<int32_t>& Pj, std::vector<int32_t>& Plev)
{
    constexpr int32_t kEnd = -1;
    const int32_t head = nb;
    std::vector<int32_t> next(static_cast<size_t>(nb) + 1, kEnd);
    std::vector<int32_t> lev(static_cast<size_t>(nb), 0);
    std::vector<int32_t> diag(static_cast<size_t>(nb), 0);
    Pp.assign(1, 0);
    Pj.clear();
    Plev.clear();
    Pj.reserve(static_cast<size_t>(Ap[nb]) * (k > 0 ? 2 : 1));
    Plev.reserve(Pj.capacity());
    for (int32_t i = 0; i < nb; ++i) {
        int32_t tail = head;
        for (int32_t e = Ap[i]; e < Ap[i + 1]; ++e) {
            next[tail] = Aj[e];
            tail = Aj[e];
            lev[tail] = 0;
        }
        next[tail] = kEnd;
        for (int32_t p = next[head]; p != kEnd && p < i; p = next[p]) {
            const int32_t lip = lev[p];
            if (lip > k) continue;
            int32_t at = p;  // list node after which the next column goes
            for (int32_t g = diag[p] + 1; g < Pp[p + 1]; ++g) {
                const int32_t j = Pj[g];
                const int32_t cand = lip + Plev[g] + 1;
                if (cand > k) continue;
                while (next[at] != kEnd && next[at] < j) at = next[at];
                if (next[at] == j) {
                    if (cand < lev[j]) lev[j] = cand;
                } else {
                    next[j] = next[at];
                    next[at] = j;
                    lev[j] = cand;
                }
                at = j;
            }
        }
        for (int32_t j = next[head]; j != kEnd; j = next[j]) {
            if (j == i) diag[i] = static_cast<int32_t>(Pj.size());
            Pj.push_back(j);
            Plev.push_back(lev[j]);
        }
        Pp.push_back(static_cast<int32_t>(Pj.size()));
        if (Pj.size() > static_cast<size_t>(INT32_MAX) - static_cast<size_t>(nb)) return BILU_ERR_ALLOC;
    }
    return BILU_OK;
}

// 0-based level of every row for one sweep (Eq 4: one more than the deepest
// row it reads, 0 for a row that reads none).  Returns the level count.
int sweep_levels(int nb, const std::vector<int32_t>& Pp, const std::vector<int32_t>& Pj, int which,
                 std::vector<int32_t>& lvl)
{
    lvl.assign(static_cast<size_t>(nb), 0);
    switch (which) {
    case BILU_SWEEP_L:   // row i reads y_j, j < i
        for (int32_t i = 0; i < nb; ++i)
            for (int32_t e = Pp[i]; e < Pp[i + 1] && Pj[e] < i; ++e)
                lvl[i] = std::max(lvl[i], lvl[Pj[e]] + 1);
        break;
    case BILU_SWEEP_U:   // row i reads x_j, j > i
        for (int32_t i = nb - 1; i >= 0; --i)
            for (int32_t e = Pp[i + 1] - 1; e >= Pp[i] && Pj[e] > i; --e)
                lvl[i] = std::max(lvl[i], lvl[Pj[e]] + 1);
        break;
    case BILU_SWEEP_UT:  // row j of U'^T reads w_i for (i, j) in P, i < j
        for (int32_t i = 0; i < nb; ++i)
            for (int32_t e = Pp[i + 1] - 1; e >= Pp[i] && Pj[e] > i; --e)
                lvl[Pj[e]] = std::max(lvl[Pj[e]], lvl[i] + 1);
        break;
    case BILU_SWEEP_LT:  // row p of L^T reads s_i for (i, p) in P, i > p
        for (int32_t i = nb - 1; i >= 0; --i)
            for (int32_t e = Pp[i]; e < Pp[i + 1] && Pj[e] < i; ++e)
                lvl[Pj[e]] = std::max(lvl[Pj[e]], lvl[i] + 1);
        break;
    default:
        return -1;
    }
    int nlev = 0;
    for (int32_t v : lvl) nlev = std::max(nlev, v + 1);
    return nlev;
}

namespace {

struct Dep {
    int32_t col;
    int64_t src;
};

// Dependencies of every row of a sweep, in ascending column order.
void sweep_deps(const Host& h, int which, std::vector<int32_t>& ptr, std::vector<Dep>& deps)
{
    const int nb = h.nb;
    ptr.assign(static_cast<size_t>(nb) + 1, 0);
    auto lower = [&](int32_t i, int32_t e) { return h.Pj[e] < i; };
    auto upper = [&](int32_t i, int32_t e) { return h.Pj[e] > i; };
    if (which == BILU_SWEEP_L || which == BILU_SWEEP_U) {
        for (int32_t i = 0; i < nb; ++i)
            for (int32_t e = h.Pp[i]; e < h.Pp[i + 1]; ++e)
                if (which == BILU_SWEEP_L ? lower(i, e) : upper(i, e)) ptr[i + 1]++;
        for (int i = 0; i < nb; ++i) ptr[i + 1] += ptr[i];
        deps.resize(static_cast<size_t>(ptr[nb]));
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int32_t i = 0; i < nb; ++i)
            for (int32_t e = h.Pp[i]; e < h.Pp[i + 1]; ++e)
                if (which == BILU_SWEEP_L ? lower(i, e) : upper(i, e))
                    deps[fill[i]++] = Dep{h.Pj[e], e};
    } else {
        // transposed sweeps: entry (i, j) of P feeds row j, reading row i
        const bool ut = (which == BILU_SWEEP_UT);
        for (int32_t i = 0; i < nb; ++i)
            for (int32_t e = h.Pp[i]; e < h.Pp[i + 1]; ++e)
                if (ut ? upper(i, e) : lower(i, e)) ptr[h.Pj[e] + 1]++;
        for (int i = 0; i < nb; ++i) ptr[i + 1] += ptr[i];
        deps.resize(static_cast<size_t>(ptr[nb]));
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int32_t i = 0; i < nb; ++i)        // ascending i => ascending columns
            for (int32_t e = h.Pp[i]; e < h.Pp[i + 1]; ++e)
                if (ut ? upper(i, e) : lower(i, e)) deps[fill[h.Pj[e]]++] = Dep{i, e};
    }
}

}  // namespace

// Level sets plus the chunked layout of one sweep.  Inside a level the rows
// are independent, so the chunks may order them freely: rows are sorted by
// decreasing dependency count (ties by row id) to keep the per-chunk
// padding small; the canonical level_rows stay in ascending order.
void build_sweep(const Host& h, int which, int rpc, HostSweep& s)
{
    const int nb = h.nb;
    std::vector<int32_t> lvl;
    s.which = which;
    s.rpc = rpc;
    s.transposed_blocks = (which == BILU_SWEEP_UT || which == BILU_SWEEP_LT);
    if (!h.dev_lvl[which].empty()) {
        lvl = h.dev_lvl[which];
        s.nlev = 0;
        for (int32_t v : lvl) s.nlev = std::max(s.nlev, v + 1);
    } else {
        s.nlev = sweep_levels(nb, h.Pp, h.Pj, which, lvl);
    }
    s.level_ptr.assign(static_cast<size_t>(s.nlev) + 1, 0);
    for (int32_t i = 0; i < nb; ++i) s.level_ptr[lvl[i] + 1]++;
    for (int l = 0; l < s.nlev; ++l) s.level_ptr[l + 1] += s.level_ptr[l];
    s.level_rows.resize(static_cast<size_t>(nb));
    {
        std::vector<int32_t> fill(s.level_ptr.begin(), s.level_ptr.end() - 1);
        for (int32_t i = 0; i < nb; ++i) s.level_rows[fill[lvl[i]]++] = i;
    }
    std::vector<int32_t> dptr;
    std::vector<Dep> deps;
    sweep_deps(h, which, dptr, deps);

    s.level_chunk_ptr.assign(static_cast<size_t>(s.nlev) + 1, 0);
    s.chunk_off.assign(1, 0);
    s.rows.clear();
    s.cols.clear();
    s.src.clear();
    std::vector<int32_t> order;
    for (int l = 0; l < s.nlev; ++l) {
        order.assign(s.level_rows.begin() + s.level_ptr[l], s.level_rows.begin() + s.level_ptr[l + 1]);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return (dptr[a + 1] - dptr[a]) > (dptr[b + 1] - dptr[b]);
        });
        s.level_chunk_ptr[l] = static_cast<int32_t>(s.chunk_off.size() - 1);
        for (size_t c0 = 0; c0 < order.size(); c0 += rpc) {
            const size_t cn = std::min(order.size() - c0, static_cast<size_t>(rpc));
            const int32_t w = dptr[order[c0] + 1] - dptr[order[c0]];
            const int64_t base = s.chunk_off.back();
            s.chunk_off.push_back(base + static_cast<int64_t>(w) * rpc);
            s.cols.resize(static_cast<size_t>(base) + static_cast<size_t>(w) * rpc, -1);
            s.src.resize(s.cols.size(), -1);
            for (int q = 0; q < rpc; ++q) {
                if (static_cast<size_t>(q) >= cn) {
                    s.rows.push_back(-1);
                    continue;
                }
                const int32_t r = order[c0 + q];
                s.rows.push_back(r);
                for (int32_t d = dptr[r]; d < dptr[r + 1]; ++d) {
                    const size_t slot = static_cast<size_t>(base) + static_cast<size_t>(d - dptr[r]) * rpc + q;
                    s.cols[slot] = deps[d].col;
                    s.src[slot] = deps[d].src;
                }
            }
        }
    }
    s.nchunks = static_cast<int>(s.chunk_off.size() - 1);
    s.level_chunk_ptr[s.nlev] = s.nchunks;
    s.nslots = s.chunk_off.back();
    s.built = true;
}

namespace {

// Rows [lo, hi] of tile t; tiles are numbered in sweep order.
inline void tile_range(int nb, int tile_rows, bool forward, int t, int& lo, int& hi)
{
    if (forward) {
        lo = t * tile_rows;
        hi = std::min(nb, lo + tile_rows) - 1;
    } else {
        hi = nb - 1 - t * tile_rows;
        lo = std::max(0, hi - tile_rows + 1);
    }
}

inline int tile_of_row(int nb, int tile_rows, bool forward, int j)
{
    return forward ? j / tile_rows : (nb - 1 - j) / tile_rows;
}

// The most frequent distance (in tiles) of the dependencies that cross
// tiles, over the first `rows` rows in sweep order; 0 if none cross.
int group_stride(int nb, int tile_rows, bool forward, const std::vector<int32_t>& dptr, const std::vector<Dep>& deps,
                 int rows)
{
    const int ntiles = (nb + tile_rows - 1) / tile_rows;
    std::vector<int64_t> cnt(static_cast<size_t>(ntiles) + 1, 0);
    for (int step = 0; step < rows; ++step) {
        const int32_t i = forward ? step : nb - 1 - step;
        const int ti = tile_of_row(nb, tile_rows, forward, i);
        for (int32_t d = dptr[i]; d < dptr[i + 1]; ++d) {
            const int tj = tile_of_row(nb, tile_rows, forward, deps[d].col);
            if (tj != ti) cnt[static_cast<size_t>(ti - tj)]++;
        }
    }
    int best = 0;
    for (int d = 1; d <= ntiles; ++d)
        if (cnt[d] > cnt[best]) best = d;
    return cnt[best] > 0 ? best : 0;
}

// Whether grouping keeps the ticket order over the first `rows` rows in
// sweep order: a dependency on another tile of the group is on an earlier
// member (all members run together), one on another group is on a group
// with a smaller ticket.
bool groups_ordered(int nb, int tile_rows, bool forward, const TileGroups& tg, const std::vector<int32_t>& dptr,
                    const std::vector<Dep>& deps, int rows)
{
    for (int step = 0; step < rows; ++step) {
        const int32_t i = forward ? step : nb - 1 - step;
        const int ti = tile_of_row(nb, tile_rows, forward, i);
        for (int32_t d = dptr[i]; d < dptr[i + 1]; ++d) {
            const int tj = tile_of_row(nb, tile_rows, forward, deps[d].col);
            if (tj == ti) continue;
            const int gi = tg.group(ti), gj = tg.group(tj);
            if (gi == gj ? tg.member(tj) >= tg.member(ti) : gj >= gi) return false;
        }
    }
    return true;
}

}  // namespace

namespace {

// LDS ring: a wavefront sweeping a tile alone reads a row of its tile only a
// few chunks after the chunk that formed it.  If every tile-local dependency
// spans at most maxd chunks (maxd < kRingMax), the wavefront keeps just the
// rows of its last maxd + 1 chunks: the row in lane slot q of the chunk at
// position k of its tile lives in LDS row (k mod ring)*rpc + q, and the
// codes are rewritten to those rows (the zero row moves to ring*rpc).
constexpr int kRingMax = 16;

void apply_ring(HostTiled& s, int nb, int bs)
{
    const int rpc = s.rpc;
    const int32_t row_bytes = bs * 8;
    std::vector<int32_t> chunk_of(static_cast<size_t>(nb), -1), q_of(static_cast<size_t>(nb), -1);
    for (int c = 0; c < s.nchunks; ++c)
        for (int q = 0; q < rpc; ++q) {
            const int32_t r = s.rows[static_cast<size_t>(c) * rpc + q];
            if (r >= 0) {
                chunk_of[r] = c;
                q_of[r] = q;
            }
        }
    const int32_t old_pad = tiled_local_code(s.tile_rows, bs);
    int maxd = 0;
    for (int t = 0; t < s.ntiles; ++t)
        for (int c = s.tile_chunk_ptr[t]; c < s.tile_chunk_ptr[t + 1]; ++c)
            for (int64_t x = s.chunk_off[c]; x < s.chunk_off[c + 1]; ++x) {
                const int32_t code = s.deps[x];
                if (code >= 0 || code == old_pad) continue;
                const int32_t j = s.tile_lo[t] + (code & INT32_MAX) / row_bytes;
                maxd = std::max(maxd, c - chunk_of[j]);
            }
    if (maxd < 1 || maxd >= kRingMax) return;
    const int ring = maxd + 1;
    if (static_cast<int64_t>(ring) * rpc >= s.tile_rows) return;     // no smaller than the tile
    const int32_t new_pad = tiled_local_code(ring * rpc, bs);
    for (int t = 0; t < s.ntiles; ++t) {
        const int first = s.tile_chunk_ptr[t];
        for (int c = first; c < s.tile_chunk_ptr[t + 1]; ++c)
            for (int64_t x = s.chunk_off[c]; x < s.chunk_off[c + 1]; ++x) {
                const int32_t code = s.deps[x];
                if (code >= 0) continue;
                if (code == old_pad) {
                    s.deps[x] = new_pad;
                    continue;
                }
                const int32_t j = s.tile_lo[t] + (code & INT32_MAX) / row_bytes;
                s.deps[x] = tiled_local_code(((chunk_of[j] - first) % ring) * rpc + q_of[j], bs);
            }
    }
    s.ring = ring;
}

}  // namespace

void build_tiled(const Host& h, int which, int rpc, int tile_rows, int group, int64_t lds_limit, bool allow_ring,
                 HostTiled& s)
{
    const int nb = h.nb;
    const int bs = h.bs;
    const bool forward = (which == BILU_SWEEP_L || which == BILU_SWEEP_UT);
    s = HostTiled{};
    // dependency codes are byte offsets into int32
    if (static_cast<int64_t>(nb) * bs * 8 > INT32_MAX) return;
    std::vector<int32_t> dptr;
    std::vector<Dep> deps;
    sweep_deps(h, which, dptr, deps);
    int max_ndep = 0;
    for (int i = 0; i < nb; ++i) max_ndep = std::max(max_ndep, dptr[i + 1] - dptr[i]);
    s.kmax = tiled_kmax(bs, max_ndep);
    s.which = which;
    s.rpc = rpc;
    s.tile_rows = tile_rows;
    s.ntiles = (nb + tile_rows - 1) / tile_rows;
    // the largest usable group not above the request
    TileGroups tg{1, 1, s.ntiles};
    s.group_req = group;
    group = std::max(1, std::min(group, kGroupMax));
    while (group > 1 && tiled_lds_bytes(tile_rows, group, bs) > lds_limit) --group;
    const int D = group > 1 ? group_stride(nb, tile_rows, forward, dptr, deps, nb) : 0;
    for (int g = group; g > 1 && D > 0; --g) {
        const TileGroups cand{g, D, s.ntiles};
        if (groups_ordered(nb, tile_rows, forward, cand, dptr, deps, nb)) {
            tg = cand;
            break;
        }
    }
    s.group = tg.G;
    s.gstride = tg.D;
    s.ngroups = tg.count();
    s.group_tiles.assign(static_cast<size_t>(s.ngroups) * tg.G, -1);
    for (int g = 0; g < s.ngroups; ++g)
        for (int m = 0; m < tg.G; ++m) s.group_tiles[static_cast<size_t>(g) * tg.G + m] = tg.tile(g, m);
    s.tile_chunk_ptr.assign(static_cast<size_t>(s.ntiles) + 1, 0);
    s.tile_lo.assign(static_cast<size_t>(s.ntiles), 0);
    s.chunk_off.assign(1, 0);
    const int32_t pad_code = tiled_local_code(tg.G * tile_rows, bs);      // the zero row
    std::vector<int32_t> il(static_cast<size_t>(tile_rows));            // level inside the tile
    std::vector<int32_t> cit(tg.G > 1 ? static_cast<size_t>(nb) : 0);   // chunk of a row inside its tile
    std::vector<int32_t> order;
    for (int t = 0; t < s.ntiles; ++t) {
        int lo, hi;
        tile_range(nb, tile_rows, forward, t, lo, hi);
        s.tile_lo[t] = lo;
        s.tile_chunk_ptr[t] = static_cast<int32_t>(s.chunk_off.size() - 1);
        const int gt = tg.group(t);
        // levels over the dependencies inside [lo, hi], rows in sweep order
        for (int step = 0; step <= hi - lo; ++step) {
            const int32_t i = forward ? lo + step : hi - step;
            int32_t l = 0;
            for (int32_t d = dptr[i]; d < dptr[i + 1]; ++d) {
                const int32_t j = deps[d].col;
                if (j >= lo && j <= hi) l = std::max(l, il[j - lo] + 1);
            }
            il[i - lo] = l;
        }
        order.resize(static_cast<size_t>(hi - lo + 1));
        std::iota(order.begin(), order.end(), lo);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            if (il[a - lo] != il[b - lo]) return il[a - lo] < il[b - lo];
            return (dptr[a + 1] - dptr[a]) > (dptr[b + 1] - dptr[b]);
        });
        size_t pos = 0;
        while (pos < order.size()) {
            const int32_t lev = il[order[pos] - lo];
            size_t cn = 0;
            while (pos + cn < order.size() && cn < static_cast<size_t>(rpc) && il[order[pos + cn] - lo] == lev) ++cn;
            // at least kmax slot rows: the kernel reads the first kmax of every chunk
            const int32_t w = std::max(dptr[order[pos] + 1] - dptr[order[pos]], s.kmax);
            const int64_t base = s.chunk_off.back();
            const int32_t chunk_in_tile = static_cast<int32_t>(s.chunk_off.size() - 1) - s.tile_chunk_ptr[t];
            s.chunk_off.push_back(base + static_cast<int64_t>(w) * rpc);
            s.deps.resize(static_cast<size_t>(base) + static_cast<size_t>(w) * rpc, pad_code);
            s.src.resize(s.deps.size(), -1);
            int32_t wait[kGroupMax] = {0, 0, 0, 0};
            for (int q = 0; q < rpc; ++q) {
                if (static_cast<size_t>(q) >= cn) {
                    s.rows.push_back(-1);
                    continue;
                }
                const int32_t i = order[pos + q];
                s.rows.push_back(i);
                if (tg.G > 1) cit[i] = chunk_in_tile;
                for (int32_t d = dptr[i]; d < dptr[i + 1]; ++d) {
                    const size_t slot = static_cast<size_t>(base) + static_cast<size_t>(d - dptr[i]) * rpc + q;
                    const int32_t j = deps[d].col;
                    const int tj = tile_of_row(nb, tile_rows, forward, j);
                    int32_t code;
                    if (tg.group(tj) == gt) {          // a row of this group: in its LDS
                        const int mj = tg.member(tj);
                        code = tiled_local_code(mj * tile_rows + (j - s.tile_lo[tj]), bs);
                        if (tj != t) wait[mj] = std::max(wait[mj], cit[j] + 1);
                    } else {
                        code = tiled_global_code(j, bs);
                    }
                    s.deps[slot] = code;
                    s.src[slot] = deps[d].src;
                }
            }
            if (tg.G > 1) s.chunk_wait.insert(s.chunk_wait.end(), wait, wait + kGroupMax);
            pos += cn;
        }
    }
    s.nchunks = static_cast<int>(s.chunk_off.size() - 1);
    s.tile_chunk_ptr[s.ntiles] = s.nchunks;
    s.nslots = s.chunk_off.back();
    if (tg.G == 1 && allow_ring) apply_ring(s, nb, bs);
    s.built = true;
}

bool grid_lines(const Host& h, int& nx, int& nxy)
{
    const int nb = h.nb;
    std::vector<int32_t> dptr;
    std::vector<Dep> deps;
    sweep_deps(h, BILU_SWEEP_L, dptr, deps);
    auto has = [&](int32_t i, int32_t d) {
        for (int32_t e = dptr[i]; e < dptr[i + 1]; ++e)
            if (deps[e].col == i - d) return true;
        return false;
    };
    // line starts: rows without a dependency on the previous row
    nx = 0;
    for (int32_t i = 1; i < nb && !nx; ++i)
        if (!has(i, 1)) nx = i;
    if (nx < 2 || nb % nx != 0) return false;
    for (int32_t i = 1; i < nb; ++i)
        if (has(i, 1) == (i % nx == 0)) return false;
    // plane starts: line starts without a dependency on the line before
    nxy = 0;
    for (int32_t i = nx; i < nb && !nxy; i += nx)
        if (!has(i, nx)) nxy = i;
    if (nxy == 0) nxy = nb;                 // a single plane
    if (nxy % nx != 0 || nb % nxy != 0) return false;
    for (int32_t i = nx; i < nb; i += nx)
        if (has(i, nx) == (i % nxy == 0)) return false;
    return true;
}

void build_tiled_blocks(const Host& h, int which, int rpc, int ny_b, int nz_b, HostTiled& s)
{
    const int nb = h.nb;
    const int bs = h.bs;
    const bool forward = (which == BILU_SWEEP_L || which == BILU_SWEEP_UT);
    s = HostTiled{};
    int nx = 0, nxy = 0;
    if (ny_b < 1 || nz_b < 1 || !grid_lines(h, nx, nxy)) return;
    if (static_cast<int64_t>(nb) * bs * 8 > INT32_MAX) return;
    const int ny = nxy / nx, nz = nb / nxy;
    const int NYb = (ny + ny_b - 1) / ny_b, NZb = (nz + nz_b - 1) / nz_b;
    std::vector<int32_t> dptr;
    std::vector<Dep> deps;
    sweep_deps(h, which, dptr, deps);
    int max_ndep = 0;
    for (int i = 0; i < nb; ++i) max_ndep = std::max(max_ndep, dptr[i + 1] - dptr[i]);
    s.kmax = tiled_kmax(bs, max_ndep);
    s.which = which;
    s.rpc = rpc;
    s.block_ny = ny_b;
    s.block_nz = nz_b;
    s.ntiles = NYb * NZb;
    // tile of a row: blocks numbered plane-block by plane-block in the
    // forward sweep, the reverse for backward sweeps
    auto tile_of = [&](int32_t i) {
        const int line = i / nx;
        const int t = (line / ny / nz_b) * NYb + (line % ny) / ny_b;
        return forward ? t : s.ntiles - 1 - t;
    };
    std::vector<int32_t> tile_ptr(static_cast<size_t>(s.ntiles) + 1, 0), trow(static_cast<size_t>(nb));
    for (int32_t i = 0; i < nb; ++i) tile_ptr[tile_of(i) + 1]++;
    for (int t = 0; t < s.ntiles; ++t) tile_ptr[t + 1] += tile_ptr[t];
    {
        std::vector<int32_t> fill(tile_ptr.begin(), tile_ptr.end() - 1);
        for (int step = 0; step < nb; ++step) {        // rows of a tile in sweep order
            const int32_t i = forward ? step : nb - 1 - step;
            trow[fill[tile_of(i)]++] = i;
        }
    }
    // every dependency on another tile must be on an earlier one
    for (int32_t i = 0; i < nb; ++i)
        for (int32_t d = dptr[i]; d < dptr[i + 1]; ++d)
            if (tile_of(deps[d].col) > tile_of(i)) return;
    s.group = 1;
    s.gstride = 1;
    s.ngroups = s.ntiles;
    s.group_tiles.resize(static_cast<size_t>(s.ntiles));
    std::iota(s.group_tiles.begin(), s.group_tiles.end(), 0);
    s.tile_chunk_ptr.assign(static_cast<size_t>(s.ntiles) + 1, 0);
    s.tile_lo.assign(static_cast<size_t>(s.ntiles), 0);
    s.chunk_off.assign(1, 0);
    std::vector<int32_t> lev(static_cast<size_t>(nb), 0), chunk_of(static_cast<size_t>(nb), -1),
        q_of(static_cast<size_t>(nb), -1);
    // chunks: rows of a tile by level inside the tile, at most rpc per chunk
    std::vector<int32_t> order;
    std::vector<int32_t> chunk_tile;
    for (int t = 0; t < s.ntiles; ++t) {
        const int32_t b0 = tile_ptr[t], b1 = tile_ptr[t + 1];
        s.tile_lo[t] = trow[b0];
        s.tile_chunk_ptr[t] = static_cast<int32_t>(chunk_tile.size());
        for (int32_t p = b0; p < b1; ++p) {
            const int32_t i = trow[p];
            int32_t l = 0;
            for (int32_t d = dptr[i]; d < dptr[i + 1]; ++d) {
                const int32_t j = deps[d].col;
                if (tile_of(j) == t) l = std::max(l, lev[j] + 1);
            }
            lev[i] = l;
        }
        order.assign(trow.begin() + b0, trow.begin() + b1);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            if (lev[a] != lev[b]) return lev[a] < lev[b];
            return (dptr[a + 1] - dptr[a]) > (dptr[b + 1] - dptr[b]);
        });
        size_t pos = 0;
        while (pos < order.size()) {
            size_t cn = 0;
            while (pos + cn < order.size() && cn < static_cast<size_t>(rpc) && lev[order[pos + cn]] == lev[order[pos]])
                ++cn;
            const int32_t c = static_cast<int32_t>(chunk_tile.size());
            chunk_tile.push_back(t);
            for (size_t q = 0; q < static_cast<size_t>(rpc); ++q) {
                const int32_t i = q < cn ? order[pos + q] : -1;
                s.rows.push_back(i);
                if (i >= 0) {
                    chunk_of[i] = c;
                    q_of[i] = static_cast<int32_t>(q);
                }
            }
            pos += cn;
        }
    }
    s.nchunks = static_cast<int>(chunk_tile.size());
    s.tile_chunk_ptr[s.ntiles] = s.nchunks;
    // ring depth: the farthest in-tile dependency, in chunks
    int maxd = 0;
    for (int32_t i = 0; i < nb; ++i)
        for (int32_t d = dptr[i]; d < dptr[i + 1]; ++d) {
            const int32_t j = deps[d].col;
            if (tile_of(j) == tile_of(i)) maxd = std::max(maxd, chunk_of[i] - chunk_of[j]);
        }
    if (maxd >= kRingMax) return;
    s.ring = std::max(1, maxd + 1);
    s.tile_rows = s.ring * rpc;
    const int32_t pad_code = tiled_local_code(s.ring * rpc, bs);        // the zero row
    for (int c = 0; c < s.nchunks; ++c) {
        const int t = chunk_tile[c];
        const int32_t first = s.tile_chunk_ptr[t];
        const int32_t* rowc = &s.rows[static_cast<size_t>(c) * rpc];
        const int32_t w = std::max(dptr[rowc[0] + 1] - dptr[rowc[0]], s.kmax);
        const int64_t base = s.chunk_off.back();
        s.chunk_off.push_back(base + static_cast<int64_t>(w) * rpc);
        s.deps.resize(static_cast<size_t>(base) + static_cast<size_t>(w) * rpc, pad_code);
        s.src.resize(s.deps.size(), -1);
        for (int q = 0; q < rpc; ++q) {
            const int32_t i = rowc[q];
            if (i < 0) continue;
            for (int32_t d = dptr[i]; d < dptr[i + 1]; ++d) {
                const size_t slot = static_cast<size_t>(base) + static_cast<size_t>(d - dptr[i]) * rpc + q;
                const int32_t j = deps[d].col;
                s.deps[slot] = tile_of(j) == t
                                   ? tiled_local_code(((chunk_of[j] - first) % s.ring) * rpc + q_of[j], bs)
                                   : tiled_global_code(j, bs);
                s.src[slot] = deps[d].src;
            }
        }
    }
    s.nslots = s.chunk_off.back();
    s.built = true;
}

namespace {
// Grid coordinates of the sweep: a forward sweep (L, U'^T) walks rows
// ascending, a backward one (U', L^T) descending; sweep coordinates mirror
// the grid for backward sweeps.
struct LineGeom {
    int nx = 0, ny = 0, nz = 0;
    bool forward = true;
    int32_t row(int xs, int ys, int zs) const
    {
        const int x = forward ? xs : nx - 1 - xs, y = forward ? ys : ny - 1 - ys, z = forward ? zs : nz - 1 - zs;
        return x + nx * (y + ny * z);
    }
    void coords(int32_t i, int& xs, int& ys, int& zs) const
    {
        int x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
        xs = forward ? x : nx - 1 - x;
        ys = forward ? y : ny - 1 - y;
        zs = forward ? z : nz - 1 - z;
    }
};
}  // namespace

void build_line_layout(const Host& h, int which, int rpc, int ny_b, int nz_b, HostTiled& s)
{
    s = HostTiled{};
    if (which != BILU_SWEEP_L && which != BILU_SWEEP_U) return;
    if (ny_b < 1 || nz_b < 1 || ny_b * nz_b > rpc) return;
    const int nb = h.nb;
    if (static_cast<int64_t>(nb) * h.bs * 8 > INT32_MAX) return;
    int nx = 0, nxy = 0;
    if (!grid_lines(h, nx, nxy)) return;
    LineGeom g;
    g.nx = nx;
    g.ny = nxy / nx;
    g.nz = nb / nxy;
    g.forward = which == BILU_SWEEP_L;
    std::vector<int32_t> dptr;
    std::vector<Dep> deps;
    sweep_deps(h, which, dptr, deps);
    // slot order: the dependencies in ascending column order, as every sweep
    // forms a row (L: z-1, y-1, x-1; U': x+1, y+1, z+1)
    const int dims[3] = {g.forward ? 2 : 0, 1, g.forward ? 0 : 2};
    // eligibility: each row depends on exactly its grid neighbours before it,
    // listed in that order
    for (int32_t i = 0; i < nb; ++i) {
        int xs, ys, zs;
        g.coords(i, xs, ys, zs);
        int32_t want[3];
        int n = 0;
        for (int k = 0; k < 3; ++k) {
            const int d = dims[k];
            const int cx = xs - (d == 0), cy = ys - (d == 1), cz = zs - (d == 2);
            if (cx >= 0 && cy >= 0 && cz >= 0) want[n++] = g.row(cx, cy, cz);
        }
        if (dptr[i + 1] - dptr[i] != n) return;
        for (int k = 0; k < n; ++k)
            if (deps[dptr[i] + k].col != want[k]) return;
    }
    const int NYb = (g.ny + ny_b - 1) / ny_b, NZb = (g.nz + nz_b - 1) / nz_b;
    const int nsteps = nx + ny_b + nz_b - 2;
    s.which = which;
    s.rpc = rpc;
    s.kmax = 3;
    s.lines = true;
    s.block_ny = ny_b;
    s.block_nz = nz_b;
    s.line_nx = nx;
    s.line_ny = g.ny;
    s.line_nz = g.nz;
    s.line_steps = nsteps;
    s.line_NYb = NYb;
    for (int k = 0; k < 3; ++k) s.line_dim[k] = dims[k];
    s.ntiles = NYb * NZb;
    s.nchunks = s.ntiles * nsteps;
    s.tile_rows = 1;
    s.group = 1;
    s.gstride = 1;
    s.ngroups = s.ntiles;
    s.group_tiles.resize(static_cast<size_t>(s.ntiles));
    std::iota(s.group_tiles.begin(), s.group_tiles.end(), 0);
    s.tile_chunk_ptr.resize(static_cast<size_t>(s.ntiles) + 1);
    s.tile_lo.assign(static_cast<size_t>(s.ntiles), 0);
    for (int t = 0; t <= s.ntiles; ++t) s.tile_chunk_ptr[t] = t * nsteps;
    s.chunk_off.resize(static_cast<size_t>(s.nchunks) + 1);
    for (int c = 0; c <= s.nchunks; ++c) s.chunk_off[c] = static_cast<int64_t>(c) * 3 * rpc;
    s.nslots = s.chunk_off.back();
    s.rows.assign(static_cast<size_t>(s.nchunks) * rpc, -1);
    s.deps.assign(static_cast<size_t>(s.nslots), tiled_local_code(0, h.bs));
    s.src.assign(static_cast<size_t>(s.nslots), -1);
    for (int t = 0; t < s.ntiles; ++t) {
        const int Yb = t % NYb, Zb = t / NYb;
        s.tile_lo[t] = g.row(0, std::min(Yb * ny_b, g.ny - 1), std::min(Zb * nz_b, g.nz - 1));
        for (int q = 0; q < ny_b * nz_b; ++q) {
            const int yl = q % ny_b, zl = q / ny_b;
            const int ys = Yb * ny_b + yl, zs = Zb * nz_b + zl;
            if (ys >= g.ny || zs >= g.nz) continue;
            for (int xs = 0; xs < nx; ++xs) {
                const int step = xs + yl + zl;
                const int64_t c = static_cast<int64_t>(t) * nsteps + step;
                const int32_t i = g.row(xs, ys, zs);
                s.rows[static_cast<size_t>(c) * rpc + q] = i;
                int n = 0;
                for (int k = 0; k < 3; ++k) {
                    const int d = dims[k];
                    const int cx = xs - (d == 0), cy = ys - (d == 1), cz = zs - (d == 2);
                    if (cx < 0 || cy < 0 || cz < 0) continue;
                    const int64_t slot = s.chunk_off[c] + static_cast<int64_t>(k) * rpc + q;
                    const Dep& dp = deps[dptr[i] + n++];
                    s.src[static_cast<size_t>(slot)] = dp.src;
                    s.deps[static_cast<size_t>(slot)] = tiled_global_code(dp.col, h.bs);
                }
            }
        }
    }
    s.built = true;
}

int validate_line_layout(const Host& h, const HostTiled& s)
{
    if (!s.lines || !s.built) return BILU_ERR_STATE;
    const int nb = h.nb, rpc = s.rpc;
    const int WY = s.block_ny, WZ = s.block_nz;
    if (WY < 1 || WZ < 1 || WY * WZ > rpc || rpc * h.bs > kWave) return BILU_ERR_STATE;
    LineGeom g;
    g.nx = s.line_nx;
    g.ny = s.line_ny;
    g.nz = s.line_nz;
    g.forward = s.which == BILU_SWEEP_L;
    if (s.which != BILU_SWEEP_L && s.which != BILU_SWEEP_U) return BILU_ERR_STATE;
    if (g.nx < 1 || g.ny < 1 || g.nz < 1 || static_cast<int64_t>(g.nx) * g.ny * g.nz != nb) return BILU_ERR_STATE;
    if (static_cast<int64_t>(nb) * h.bs * 8 > INT32_MAX) return BILU_ERR_STATE;
    const int NYb = (g.ny + WY - 1) / WY, NZb = (g.nz + WZ - 1) / WZ;
    if (s.line_NYb != NYb || s.ntiles != NYb * NZb || s.line_steps != g.nx + WY + WZ - 2) return BILU_ERR_STATE;
    if (s.nchunks != s.ntiles * s.line_steps || static_cast<int64_t>(s.rows.size()) != static_cast<int64_t>(s.nchunks) * rpc ||
        s.nslots != static_cast<int64_t>(s.nchunks) * 3 * rpc || static_cast<int64_t>(s.src.size()) != s.nslots ||
        static_cast<int>(s.chunk_off.size()) != s.nchunks + 1)
        return BILU_ERR_STATE;
    for (int c = 0; c <= s.nchunks; ++c)
        if (s.chunk_off[c] != static_cast<int64_t>(c) * 3 * rpc) return BILU_ERR_STATE;
    int dims_seen = 0;
    for (int k = 0; k < 3; ++k) {
        if (s.line_dim[k] < 0 || s.line_dim[k] > 2) return BILU_ERR_STATE;
        dims_seen |= 1 << s.line_dim[k];
    }
    if (dims_seen != 7) return BILU_ERR_STATE;
    std::vector<int32_t> seen(static_cast<size_t>(nb), 0);
    const int64_t nP = static_cast<int64_t>(h.Pj.size());
    const bool rowwise = true;   // L and U': the entry of row i, column j
    std::vector<int32_t> ndep(static_cast<size_t>(nb), 0), used(static_cast<size_t>(nb), 0);
    for (int32_t i = 0; i < nb; ++i)
        for (int32_t e = h.Pp[i]; e < h.Pp[i + 1]; ++e) {
            const int32_t j = h.Pj[e];
            if (g.forward ? j < i : j > i) ndep[i]++;
        }
    for (int t = 0; t < s.ntiles; ++t) {
        const int Yb = t % NYb, Zb = t / NYb;
        for (int st = 0; st < s.line_steps; ++st) {
            const int64_t c = static_cast<int64_t>(t) * s.line_steps + st;
            for (int q = 0; q < rpc; ++q) {
                const int32_t i = s.rows[static_cast<size_t>(c) * rpc + q];
                // the row the kernel computes for this lane, if any
                const bool lane_line = q < WY * WZ;
                const int yl = lane_line ? q % WY : 0, zl = lane_line ? q / WY : 0;
                const int ys = Yb * WY + yl, zs = Zb * WZ + zl, xs = st - yl - zl;
                const bool act = lane_line && ys < g.ny && zs < g.nz && xs >= 0 && xs < g.nx;
                if (act != (i >= 0)) return BILU_ERR_STATE;
                if (!act) {
                    for (int k = 0; k < 3; ++k)
                        if (s.src[static_cast<size_t>(s.chunk_off[c] + k * rpc + q)] != -1) return BILU_ERR_STATE;
                    continue;
                }
                if (i != g.row(xs, ys, zs) || seen[i]++) return BILU_ERR_STATE;
                for (int k = 0; k < 3; ++k) {
                    const int d = s.line_dim[k];
                    const int cx = xs - (d == 0), cy = ys - (d == 1), cz = zs - (d == 2);
                    const int64_t e = s.src[static_cast<size_t>(s.chunk_off[c] + k * rpc + q)];
                    const bool exists = cx >= 0 && cy >= 0 && cz >= 0;
                    if (!exists) {
                        // the kernel reads zero for a neighbour outside the grid
                        if (e != -1) return BILU_ERR_STATE;
                        continue;
                    }
                    // every grid neighbour before the row is a dependency
                    if (e < 0 || e >= nP) return BILU_ERR_STATE;
                    const int32_t j = g.row(cx, cy, cz);
                    if (!rowwise || h.Prow[e] != i || h.Pj[e] != j) return BILU_ERR_STATE;
                    used[i]++;
                    // where the kernel reads it: the same block one step
                    // earlier, or a block with a smaller ticket
                    const bool inside = (d == 0) || (d == 1 && yl > 0) || (d == 2 && zl > 0);
                    if (inside) {
                        const int qq = d == 0 ? q : (d == 1 ? q - 1 : q - WY);
                        if (st < 1 || s.rows[static_cast<size_t>(c - 1) * rpc + qq] != j) return BILU_ERR_STATE;
                    } else {
                        const int tb = (cz / WZ) * NYb + cy / WY;
                        if (tb >= t) return BILU_ERR_STATE;
                    }
                }
            }
        }
    }
    for (int32_t i = 0; i < nb; ++i)
        if (seen[i] != 1 || used[i] != ndep[i]) return BILU_ERR_STATE;
    return BILU_OK;
}

// Event simulation of the tiled schedule: tiles run concurrently, a tile
// walks its chunks in order, a chunk costs one step and may start once the
// previous chunk of its tile is done and every row it reads from another
// tile has been finished for `hop` steps (a tile of the same group: for
// kLocalHop steps, the cost of an LDS handoff).  Chunks are formed exactly as
// in build_tiled.  Returns the finishing time of the last chunk, or +inf
// where the grouping breaks the ticket order.
namespace {
constexpr double kLocalHop = 0.5;

double simulate_deps(const Host& h, int which, const std::vector<int32_t>& dptr, const std::vector<Dep>& deps,
                     int rpc, int tile_rows, int group, double hop, int row_limit)
{
    const int nb = row_limit > 0 ? std::min(h.nb, row_limit) : h.nb;
    const bool forward = (which == BILU_SWEEP_L || which == BILU_SWEEP_UT);
    // a forward sweep restricted to its first `nb` rows is itself a sweep
    const int ntiles = forward ? (nb + tile_rows - 1) / tile_rows : (h.nb + tile_rows - 1) / tile_rows;
    TileGroups tg{1, 1, ntiles};
    if (group > 1) {
        const int rows = forward ? nb : h.nb;
        const int D = group_stride(h.nb, tile_rows, forward, dptr, deps, rows);
        if (D <= 0) return std::numeric_limits<double>::infinity();
        tg = TileGroups{group, D, ntiles};
        if (!groups_ordered(h.nb, tile_rows, forward, tg, dptr, deps, rows))
            return std::numeric_limits<double>::infinity();
    }
    std::vector<double> done(static_cast<size_t>(h.nb), 0.0);
    std::vector<int32_t> il(static_cast<size_t>(tile_rows)), order;
    double makespan = 0.0;
    for (int t = 0; t < ntiles; ++t) {
        int lo, hi;
        if (forward) {
            lo = t * tile_rows;
            hi = std::min(nb, lo + tile_rows) - 1;
        } else {
            tile_range(h.nb, tile_rows, false, t, lo, hi);
        }
        const int gt = tg.group(t);
        for (int step = 0; step <= hi - lo; ++step) {
            const int32_t i = forward ? lo + step : hi - step;
            int32_t l = 0;
            for (int32_t d = dptr[i]; d < dptr[i + 1]; ++d) {
                const int32_t j = deps[d].col;
                if (j >= lo && j <= hi) l = std::max(l, il[j - lo] + 1);
            }
            il[i - lo] = l;
        }
        // rows grouped by level (ties: more dependencies first, then row order)
        order.resize(static_cast<size_t>(hi - lo + 1));
        std::iota(order.begin(), order.end(), lo);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            if (il[a - lo] != il[b - lo]) return il[a - lo] < il[b - lo];
            return (dptr[a + 1] - dptr[a]) > (dptr[b + 1] - dptr[b]);
        });
        double now = 0.0;
        size_t pos = 0;
        while (pos < order.size()) {
            const int32_t lev = il[order[pos] - lo];
            size_t cn = 0;
            while (pos + cn < order.size() && cn < static_cast<size_t>(rpc) && il[order[pos + cn] - lo] == lev) ++cn;
            double ready = now;
            for (size_t q = 0; q < cn; ++q) {
                const int32_t i = order[pos + q];
                for (int32_t d = dptr[i]; d < dptr[i + 1]; ++d) {
                    const int32_t j = deps[d].col;
                    if (j >= lo && j <= hi) continue;
                    const bool same = tg.G > 1 && tg.group(tile_of_row(h.nb, tile_rows, forward, j)) == gt;
                    ready = std::max(ready, done[j] + (same ? kLocalHop : hop));
                }
            }
            now = ready + 1.0;
            for (size_t q = 0; q < cn; ++q) done[order[pos + q]] = now;
            pos += cn;
        }
        makespan = std::max(makespan, now);
    }
    return makespan;
}

// Dependency distance histogram of the L sweep, most frequent first.
std::vector<std::pair<int64_t, int32_t>> distance_histogram(const Host& h)
{
    std::vector<std::pair<int64_t, int32_t>> hist;
    std::vector<int32_t> dist;
    dist.reserve(static_cast<size_t>(h.nb) * 4);
    for (int32_t i = 0; i < h.nb; ++i)
        for (int32_t e = h.Pp[i]; e < h.Pp[i + 1] && h.Pj[e] < i; ++e) dist.push_back(i - h.Pj[e]);
    std::sort(dist.begin(), dist.end());
    for (size_t a = 0; a < dist.size();) {
        size_t b = a;
        while (b < dist.size() && dist[b] == dist[a]) ++b;
        hist.emplace_back(static_cast<int64_t>(b - a), dist[a]);
        a = b;
    }
    std::sort(hist.begin(), hist.end(), std::greater<>());
    return hist;
}

// Candidate tile sizes: a geometric grid, plus divisors and multiples of the
// most frequent dependency distances (on a grid these are the line and plane
// periods; a tile aligned with them keeps corresponding rows of consecutive
// tiles at the same level inside their tiles).
std::vector<int> tile_candidates(const Host& h, int rpc, int max_rows,
                                 const std::vector<std::pair<int64_t, int32_t>>& hist)
{
    const int min_rows = std::min(max_rows, std::max(1, 2 * rpc));
    std::vector<int> cand;
    for (double m = min_rows; m <= max_rows; m *= 1.5) cand.push_back(static_cast<int>(m));
    cand.push_back(max_rows);
    const size_t top = std::min<size_t>(hist.size(), 4);
    static const int kMult[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56, 64};
    for (size_t a = 0; a < top; ++a) {
        const int d = hist[a].second;
        for (int j : kMult) {
            if (d / j >= min_rows && d / j <= max_rows && d % j == 0) cand.push_back(d / j);
            if (static_cast<int64_t>(d) * j >= min_rows && static_cast<int64_t>(d) * j <= max_rows) cand.push_back(d * j);
        }
    }
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    (void)h;
    return cand;
}

// A prefix of the sweep shows how tiles pipeline: a few multiples of the
// longest frequent dependency distance and of the largest tile.
int sim_row_limit(const Host& h, int max_rows, const std::vector<std::pair<int64_t, int32_t>>& hist)
{
    int64_t longest = 1;
    for (size_t a = 0; a < std::min<size_t>(hist.size(), 4); ++a) longest = std::max<int64_t>(longest, hist[a].second);
    return static_cast<int>(std::min<int64_t>(h.nb, std::max<int64_t>({8 * longest, 16LL * max_rows, 65536})));
}
}  // namespace

double simulate_tiled(const Host& h, int which, int rpc, int tile_rows, int group, double hop, int row_limit)
{
    std::vector<int32_t> dptr;
    std::vector<Dep> deps;
    sweep_deps(h, which, dptr, deps);
    return simulate_deps(h, which, dptr, deps, rpc, tile_rows, group, hop, row_limit);
}

// The smallest simulated makespan of the L sweep wins; ties go to the larger
// tile.
std::vector<std::pair<double, int>> rank_tile_rows(const Host& h, int rpc, int max_rows)
{
    max_rows = std::max(1, std::min(max_rows, h.nb));
    const auto hist = distance_histogram(h);
    const std::vector<int> cand = tile_candidates(h, rpc, max_rows, hist);
    const int limit = sim_row_limit(h, max_rows, hist);
    std::vector<int32_t> dptr;
    std::vector<Dep> deps;
    sweep_deps(h, BILU_SWEEP_L, dptr, deps);
    std::vector<std::pair<double, int>> ranked;
    for (int m : cand) ranked.emplace_back(simulate_deps(h, BILU_SWEEP_L, dptr, deps, rpc, m, 1, 5.0, limit), m);
    // shortest predicted sweep first; on (near) ties the larger tile
    std::sort(ranked.begin(), ranked.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
        if (std::fabs(a.first - b.first) > 1e-9 * std::max(a.first, b.first)) return a.first < b.first;
        return a.second > b.second;
    });
    return ranked;
}

// Group sizes in order of preference.  The simulation above models the
// dependency structure only; measured on MI355X (60x220x85 and 64^3 grids,
// ILU(0)), groups of 3 beat groups of 4 and 2: the member tiles of a group
// share one compute unit and near the sweep front all of them issue loads
// at once, which the model does not see.
constexpr int kGroupPreference[] = {3, 4, 2};

std::vector<TileChoice> rank_tile_layouts(const Host& h, int rpc, int64_t lds_limit, int tile_req, int group_req)
{
    // one tile's rows stay within 64 KiB of LDS, so several tiles share a CU
    const int64_t tile_lds = std::min<int64_t>(lds_limit, 65536);
    const int max_rows = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(h.nb, tile_lds / (8LL * h.bs) - 1)));
    const auto hist = distance_histogram(h);
    const int limit = sim_row_limit(h, max_rows, hist);
    std::vector<int32_t> dptr;
    std::vector<Dep> deps;
    sweep_deps(h, BILU_SWEEP_L, dptr, deps);
    // tile sizes with one wavefront per tile, best first
    std::vector<TileChoice> single;
    const std::vector<int> cand = tile_req > 0 ? std::vector<int>{std::min(tile_req, max_rows)}
                                               : tile_candidates(h, rpc, max_rows, hist);
    for (int m : cand) single.push_back(TileChoice{simulate_deps(h, BILU_SWEEP_L, dptr, deps, rpc, m, 1, 5.0, limit), m, 1});
    std::sort(single.begin(), single.end(), [](const TileChoice& a, const TileChoice& b) {
        if (std::fabs(a.t - b.t) > 1e-9 * std::max(a.t, b.t)) return a.t < b.t;
        return a.tile_rows > b.tile_rows;
    });
    if (group_req == 1) return single;
    // groups of the best tile size: usable (LDS, ticket order) and shorter
    // than the single tiles in the simulation, in order of preference
    const TileChoice best = single.front();
    std::vector<TileChoice> grouped;
    auto consider = [&](int g) {
        if (g < 2 || g > kGroupMax || tiled_lds_bytes(best.tile_rows, g, h.bs) > lds_limit) return;
        const double t = simulate_deps(h, BILU_SWEEP_L, dptr, deps, rpc, best.tile_rows, g, 5.0, limit);
        if (std::isfinite(t) && (group_req > 1 || t < best.t)) grouped.push_back(TileChoice{t, best.tile_rows, g});
    };
    if (group_req > 1) {
        consider(std::min(group_req, kGroupMax));
    } else {
        for (int g : kGroupPreference) consider(g);
    }
    grouped.insert(grouped.end(), single.begin(), single.end());
    return grouped;
}

int choose_tile_rows(const Host& h, int rpc, int max_rows)
{
    return rank_tile_rows(h, rpc, max_rows).front().second;
}


int analyze_host(Host& h, int nb, int bs, const int32_t* Ap, const int32_t* Aj, int k, int flags)
{
    if (nb < 1 || bs < 1 || bs > kMaxBs || k < 0 || !Ap || !Aj) return BILU_ERR_ARG;
    int st = validate_pattern(nb, Ap, Aj);
    if (st != BILU_OK) return st;
    h.nb = nb;
    h.bs = bs;
    h.k = k;
    h.flags = flags;
    h.rpc = kWave / bs;
    h.Ap.assign(Ap, Ap + nb + 1);
    h.Aj.assign(Aj, Aj + Ap[nb]);
    h.Arow.resize(h.Aj.size());
    for (int32_t i = 0; i < nb; ++i)
        for (int32_t e = Ap[i]; e < Ap[i + 1]; ++e) h.Arow[e] = i;

    if (flags & BILU_DEVICE_SYMBOLIC)
        st = device_analysis(nb, Ap, Aj, k, (flags & BILU_WANT_TRANSPOSE) ? 4 : 2, h.Pp, h.Pj, h.Plev, h.dev_lvl);
    else
        st = symbolic_iluk(nb, Ap, Aj, k, h.Pp, h.Pj, h.Plev);
    if (st != BILU_OK) return st;
    const size_t nP = h.Pj.size();
    h.Pdiag.resize(static_cast<size_t>(nb));
    h.Prow.resize(nP);
    for (int32_t i = 0; i < nb; ++i)
        for (int32_t e = h.Pp[i]; e < h.Pp[i + 1]; ++e) {
            h.Prow[e] = i;
            if (h.Pj[e] == i) h.Pdiag[i] = e;
        }
    // A's blocks inside P (Algorithm 5, backfill): both rows are sorted.
    h.AtoP.resize(h.Aj.size());
    std::vector<char> inA(nP, 0);
    for (int32_t i = 0; i < nb; ++i) {
        int32_t f = h.Pp[i];
        for (int32_t e = Ap[i]; e < Ap[i + 1]; ++e) {
            while (h.Pj[f] < Aj[e]) ++f;
            h.AtoP[e] = f;
            inA[f] = 1;
        }
    }
    h.Pfill.clear();
    for (size_t e = 0; e < nP; ++e)
        if (!inA[e]) h.Pfill.push_back(static_cast<int32_t>(e));

    build_sweep(h, BILU_SWEEP_L, h.rpc, h.sweep[BILU_SWEEP_L]);
    build_sweep(h, BILU_SWEEP_U, h.rpc, h.sweep[BILU_SWEEP_U]);
    if (flags & BILU_WANT_TRANSPOSE) {
        build_sweep(h, BILU_SWEEP_UT, h.rpc, h.sweep[BILU_SWEEP_UT]);
        build_sweep(h, BILU_SWEEP_LT, h.rpc, h.sweep[BILU_SWEEP_LT]);
        h.ATp.assign(static_cast<size_t>(nb) + 1, 0);
        for (int32_t j : h.Aj) h.ATp[j + 1]++;
        for (int i = 0; i < nb; ++i) h.ATp[i + 1] += h.ATp[i];
        h.ATj.resize(h.Aj.size());
        h.ATsrc.resize(h.Aj.size());
        std::vector<int32_t> fill(h.ATp.begin(), h.ATp.end() - 1);
        for (int32_t i = 0; i < nb; ++i)
            for (int32_t e = Ap[i]; e < Ap[i + 1]; ++e) {
                const int32_t j = Aj[e];
                h.ATj[fill[j]] = i;
                h.ATsrc[fill[j]++] = e;
            }
    }
    return BILU_OK;
}

namespace {
// Replays, for every chunk and every lane of a wavefront, the index
// arithmetic of the tiled sweep kernel (batch loads, dependency reads, LDS
// accesses, stores) and checks each index against the size of the array it
// addresses.  Mirrors k_sweep_tiled / tile_meta / tile_data / tile_compute
// in kernels.h (chunk indices past a tile's end clamp to its last chunk, so
// visiting every chunk covers them).
bool tiled_accesses_in_bounds(const Host& h, const HostTiled& s, int which)
{
    const int B = h.bs;
    const int RPC = kWave / B;
    const int64_t BB = static_cast<int64_t>(B) * B;
    const int KMAX = s.kmax;
    if (!(KMAX == 3 || KMAX == 6 || KMAX == 9)) return false;
    if (B >= 5 && KMAX != 3) return false;
    const bool fuse = (which == BILU_SWEEP_U || which == BILU_SWEEP_LT);
    const int64_t n_rows_arr = static_cast<int64_t>(s.rows.size());
    const int64_t n_slots_arr = static_cast<int64_t>(s.deps.size());
    const int64_t n_vals = n_slots_arr * BB;
    const int64_t n_dinv = static_cast<int64_t>(s.nchunks) * RPC * BB;
    const int64_t vec_bytes = static_cast<int64_t>(h.nb) * B * 8;
    const int G = s.group;
    if (s.ring > 0 && G != 1) return false;
    // the member tiles' rows (or the ring's) + the zero row (progress counters follow)
    const int64_t lds_rows = s.ring > 0 ? static_cast<int64_t>(s.ring) * RPC : static_cast<int64_t>(G) * s.tile_rows;
    const int64_t lds_bytes = (lds_rows + 1) * B * 8;
    if (vec_bytes > INT32_MAX) return false;
    if (G < 1 || G > kGroupMax) return false;
    auto in = [](int64_t i, int64_t n) { return i >= 0 && i < n; };
    auto in8 = [](int64_t byte, int64_t nbytes) { return byte >= 0 && byte % 8 == 0 && byte + 8 <= nbytes; };
    // k_sweep_grouped: member m of group g sweeps group_tiles[g*G + m]
    if (G > 1 && static_cast<int64_t>(s.group_tiles.size()) != static_cast<int64_t>(s.ngroups) * G) return false;
    std::vector<int> member_of(static_cast<size_t>(s.ntiles), 0);
    if (G > 1)
        for (int64_t e = 0; e < static_cast<int64_t>(s.group_tiles.size()); ++e) {
            const int t = s.group_tiles[e];
            if (t < -1 || t >= s.ntiles) return false;
            if (t >= 0) member_of[t] = static_cast<int>(e % G);
        }
    for (int t = 0; t < s.ntiles; ++t) {
        const int lo = s.tile_lo[t];
        const int64_t own = static_cast<int64_t>(member_of[t]) * s.tile_rows;   // first LDS row of the tile
        for (int c = s.tile_chunk_ptr[t]; c < s.tile_chunk_ptr[t + 1]; ++c) {
            if (G > 1 && !in(static_cast<int64_t>(c) * kGroupMax + kGroupMax - 1,
                             static_cast<int64_t>(s.chunk_wait.size())))
                return false;
            const int64_t off = s.chunk_off[c];
            const int w = static_cast<int>((s.chunk_off[c + 1] - off) / RPC);
            if (w < KMAX) return false;
            for (int lane = 0; lane < kWave; ++lane) {
                const int q = lane / B, r = lane - q * B;
                const bool lane_ok = q < RPC;
                const int qc = lane_ok ? q : RPC - 1;
                const int64_t lane_off = static_cast<int64_t>(r) * RPC + qc;
                const int64_t ri = static_cast<int64_t>(c) * RPC + qc;          // tile_meta
                if (!in(ri, n_rows_arr)) return false;
                const int row = s.rows[ri];
                std::vector<int32_t> code(static_cast<size_t>(KMAX));
                for (int k = 0; k < KMAX; ++k) {
                    const int64_t di = off + static_cast<int64_t>(k) * RPC + qc;
                    if (!in(di, n_slots_arr)) return false;
                    code[k] = s.deps[di];                                   // tile_data
                    const int64_t vb = off * BB + k * RPC * BB + lane_off;
                    if (!in(vb, n_vals) || !in(vb + static_cast<int64_t>(B - 1) * B * RPC, n_vals)) return false;
                }
                const int64_t rowc_b = static_cast<int64_t>(row >= 0 ? row : 0) * B * 8;
                if (!in8(rowc_b, vec_bytes) || !in8(rowc_b + (B - 1) * 8, vec_bytes)) return false;
                if (fuse) {
                    const int64_t db = static_cast<int64_t>(c) * RPC * BB + lane_off;
                    if (!in(db, n_dinv) || !in(db + static_cast<int64_t>(B - 1) * B * RPC, n_dinv)) return false;
                }
                for (int k = 0; k < KMAX; ++k) {
                    const int64_t xb = code[k] >= 0 ? code[k] : 0;
                    if (!in8(xb, vec_bytes) || !in8(xb + (B - 1) * 8, vec_bytes)) return false;
                    const int64_t lb = code[k] < 0 ? (code[k] & INT32_MAX) : 0;     // tile_compute
                    if (!in8(lb, lds_bytes) || !in8(lb + (B - 1) * 8, lds_bytes)) return false;
                }
                if (!lane_ok || row < 0) continue;
                for (int k = KMAX; k < w; ++k) {                                // unpipelined slots
                    const int64_t sl = off + static_cast<int64_t>(k) * RPC;
                    if (!in(sl + qc, n_slots_arr)) return false;
                    const int32_t cd = s.deps[sl + qc];
                    const int64_t b0 = cd < 0 ? (cd & INT32_MAX) : cd;
                    if (!in8(b0, cd < 0 ? lds_bytes : vec_bytes) ||
                        !in8(b0 + (B - 1) * 8, cd < 0 ? lds_bytes : vec_bytes))
                        return false;
                    const int64_t vb = sl * BB + lane_off;
                    if (!in(vb + static_cast<int64_t>(B - 1) * B * RPC, n_vals)) return false;
                }
                if (!in8((static_cast<int64_t>(row) * B + r) * 8, vec_bytes)) return false;
                if (!s.block_ny && (row - lo < 0 || row - lo >= s.tile_rows)) return false;
                if (s.block_ny && s.ring < 1) return false;
                const int64_t wrow = s.ring > 0 ? ((c - s.tile_chunk_ptr[t]) % s.ring) * RPC + qc : own + row - lo;
                if (!in8((wrow * B + r) * 8, lds_bytes - B * 8)) return false;
            }
        }
    }
    return true;
}
}  // namespace

int validate_layout(const Host& h)
{
    for (int w = 0; w < 4; ++w)
        if (h.lines[w].built && validate_line_layout(h, h.lines[w]) != BILU_OK) return BILU_ERR_STATE;
    const int nb = h.nb;
    const int64_t nP = static_cast<int64_t>(h.Pj.size());
    for (int w = 0; w < 4; ++w) {
        const HostSweep& s = h.sweep[w];
        if (!s.built) continue;
        const int rpc = s.rpc;
        if (rpc < 1 || rpc * h.bs > kWave) return BILU_ERR_STATE;
        if (static_cast<int>(s.chunk_off.size()) != s.nchunks + 1 || s.chunk_off[0] != 0) return BILU_ERR_STATE;
        if (static_cast<int64_t>(s.rows.size()) != static_cast<int64_t>(s.nchunks) * rpc) return BILU_ERR_STATE;
        if (s.chunk_off.back() != s.nslots || static_cast<int64_t>(s.cols.size()) != s.nslots ||
            static_cast<int64_t>(s.src.size()) != s.nslots)
            return BILU_ERR_STATE;
        if (static_cast<int>(s.level_chunk_ptr.size()) != s.nlev + 1 || s.level_chunk_ptr[0] != 0 ||
            s.level_chunk_ptr[s.nlev] != s.nchunks)
            return BILU_ERR_STATE;
        for (int l = 0; l < s.nlev; ++l)
            if (s.level_chunk_ptr[l + 1] < s.level_chunk_ptr[l]) return BILU_ERR_STATE;
        std::vector<int32_t> chunk_of(static_cast<size_t>(nb), -1);
        for (int c = 0; c < s.nchunks; ++c) {
            const int64_t span = s.chunk_off[c + 1] - s.chunk_off[c];
            if (span < 0 || span % rpc != 0) return BILU_ERR_STATE;
            for (int q = 0; q < rpc; ++q) {
                const int32_t r = s.rows[static_cast<size_t>(c) * rpc + q];
                if (r < -1 || r >= nb) return BILU_ERR_STATE;
                if (r >= 0) {
                    if (chunk_of[r] != -1) return BILU_ERR_STATE;
                    chunk_of[r] = c;
                }
            }
        }
        for (int i = 0; i < nb; ++i)
            if (chunk_of[i] < 0) return BILU_ERR_STATE;
        // dependency count per row straight from the pattern
        std::vector<int32_t> ndep(static_cast<size_t>(nb), 0);
        for (int32_t i = 0; i < nb; ++i)
            for (int32_t e = h.Pp[i]; e < h.Pp[i + 1]; ++e) {
                const int32_t j = h.Pj[e];
                if (w == BILU_SWEEP_L && j < i) ndep[i]++;
                if (w == BILU_SWEEP_U && j > i) ndep[i]++;
                if (w == BILU_SWEEP_UT && j > i) ndep[j]++;
                if (w == BILU_SWEEP_LT && j < i) ndep[j]++;
            }
        for (int c = 0; c < s.nchunks; ++c) {
            const int64_t off = s.chunk_off[c];
            const int64_t width = (s.chunk_off[c + 1] - off) / rpc;
            for (int q = 0; q < rpc; ++q) {
                const int32_t r = s.rows[static_cast<size_t>(c) * rpc + q];
                int32_t seen = 0;
                for (int64_t k = 0; k < width; ++k) {
                    const int64_t slot = off + k * rpc + q;
                    const int32_t j = s.cols[slot];
                    const int64_t e = s.src[slot];
                    if (j == -1 && e == -1) continue;
                    if (r < 0 || j < 0 || j >= nb || e < 0 || e >= nP) return BILU_ERR_STATE;
                    if (chunk_of[j] >= c) return BILU_ERR_STATE;        // must be strictly earlier
                    const bool rowwise = (w == BILU_SWEEP_L || w == BILU_SWEEP_U);
                    const int32_t pi = h.Prow[e], pj = h.Pj[e];
                    if (rowwise ? (pi != r || pj != j) : (pi != j || pj != r)) return BILU_ERR_STATE;
                    ++seen;
                }
                if (r >= 0 && seen != ndep[r]) return BILU_ERR_STATE;
            }
        }
    }
    for (int w = 0; w < 4; ++w) {
        const HostTiled& s = h.tiled[w];
        if (!s.built) continue;
        const int rpc = s.rpc;
        const bool forward = (w == BILU_SWEEP_L || w == BILU_SWEEP_UT);
        const bool rowwise = (w == BILU_SWEEP_L || w == BILU_SWEEP_U);
        if (rpc < 1 || rpc * h.bs > kWave || s.tile_rows < 1) return BILU_ERR_STATE;
        if (static_cast<int>(s.tile_chunk_ptr.size()) != s.ntiles + 1 || s.tile_chunk_ptr[0] != 0 ||
            s.tile_chunk_ptr[s.ntiles] != s.nchunks || static_cast<int>(s.tile_lo.size()) != s.ntiles)
            return BILU_ERR_STATE;
        if (static_cast<int>(s.chunk_off.size()) != s.nchunks + 1 || s.chunk_off[0] != 0 ||
            s.chunk_off.back() != s.nslots || static_cast<int64_t>(s.deps.size()) != s.nslots ||
            static_cast<int64_t>(s.src.size()) != s.nslots ||
            static_cast<int64_t>(s.rows.size()) != static_cast<int64_t>(s.nchunks) * rpc)
            return BILU_ERR_STATE;
        if (static_cast<int64_t>(nb) * h.bs * 8 > INT32_MAX) return BILU_ERR_STATE;
        // groups: the arithmetic numbering, every tile in exactly one slot
        const int G = s.group;
        if (G < 1 || G > kGroupMax || s.gstride < 1) return BILU_ERR_STATE;
        const TileGroups tg{G, s.gstride, s.ntiles};
        if (s.ngroups != tg.count() || static_cast<int64_t>(s.group_tiles.size()) != static_cast<int64_t>(s.ngroups) * G)
            return BILU_ERR_STATE;
        if (G > 1 ? static_cast<int64_t>(s.chunk_wait.size()) != static_cast<int64_t>(s.nchunks) * kGroupMax
                  : !s.chunk_wait.empty())
            return BILU_ERR_STATE;
        {
            std::vector<char> placed(static_cast<size_t>(s.ntiles), 0);
            for (int g = 0; g < s.ngroups; ++g)
                for (int m = 0; m < G; ++m) {
                    const int t = s.group_tiles[static_cast<size_t>(g) * G + m];
                    if (t != tg.tile(g, m)) return BILU_ERR_STATE;
                    if (t < 0) continue;
                    if (placed[t] || tg.group(t) != g || tg.member(t) != m) return BILU_ERR_STATE;
                    placed[t] = 1;
                }
            for (int t = 0; t < s.ntiles; ++t)
                if (!placed[t]) return BILU_ERR_STATE;
        }
        const int32_t row_bytes = h.bs * 8;
        if (s.ring < 0 || s.ring >= kRingMax + 1 || (s.ring > 0 && G != 1)) return BILU_ERR_STATE;
        const int32_t pad_code = tiled_local_code(s.ring > 0 ? s.ring * rpc : G * s.tile_rows, h.bs);
        std::vector<int32_t> tile_of(static_cast<size_t>(nb), -1), chunk_of(static_cast<size_t>(nb), -1);
        for (int t = 0; t < s.ntiles; ++t) {
            const int lo = s.tile_lo[t];
            if (lo < 0 || lo >= nb) return BILU_ERR_STATE;
            if (s.tile_chunk_ptr[t + 1] < s.tile_chunk_ptr[t]) return BILU_ERR_STATE;
            for (int c = s.tile_chunk_ptr[t]; c < s.tile_chunk_ptr[t + 1]; ++c) {
                const int64_t span = s.chunk_off[c + 1] - s.chunk_off[c];
                if (span < 0 || span % rpc != 0 || span / rpc < s.kmax) return BILU_ERR_STATE;
                for (int q = 0; q < rpc; ++q) {
                    const int32_t r = s.rows[static_cast<size_t>(c) * rpc + q];
                    if (r < -1 || r >= nb) return BILU_ERR_STATE;
                    if (r < 0) continue;
                    if (tile_of[r] != -1) return BILU_ERR_STATE;
                    if (!s.block_ny && (r < lo || r - lo >= s.tile_rows)) return BILU_ERR_STATE;
                    tile_of[r] = t;
                    chunk_of[r] = c;
                }
            }
        }
        for (int i = 0; i < nb; ++i)
            if (tile_of[i] < 0) return BILU_ERR_STATE;
        std::vector<int32_t> ndep(static_cast<size_t>(nb), 0), seen(static_cast<size_t>(nb), 0);
        for (int32_t i = 0; i < nb; ++i)
            for (int32_t e = h.Pp[i]; e < h.Pp[i + 1]; ++e) {
                const int32_t j = h.Pj[e];
                if (w == BILU_SWEEP_L && j < i) ndep[i]++;
                if (w == BILU_SWEEP_U && j > i) ndep[i]++;
                if (w == BILU_SWEEP_UT && j > i) ndep[j]++;
                if (w == BILU_SWEEP_LT && j < i) ndep[j]++;
            }
        for (int t = 0; t < s.ntiles; ++t) {
            const int mt = tg.member(t);
            const int gt = tg.group(t);
            for (int c = s.tile_chunk_ptr[t]; c < s.tile_chunk_ptr[t + 1]; ++c) {
                const int64_t off = s.chunk_off[c];
                const int64_t width = (s.chunk_off[c + 1] - off) / rpc;
                // waits: only on earlier members, never past their last chunk
                for (int m = 0; G > 1 && m < kGroupMax; ++m) {
                    const int32_t need = s.chunk_wait[static_cast<size_t>(c) * kGroupMax + m];
                    if (need == 0) continue;
                    if (need < 0 || m >= mt) return BILU_ERR_STATE;
                    const int tm = tg.tile(gt, m);
                    if (tm < 0 || need > s.tile_chunk_ptr[tm + 1] - s.tile_chunk_ptr[tm]) return BILU_ERR_STATE;
                }
                for (int q = 0; q < rpc; ++q) {
                    const int32_t r = s.rows[static_cast<size_t>(c) * rpc + q];
                    for (int64_t k = 0; k < width; ++k) {
                        const int64_t slot = off + k * rpc + q;
                        const int32_t code = s.deps[slot];
                        const int64_t e = s.src[slot];
                        if (code == pad_code && e == -1) continue;
                        if (r < 0 || code == pad_code || e < 0 || e >= nP) return BILU_ERR_STATE;
                        int32_t j;
                        if (code < 0) {          // the group's LDS: byte offset of the row
                            const int32_t off = code & INT32_MAX;
                            if (off % row_bytes != 0) return BILU_ERR_STATE;
                            const int32_t lr = off / row_bytes;
                            int tj;
                            if (s.ring > 0) {
                                // the row last written to LDS row lr before chunk c
                                if (lr >= s.ring * rpc) return BILU_ERR_STATE;
                                const int k = c - s.tile_chunk_ptr[t];
                                const int sc = lr / rpc;
                                const int kp = k - 1 - (((k - 1 - sc) % s.ring) + s.ring) % s.ring;
                                if (kp < 0) return BILU_ERR_STATE;
                                tj = t;
                                j = s.rows[static_cast<size_t>(s.tile_chunk_ptr[t] + kp) * rpc + lr % rpc];
                            } else {
                                const int mj = lr / s.tile_rows;
                                if (mj >= G) return BILU_ERR_STATE;
                                tj = tg.tile(gt, mj);
                                if (tj < 0) return BILU_ERR_STATE;
                                j = s.tile_lo[tj] + lr % s.tile_rows;
                            }
                            if (j < 0 || j >= nb || tile_of[j] != tj) return BILU_ERR_STATE;
                            const int mj = tg.member(tj);
                            if (tj == t) {
                                if (chunk_of[j] >= c) return BILU_ERR_STATE;
                            } else {             // an earlier member, covered by the chunk's wait
                                if (mj >= mt) return BILU_ERR_STATE;
                                const int32_t need = s.chunk_wait[static_cast<size_t>(c) * kGroupMax + mj];
                                if (need < chunk_of[j] - s.tile_chunk_ptr[tj] + 1) return BILU_ERR_STATE;
                            }
                        } else {                 // another group: byte offset of the row
                            if (code % row_bytes != 0) return BILU_ERR_STATE;
                            j = code / row_bytes;
                            // a tile of a group with a smaller ticket
                            if (j >= nb || tg.group(tile_of[j]) >= gt) return BILU_ERR_STATE;
                        }
                        if (forward ? j >= r : j <= r) return BILU_ERR_STATE;
                        const int32_t pi = h.Prow[e], pj = h.Pj[e];
                        if (rowwise ? (pi != r || pj != j) : (pi != j || pj != r)) return BILU_ERR_STATE;
                        ++seen[r];
                    }
                }
            }
        }
        for (int i = 0; i < nb; ++i)
            if (seen[i] != ndep[i]) return BILU_ERR_STATE;
        if (!tiled_accesses_in_bounds(h, s, w)) return BILU_ERR_STATE;
        if (s.block_ny && s.ring < 1) return BILU_ERR_STATE;
        if (w == BILU_SWEEP_U && G == 1 && !s.block_ny) {   // the order of the U' sweep fused with the SpMV
            std::vector<int32_t> sched;
            if (build_fused_schedule(h, s, sched) != BILU_OK) return BILU_ERR_STATE;
        }
    }
    return BILU_OK;
}

int build_fused_schedule(const Host& h, const HostTiled& u, std::vector<int32_t>& sched)
{
    if (u.group != 1) return BILU_ERR_STATE;      // tickets of single tiles only
    sched.clear();
    if (!u.built || u.which != BILU_SWEEP_U) return BILU_ERR_STATE;
    const int nb = h.nb;
    const int rpc = u.rpc;
    const int T = u.ntiles;
    // tile of a row in the backward sweep
    auto tile_of = [&](int32_t j) { return (nb - 1 - j) / u.tile_rows; };
    for (int t = 0; t < T; ++t) {
        const int hi = nb - 1 - t * u.tile_rows;     // backward tiles: the last one may be short
        const int lo = u.tile_lo[t];
        if (lo != std::max(0, hi - u.tile_rows + 1) || tile_of(lo) != t || tile_of(hi) != t) return BILU_ERR_STATE;
    }
    const int nblocks = (nb + rpc - 1) / rpc;
    std::vector<std::vector<int32_t>> after(static_cast<size_t>(T));
    for (int b = 0; b < nblocks; ++b) {
        int32_t minj = nb;
        for (int32_t i = b * rpc; i < std::min(nb, (b + 1) * rpc); ++i)
            for (int32_t e = h.Ap[i]; e < h.Ap[i + 1]; ++e) minj = std::min(minj, h.Aj[e]);
        after[static_cast<size_t>(tile_of(minj))].push_back(b);
    }
    // every tile first, so that no tile waits for a wavefront held by an
    // SpMV block; then the blocks in the order their tiles finish
    for (int t = 0; t < T; ++t) sched.push_back(t);
    for (int t = 0; t < T; ++t)
        for (int32_t b : after[t]) sched.push_back(-1 - b);
    // check: tiles once and in order; every block once, after every tile
    // holding a row it reads
    std::vector<int32_t> seen_b(static_cast<size_t>(nblocks), 0);
    int next_tile = 0;
    for (int32_t it : sched) {
        if (it >= 0) {
            if (it != next_tile) return BILU_ERR_STATE;
            ++next_tile;
            continue;
        }
        const int b = -1 - it;
        if (b >= nblocks || seen_b[b]++) return BILU_ERR_STATE;
        for (int32_t i = b * rpc; i < std::min(nb, (b + 1) * rpc); ++i)
            for (int32_t e = h.Ap[i]; e < h.Ap[i + 1]; ++e)
                if (tile_of(h.Aj[e]) >= next_tile) return BILU_ERR_STATE;
    }
    if (next_tile != T) return BILU_ERR_STATE;
    for (int32_t v : seen_b)
        if (v != 1) return BILU_ERR_STATE;
    return BILU_OK;
}

}  // namespace bilu
