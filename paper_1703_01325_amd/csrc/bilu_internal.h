// Internal state shared by the host analysis (analysis.cpp) and the GPU
// side (bilu_api.hip).  Not part of the ABI.
#pragma once

#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

#include "bilu.h"

namespace bilu {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxBs = 32;          // block sizes the library accepts
constexpr int kMaxKernelBs = 8;     // block sizes with block-row sweep and SpMV kernels;
                                    // larger ones sweep at point granularity

// Rows of a sweep grouped for the GPU: level by level (Eq 4), a level's rows
// cut into chunks of `rpc` rows (one wavefront each), chunk c holding
// w_c = (chunk_off[c+1]-chunk_off[c]) / rpc dependency slots per row.
// Slot (c, k, q) = chunk_off[c] + k*rpc + q is the k-th dependency of the
// q-th row of the chunk: cols[] names the row it reads, src[] the position
// of the factor block in the pattern P (-1: padding).
struct HostSweep {
    bool built = false;
    int which = 0;
    int nlev = 0;
    int rpc = 0;
    int nchunks = 0;
    int64_t nslots = 0;
    bool transposed_blocks = false;        // U'^T and L^T read blocks transposed
    std::vector<int32_t> level_ptr;        // [nlev+1]  canonical level sets
    std::vector<int32_t> level_rows;       // [nb]      rows ascending in a level
    std::vector<int32_t> level_chunk_ptr;  // [nlev+1]  first chunk of each level
    std::vector<int64_t> chunk_off;        // [nchunks+1] slot offsets
    std::vector<int32_t> rows;             // [nchunks*rpc] row ids, -1 = idle lane
    std::vector<int32_t> cols;             // [nslots]
    std::vector<int64_t> src;              // [nslots]
};

// Tiled form of a sweep: tile t is a contiguous range of block rows
// [tile_lo[t], tile_lo[t] + size), tiles numbered in sweep order (ascending
// rows for forward sweeps, descending for backward ones).  The rows of a
// tile are ordered by their level inside the tile (Eq 4 over dependencies
// within the tile only) and cut into chunks of rpc rows of one such level;
// chunk slots as in HostSweep, with deps[] holding the byte-offset codes
// below (tiled_global_code / tiled_local_code).
struct HostTiled {
    bool built = false;
    int which = 0;
    int rpc = 0;
    int tile_rows = 0;
    int ntiles = 0;
    int nchunks = 0;
    int64_t nslots = 0;
    int kmax = 0;                          // dependency slots the kernel keeps in registers
    std::vector<int32_t> tile_chunk_ptr;   // [ntiles+1]
    std::vector<int32_t> tile_lo;          // [ntiles]
    std::vector<int64_t> chunk_off;        // [nchunks+1]
    std::vector<int32_t> rows;             // [nchunks*rpc]
    std::vector<int32_t> deps;             // [nslots]
    std::vector<int64_t> src;              // [nslots]
    // U' sweep fused with y = A x on its output (built on demand): ticket
    // order of tiles (>= 0) and SpMV blocks of rpc rows (-(1 + block))
    std::vector<int32_t> fused;
    // Tile groups (group > 1): the member tiles of a group run as the
    // wavefronts of one workgroup and share its LDS (TileGroups).  Codes of
    // rows in any member tile are local; chunk_wait[c*kGroupMax + m] is the
    // number of chunks member m must have finished before chunk c reads LDS.
    int ring = 0;                          // > 0: LDS ring of this many chunks (group 1 only)
    // line blocks (block_ny > 0): a tile is a block of block_ny x block_nz
    // grid lines (rows of nx consecutive block rows), not a contiguous row
    // range; tile-local rows are always addressed through the LDS ring, and
    // tile_lo holds the tile's first row only
    int block_ny = 0, block_nz = 0;
    // line sweep (lines = true): tiles are blocks of block_ny x block_nz grid
    // lines swept one diagonal per step by k_sweep_lines; chunk
    // b*line_steps + s holds step s of block b, row slot q = line, slot k =
    // the neighbour along dimension line_dim[k] of the sweep coordinates
    bool lines = false;
    int line_nx = 0, line_ny = 0, line_nz = 0, line_steps = 0, line_NYb = 0;
    int line_dim[3] = {0, 0, 0};
    int group = 1;
    int group_req = 1;                     // the group size asked of build_tiled
    int gstride = 1;
    int ngroups = 0;
    std::vector<int32_t> group_tiles;      // [ngroups*group], -1 past the last tile
    std::vector<int32_t> chunk_wait;       // [nchunks*kGroupMax], group > 1 only
};

constexpr int kGroupMax = 4;

// Tiles in sweep order, cut into blocks of G*D consecutive tiles; inside a
// block, tiles t0 + m*D (m = 0..G-1) form one group (member m).  On a grid
// whose planes hold D tiles, a group is a stack of G tiles in consecutive
// planes.  Groups are numbered block by block; only the last block can hold
// groups without member 0, and those are dropped, so 0..count()-1 are used.
struct TileGroups {
    int G = 1, D = 1, ntiles = 0;
    int member(int t) const { return (t % (G * D)) / D; }
    int group(int t) const { return (t / (G * D)) * D + (t % (G * D)) % D; }
    int tile(int g, int m) const
    {
        const int t = (g / D) * G * D + m * D + g % D;
        return t < ntiles ? t : -1;
    }
    int count() const
    {
        const int full = ntiles / (G * D);
        return full * D + std::min(D, ntiles - full * G * D);
    }
};

// LDS bytes of one workgroup of the tiled sweep: the member tiles' rows, the
// zero row, and (grouped) the members' progress counters.
inline int64_t tiled_lds_bytes(int tile_rows, int group, int bs)
{
    return (static_cast<int64_t>(group) * tile_rows + 1) * bs * 8 + (group > 1 ? kGroupMax * 4 : 0);
}

// Chunks held by the LDS ring through which a helper wavefront hands its
// member the values of other tiles, and the largest tile group that runs
// with helpers.
constexpr int kHelpRing = 4;
constexpr int kHelpGroupMax = 2;

// LDS bytes of a tile-group workgroup with helper wavefronts: the member
// tiles' rows, the zero row, progress and delivered counts, and each
// member's ring of kHelpRing chunks of kmax * bs values per lane.
inline int64_t helped_lds_bytes(int tile_rows, int group, int bs, int kmax)
{
    return (static_cast<int64_t>(group) * tile_rows + 1) * bs * 8 + 2 * kGroupMax * 4 +
           static_cast<int64_t>(group) * kHelpRing * kmax * bs * 64 * 8;
}

// Dependency slots per row that the tiled sweep kernel loads ahead into
// registers, from the widest chunk of the layout; wider rows finish their
// remaining slots unpipelined.  Register budget: 3 for blocks of 5..8,
// else 3, 6 or 9.
inline int tiled_kmax(int bs, int max_width)
{
    if (bs >= 5 || max_width <= 3) return 3;
    return max_width <= 6 ? 6 : 9;
}

// Dependency codes of the tiled layout are byte offsets: a row of another
// tile is j*bs*8 (>= 0, into the vectors), a row of the same tile is
// INT32_MIN | (local row)*bs*8 (into the tile's LDS).  Padding slots point at
// local row tile_rows, which the kernel keeps at zero, with zero factor
// values.  Every chunk has at least kmax slot rows.
inline int32_t tiled_global_code(int32_t j, int bs) { return j * bs * 8; }
inline int32_t tiled_local_code(int32_t local_row, int bs)
{
    return static_cast<int32_t>(0x80000000u | static_cast<uint32_t>(local_row * bs * 8));
}

struct DevSweep {
    int64_t* chunk_off = nullptr;
    int32_t* rows = nullptr;
    int32_t* cols = nullptr;  // level-chunk form: row read; tiled form: dependency code
    int64_t* src = nullptr;
    int32_t* tile_chunk_ptr = nullptr;
    int32_t* tile_lo = nullptr;
    int32_t* chunk_row = nullptr;  // tiled form: chunk_off / rpc (first slot row)
    int32_t* fused = nullptr;      // tiled U' form: fused sweep + SpMV ticket order
    int32_t* group_tiles = nullptr;  // tiled form: member tiles of each group
    int32_t* chunk_wait = nullptr;   // tiled form, grouped: waits of each chunk
    void* vals = nullptr;     // [nslots * bs*bs] FP64 or FP32, layout [k][c][r][q]
    void* dinv = nullptr;     // [nchunks*rpc * bs*bs] same layout, fused sweeps only
    int vals_precision = -1;  // precision the values were laid out in (-1: none)
    size_t vals_bytes = 0;    // allocated bytes of vals and dinv
    size_t dinv_bytes = 0;
};

struct Host {
    int nb = 0, bs = 0, k = 0, flags = 0;
    int rpc = 0;
    std::vector<int32_t> Ap, Aj;
    std::vector<int32_t> Arow;             // block row of each stored block of A
    std::vector<int32_t> Pp, Pj, Plev;     // ILU(k) pattern
    std::vector<int32_t> Pdiag;            // position of (i,i) in P
    std::vector<int32_t> Prow;             // block row of each entry of P
    std::vector<int64_t> AtoP;             // position in P of each stored block of A
    std::vector<int32_t> Pfill;            // positions of P not stored in A
    // A^T structure: row j lists the blocks (i, j) of A; ATsrc = their position in A
    std::vector<int32_t> ATp, ATj;
    std::vector<int64_t> ATsrc;
    // levels of each sweep from the device symbolic phase (empty: computed
    // on the host)
    std::vector<int32_t> dev_lvl[4];
    HostSweep sweep[4];
    HostTiled tiled[4];
    HostTiled lines[4];     // line-sweep layouts (L and U' only; see build_line_layout)
};

// Host analysis entry points (analysis.cpp).
int validate_pattern(int nb, const int32_t* Ap, const int32_t* Aj);
int symbolic_iluk(int nb, const int32_t* Ap, const int32_t* Aj, int k, std::vector<int32_t>& Pp,
                  std::vector<int32_t>& Pj, std::vector<int32_t>& Plev);
int sweep_levels(int nb, const std::vector<int32_t>& Pp, const std::vector<int32_t>& Pj,
                 int which, std::vector<int32_t>& lvl);
void build_sweep(const Host& h, int which, int rpc, HostSweep& out);
int analyze_host(Host& h, int nb, int bs, const int32_t* Ap, const int32_t* Aj, int k, int flags);
// The symbolic phase and the level sets of the first nsweeps sweeps run on
// the current GPU (symbolic.hip), results copied back (BILU_DEVICE_SYMBOLIC).
int device_analysis(int nb, const int32_t* Ap, const int32_t* Aj, int k, int nsweeps, std::vector<int32_t>& Pp,
                    std::vector<int32_t>& Pj, std::vector<int32_t>& Plev, std::vector<int32_t> (&lvl)[4]);
// Tiled layout of one sweep with tiles of tile_rows rows in groups of up to
// `group` tiles (falls back to smaller groups, down to 1, where a grouping
// would break the ticket order or the group's LDS exceeds lds_limit bytes).
// allow_ring: a layout of single tiles may keep only a ring of recent chunks'
// rows in LDS where the dependencies allow (HostTiled::ring).
void build_tiled(const Host& h, int which, int rpc, int tile_rows, int group, int64_t lds_limit, bool allow_ring,
                 HostTiled& out);
// Predicted duration (in units of `step`) of a tiled sweep with the given
// tile size and group size (forward sweeps may be restricted to their first
// row_limit rows; 0 = all); +inf where the grouping is not usable.
double simulate_tiled(const Host& h, int which, int rpc, int tile_rows, int group, double hop_in_steps,
                      int row_limit);
int choose_tile_rows(const Host& h, int rpc, int max_rows);
// Every candidate tile size with its predicted duration, best first (one
// wavefront per tile).
std::vector<std::pair<double, int>> rank_tile_rows(const Host& h, int rpc, int max_rows);
struct TileChoice {
    double t;
    int tile_rows;
    int group;
};
// Layout choices, preferred first: groups of the tile size with the shortest
// simulated single-tile schedule (the usable ones, whose workgroup LDS fits in
// lds_limit bytes, in a fixed order of group sizes), then every candidate
// tile size with one wavefront per tile, by simulated duration.  tile_req > 0
// fixes the tile size; group_req 1 leaves groups out, > 1 asks for that size.
std::vector<TileChoice> rank_tile_layouts(const Host& h, int rpc, int64_t lds_limit, int tile_req, int group_req);
int validate_layout(const Host& h);
// Grid lines of a pattern in natural order: nx (block rows per line) and
// nxy (per plane) when the rows without an L dependency on the previous row
// are exactly the multiples of nx, and those without one on the row nx back
// exactly the multiples of nxy; false otherwise.
bool grid_lines(const Host& h, int& nx, int& nxy);
// Tiled layout of one sweep whose tiles are blocks of ny_b x nz_b grid lines
// (tickets in sweep order of the blocks, plane by plane), one wavefront per
// tile, tile-local rows in an LDS ring.  Leaves out.built false where the
// pattern has no grid lines, a dependency crosses to a later block, or the
// in-tile dependencies span more chunks than the ring can hold.
void build_tiled_blocks(const Host& h, int which, int rpc, int ny_b, int nz_b, HostTiled& out);
// Line-sweep layout of sweep `which` (L or U') with blocks of ny_b x nz_b
// grid lines (ny_b*nz_b <= rpc): built only where the pattern is a 7-point
// ILU(0) pattern in natural grid order (every row depends on exactly the
// grid neighbours before it in the sweep); out.built stays false otherwise.
void build_line_layout(const Host& h, int which, int rpc, int ny_b, int nz_b, HostTiled& out);
// Host self-check of a line-sweep layout: every row once, at the chunk and
// slot the kernel computes, each slot's factor entry the neighbour the
// kernel reads, every neighbour either one step earlier in the block or in
// an earlier block.
int validate_line_layout(const Host& h, const HostTiled& s);
// Ticket order of the backward U' tiled sweep fused with the SpMV on its
// output: all tiles, then each block of rpc rows of A, ordered by the tile
// that finishes the lowest row the block reads.  Checked before it is
// returned.
int build_fused_schedule(const Host& h, const HostTiled& u, std::vector<int32_t>& sched);

}  // namespace bilu
