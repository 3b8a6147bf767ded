// Internal layout shared by the host library and the gfx950 kernels.
//
// Everything lives in one caller-owned device workspace.  Per box:
//   - two population buffers A/B, structure of arrays [19][nz][ny][sx]
//     (sx = x pitch rounded up to a 128-byte row), storing deviations
//     f_i - w_i rho0 (scaled for FP16); a buffer holds the post-collision
//     populations of the last step and the next step pulls from it;
//   - band tiles of 32x2x1 cells (64 cells = one wavefront): an epoch
//     stamp per tile (two sets, by buffer parity, so that a step's node pass
//     can run while the previous step's stream-collide still reads its set)
//     and, in tile-major order [tile][3][64], the velocity u
//     written by the band kernel in stamped tiles (and the spread force F
//     for inspection);
//   - with a viscosity contrast, two sets of inside bits [ceil(nz/64)][ny][nx]
//     (one 64-bit word per 64 cells of a column), by step parity.
// Per droplet, nodes are renumbered once (recursive coordinate bisection of
// the initial positions) into compact blocks of 64 (one wavefront), padded
// per droplet.  Node arrays are SoA over the padded global node index.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace iblb {

constexpr int Q = 19;
// Band tile: 32 consecutive cells along x, 2 along y, 1 along z (64 cells,
// one wavefront).  Population rows are contiguous along x and padded to
// 128-byte lines, so a tile reads and writes whole 128-byte lines of each
// FP32 population row, and the bulk kernel, which skips the band tiles,
// skips whole lines.
constexpr int TX = 32, TY = 2, TZ = 1;
constexpr int TXS = 5, TYS = 1, TZS = 0;  // log2 of the tile extents
constexpr int TILE_CELLS = TX * TY * TZ;
static_assert(TILE_CELLS == 64 && (1 << TXS) == TX && (1 << TYS) == TY && (1 << TZS) == TZ, "band tile");

// Band tile of cell (x, y, z) and the cell's place in it.
__host__ __device__ inline int64_t band_tile(int x, int y, int z, int tnx, int tny) {
    return ((int64_t)(z >> TZS) * tny + (y >> TYS)) * tnx + (x >> TXS);
}
__host__ __device__ inline int band_loc(int x, int y, int z) {
    return (((z & (TZ - 1)) << (TXS + TYS)) | ((y & (TY - 1)) << TXS) | (x & (TX - 1)));
}
constexpr int NB = 64;           // nodes per block
constexpr int TRI_CHUNK = 256;   // triangles per FP64 partial-sum chunk
constexpr int TREC = 20;         // per-triangle record: five four-vectors (A, n), (N/6, 0),
                                 // and the corner forces (f_c, 0) of corners c = 0, 1, 2
static_assert(TREC == 5 * 4, "triangle record = five four-vectors");
constexpr int K1_MAX_THREADS = 256; // launch bound of the bulk stream-collide kernel
constexpr int MAXP = 2048;          // cells of a node block's partial-spread region
constexpr int BREG = 8;
constexpr int MAXC = 16;           // node blocks recorded per band tile (more: the gather scans)
constexpr int SCAN_GROUP = 256;    // boxes with at most this many node blocks: the gather scans them all

// Whether the node pass records, per band tile, the blocks covering it (a
// box whose blocks one scan pass of the gather covers needs no records).
__host__ __device__ inline bool box_records(int blk_begin, int blk_end) {
    return blk_end - blk_begin > SCAN_GROUP;
}

// Tiles (of 1 << sh cells) that the cells lo .. lo + span - 1 of an axis of
// n cells fall into, each once: `count` consecutive tiles from `first`,
// counted modulo the axis's tile count ceil(n / 2^sh) on a periodic axis.
// Periodic: lo in [0, n); a run that wraps past the last cell continues in
// tile 0, and one that reaches back into its own first tile (or spans the
// whole axis) covers every tile.  Otherwise the cells lie in [0, n).
// span < 1 gives count 0.
struct TileRun {
    int first, count;
};
__host__ __device__ inline TileRun tile_run(int lo, int span, int n, int sh, bool per) {
    if (span < 1) return {0, 0};
    const int nt = (n + (1 << sh) - 1) >> sh;
    const int t0 = lo >> sh, end = lo + span - 1;
    if (!per || end < n) return {t0, (end >> sh) - t0 + 1};
    if (span >= n) return {0, nt};
    const int t1 = (end - n) >> sh;  // last tile after the wrap
    if (t1 >= t0) return {0, nt};
    return {t0, nt - t0 + t1 + 1};
}

// Item of workgroup w when a launch of n workgroups takes n items (node
// blocks, triangle chunks) in order: the dispatcher hands workgroups to the
// eight XCDs in turn (w on XCD w % 8), and this gives each XCD one
// contiguous range of items, so that neighbouring blocks, whose stencil
// regions and incident triangles overlap, share one L2.  A bijection of
// [0, n): XCD x takes [x q + min(x, r), ...) with q = n / 8, r = n % 8.
__host__ __device__ inline int xcd_item(int w, int n) {
    const int x = w & 7, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + (w >> 3);
}

// List positions of wave v (0..3) of workgroup b when a grid of g
// workgroups (a multiple of eight) takes a list of `count` entries: the
// workgroups of XCD b % 8 share one contiguous eighth of the list, each
// wave taking every (g / 2)-th position of it from its own start.
struct ListRange {
    int first, end, stride;
};
__host__ __device__ inline ListRange xcd_list_range(int b, int v, int g, int count) {
    const int x = b & 7;
    const int lo = (int)((int64_t)count * x / 8), hi = (int)((int64_t)count * (x + 1) / 8);
    return {lo + (b >> 3) * 4 + v, hi, g / 2};
}

// Velocity set in the library's order: 0 = rest, i and i+9 opposite (i=1..9).
__host__ __device__ constexpr int cx_of(int i) {
    constexpr int t[Q] = {0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0};
    return t[i];
}
__host__ __device__ constexpr int cy_of(int i) {
    constexpr int t[Q] = {0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1};
    return t[i];
}
__host__ __device__ constexpr int cz_of(int i) {
    constexpr int t[Q] = {0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1};
    return t[i];
}
__host__ __device__ constexpr int opp_of(int i) { return i == 0 ? 0 : (i <= 9 ? i + 9 : i - 9); }
// 1/3 at rest, 1/18 along the axes, 1/36 along face diagonals.
__host__ __device__ constexpr double w_of(int i) {
    return i == 0 ? 1.0 / 3.0
                  : ((cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i) + cz_of(i) * cz_of(i)) == 1
                         ? 1.0 / 18.0
                         : 1.0 / 36.0);
}

// Ten population planes of a box are addressed with 32-bit offsets from one
// base: their bytes may not exceed this.
constexpr int64_t BUF_MAX_PLANE_GROUP = 0xFFFFFFFFll;

enum : uint32_t { BIT_RHO = 1u, BIT_MACH = 2u, BIT_WALL = 4u, BIT_JUMP = 8u };

struct BoxDev {
    int32_t nx, ny, nz, zbc;
    int32_t sx;                 // x pitch (elements)
    int32_t tnx, tny, tnz;      // tiles per axis
    int64_t plane;              // elements per direction plane
    int32_t n_tiles, tile_base; // tile_base: first global tile (multiple of 64)
    int32_t blk_begin, blk_end; // node blocks of the box's droplets
    void *f[2];                 // population buffers
    void *Fband, *uband;        // [n_tiles][3][64] of Real
    void *ufull;                // [3][plane] u of every cell (testing mode) or null
    int32_t *stamp[2];          // [n_tiles] epoch stamps, one set per buffer parity
    double tau, rho0, g[3];
    double omega, guo;          // 1/tau, 1 - 1/(2 tau)
    double cells_rho0;          // nx*ny*nz*rho0
    double omega_in, guo_in;    // the same with tau_in (cells inside droplets)
    int32_t contrast, nzw;      // tau_in set; 64-bit words per column (ceil(nz/64))
    uint64_t *mask[2];          // [nzw][ny][nx] inside bits, one set per step parity
    double uw[4];               // moving walls: u_x, u_y at z = 0, then at z = nz
    int32_t moving, pad;        // some wall velocity is nonzero
};

struct DropDev {
    int32_t box, n_nodes, n_tris, n_exp;
    int32_t m_exp, node_off, blk_off, n_blocks;
    int32_t tri_off, chunk_off, n_chunks, pad;
    double sigma, A, xi, kvol, V0;
    double ref[3];              // origin for the FP64 volume sum
};

struct RowGroup {
    int32_t box, r0, r1;        // rows r = z*ny + y in [r0, r1)
    int32_t x0, x1;             // cells x0 <= x < x1 of those rows (x1 > nx: the padding too)
    int32_t pad[3];
};

struct TriChunk {
    int32_t drop, t0, t1, pad;  // global triangle range
};

struct DevPtrs {
    BoxDev *boxes;
    DropDev *drops;
    int32_t n_boxes, n_drops;
    // node arrays, SoA [3][Ntot] unless stated
    void *qh, *ql;              // position, high and low parts (Real)
    void *phi;                  // nodal force (Real)
    void *trec;                 // [Ttot][TREC] per-triangle records (Real)
    int32_t *tile_list;         // [total_tiles][2]: stamped tiles of the epoch (global id, box)
    int32_t *tile_count;        // [2] list lengths, indexed by epoch parity
    void *wgt;                  // [12][Ntot] Peskin weights x0..3,y0..3,z0..3 (Real)
    int32_t *base;              // floor(q - 1/2), unwrapped
    int32_t *s0;                // first stencil cell base-1, wrapped where periodic
    int32_t *bbox;              // [6][nblk]: x0,x1,y0,y1,z0,z1 of stencil cells
    int32_t *breg;              // [nblk][BREG]: partial region x0,y0,z0 (wrapped), ex,ey,ez, overflow
    void *part;                 // [nblk][3][MAXP] partial spread regions (Real)
    int32_t *blk_drop;          // [nblk][2]: droplet and box of each node block
    int32_t *tri;               // [Ttot][3] global node ids
    int32_t *csr_off;           // [Ntot+1]
    int32_t *csr_ent;           // [3 Ttot]: 3*t + corner
    TriChunk *chunks;
    double *tri_part;           // [2][n_chunks]: volume, area
    RowGroup *rows;
    int32_t *tchunk_box;        // [total_tiles/64] box of each 64-tile chunk
    int32_t *tcand;             // [total_tiles][MAXC] node blocks whose stencil box covers the tile
    int32_t *tncand;            // [2][total_tiles] their number, by epoch parity
    int32_t *scan_all;          // [2][n_boxes] some block of the box could not record its tiles
    int32_t *ctr;               // step epoch
    int32_t *step_epoch;        // [2] epoch of the last node pass, by buffer parity
    uint32_t *status;
    double *obs_part;           // observables scratch
    double *obs_out;            // per droplet [12], per box [2]
    int32_t Ntot, nblk, Ttot, n_chunks;
    int32_t n_rowgroups, total_tiles, obs_groups, n_cus;  // n_cus: compute units of the device
    int32_t contrast;           // some box has tau_in set
    int32_t moving;             // some box has a moving wall
    int32_t mask_words;         // largest nzw*ny*nx over those boxes
    int32_t pad_rows;           // some row group runs into its row's padding (x1 > nx)
};

// Launch entry points (iblb_fluid.hip, iblb_mesh.hip).
struct Launch {
    int bx, by;                 // bulk stream-collide block shape
    int grid;                   // bulk stream-collide grid (<= n_rowgroups)
    int nt;                     // bulk stream-collide writes with streaming stores
    int cpt;                    // rows per thread and row group pass (1 or 2; 2 needs bx % 64 == 0)
    int maxg;                   // cap on the grid (0: one workgroup per row group)
    int after;                  // step schedule: 0 = the band kernel beside the bulk kernel, which
                                // skips the band tiles; 1 = the bulk kernel over every cell beside
                                // the mesh chain, then the band kernel over its band tiles
};

hipError_t launch_tri(const DevPtrs &P, bool f64, hipStream_t s);
hipError_t launch_set_v0(const DevPtrs &P, bool f64, hipStream_t s);
hipError_t launch_node(const DevPtrs &P, bool f64, int mode, int parity, hipStream_t s);
hipError_t launch_bulk(const DevPtrs &P, int storage, int parity, int full_u, float scale,
                       const Launch &L, bool skip_band, hipStream_t s);
hipError_t launch_band(const DevPtrs &P, int storage, int parity, int full_u, float scale,
                       bool collide, int nt, hipStream_t s);
hipError_t launch_interp(const DevPtrs &P, bool f64, int mode, double *Uout, hipStream_t s);
hipError_t launch_epoch(const DevPtrs &P, hipStream_t s);
hipError_t launch_inside(const DevPtrs &P, bool f64, int slot, hipStream_t s);
hipError_t launch_mask_clear(const DevPtrs &P, int slot, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_box_obs(const DevPtrs &P, int storage, int parity, float inv_scale,
                          hipStream_t s);
hipError_t launch_drop_obs(const DevPtrs &P, bool f64, hipStream_t s);

// vol, area, zmin, zmax, cx, cy, cz, rsum, count, then the volume moments
// about the node mean m: V, int (x-m), int (x-m)(x-m)^T (xx yy zz xy xz yz)
constexpr int OBS_DROP = 20;
constexpr int OBS_BOX = 2;   // mass, max_u
constexpr int OBS_GROUPS = 512;

}  // namespace iblb
