// Host side of the C ABI declared in include/iblb.h: validation, workspace
// layout, mesh preparation (node renumbering, node -> triangle CSR), uploads,
// step enqueueing and hipGraph replay, observables and state I/O.
#include "iblb.h"
#include "iblb_internal.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

using namespace iblb;

// Fixed device scratch of iblb_step_static: the per-step arrays of the
// spreading (triangle records and FP64 partial sums, node-block bounding
// boxes, region descriptors and partial regions, stamped-tile list and its
// lengths, per-tile block records) for callers that cannot allocate.  Each
// device holds its own copy from the library's load until the process ends.
// Host code never uses this name as an address: each device's address comes
// from hipGetSymbolAddress, taken once per device at iblb_init.
constexpr size_t SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on device dev (current), looked up once.
hipError_t scratch_address(int dev, char **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

thread_local std::string g_last_error = "no error";

constexpr size_t ALIGN = 256;
constexpr size_t BIG_ALIGN = 2u << 20;
// Steps per multi-step graph.  A run takes the longest that fits at each
// point.  The first step of a graph cannot overlap its node pass with a bulk
// kernel: a graph launch waits for the previous graph, whose last bulk
// kernel is still running.  With the shorter lengths a run of 20 steps
// replays two graphs instead of twenty single steps.
constexpr int MULTI_LEN[] = {32, 16, 8, 4, 2};
constexpr int N_MULTI = (int)(sizeof(MULTI_LEN) / sizeof(MULTI_LEN[0]));

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int elem_bytes(int storage) { return storage == IBLB_F64 ? 8 : (storage == IBLB_F32 ? 4 : 2); }

struct DropHost {
    iblb_droplet d{};
    std::vector<int32_t> perm;  // internal node k -> caller's node id
    std::vector<int32_t> inv;   // caller's node id -> internal node k
    std::vector<double> nodes;  // caller's order, copy of the input
    std::vector<int32_t> tris;  // caller's triangles (caller's node ids)
    int node_off = 0, blk_off = 0, n_blocks = 0, tri_off = 0, chunk_off = 0, n_chunks = 0;
    double A = 0.0, ref[3] = {0, 0, 0};
};

struct BoxHost {
    iblb_box b{};
    int sx = 0, tnx = 0, tny = 0, tnz = 0, n_tiles = 0, tile_base = 0;
    int64_t plane = 0;
    int blk_begin = 0, blk_end = 0;
    size_t off_f[2] = {0, 0}, off_stamp[2] = {0, 0}, off_F = 0, off_u = 0, off_ufull = 0;
    size_t off_mask[2] = {0, 0};
    int nzw = 0;  // 64-bit mask words per column (boxes with tau_in)
};

struct Plan {
    int storage = IBLB_F32;
    uint32_t flags = 0;
    double scale = 1.0;
    int real = 4;  // bytes of the compute type
    std::vector<BoxHost> boxes;
    std::vector<DropHost> drops;
    int Ntot = 0, nblk = 0, Ttot = 0, n_chunks = 0, total_tiles = 0;
    size_t max_rows = 0;  // capacity of the bulk row-group table
    bool any_kvol = false;
    // workspace offsets
    size_t off_boxes = 0, off_drops = 0, off_qh = 0, off_ql = 0, off_phi = 0, off_wgt = 0,
           off_trec = 0, off_tile_list = 0, off_tile_count = 0, off_part = 0, off_breg = 0,
           off_base = 0, off_s0 = 0, off_bbox = 0, off_blk_drop = 0, off_tri = 0,
           off_csr_off = 0, off_csr_ent = 0, off_chunks = 0, off_tri_part = 0, off_rows = 0,
           off_tchunk = 0, off_tcand = 0, off_tncand = 0, off_scan = 0, off_ctr = 0, off_step_epoch = 0, off_status = 0, off_obs_part = 0,
           off_obs_out = 0,
           off_uout = 0, total = 0;
    // the same per-step arrays inside the fixed scratch (iblb_step_static)
    size_t st_trec = 0, st_tri_part = 0, st_bbox = 0, st_breg = 0, st_part = 0, st_tile_list = 0,
           st_tile_count = 0, st_tcand = 0, st_tncand = 0, st_scan = 0, st_total = 0;
};

bool finite(double v) { return std::isfinite(v); }

iblb_status fail(std::string *err, iblb_status code, const std::string &msg) {
    if (err) *err = msg;
    return code;
}

// Closed, manifold, consistently oriented: every directed edge once and its
// reverse once; no repeated corner; every node used.
iblb_status check_mesh(const iblb_droplet &d, int di, std::string *err) {
    const int N = d.n_nodes, T = d.n_tris;
    std::unordered_map<uint64_t, int> edges;
    edges.reserve((size_t)T * 3 * 2);
    std::vector<char> used(N, 0);
    for (int t = 0; t < T; ++t) {
        const int32_t *c = d.tris + 3 * t;
        for (int k = 0; k < 3; ++k)
            if (c[k] < 0 || c[k] >= N)
                return fail(err, IBLB_E_MESH, "droplet " + std::to_string(di) + ": triangle " +
                                                  std::to_string(t) + " has a node index out of range");
        if (c[0] == c[1] || c[1] == c[2] || c[0] == c[2])
            return fail(err, IBLB_E_MESH, "droplet " + std::to_string(di) + ": degenerate triangle " +
                                              std::to_string(t));
        for (int k = 0; k < 3; ++k) {
            used[c[k]] = 1;
            const uint64_t key = ((uint64_t)(uint32_t)c[k] << 32) | (uint32_t)c[(k + 1) % 3];
            if (++edges[key] != 1)
                return fail(err, IBLB_E_MESH, "droplet " + std::to_string(di) +
                                                  ": a directed edge occurs twice (non-manifold or "
                                                  "inconsistently oriented mesh)");
        }
    }
    for (const auto &e : edges) {
        const uint64_t rev = (e.first << 32) | (e.first >> 32);
        if (!edges.count(rev))
            return fail(err, IBLB_E_MESH, "droplet " + std::to_string(di) + ": mesh is not closed");
    }
    for (int j = 0; j < N; ++j)
        if (!used[j])
            return fail(err, IBLB_E_MESH, "droplet " + std::to_string(di) + ": node " +
                                              std::to_string(j) + " belongs to no triangle");
    // orientation: the enclosed volume must be positive (outward normals)
    double V = 0.0;
    for (int t = 0; t < T; ++t) {
        const double *a = d.nodes + 3 * d.tris[3 * t], *b = d.nodes + 3 * d.tris[3 * t + 1],
                     *c = d.nodes + 3 * d.tris[3 * t + 2];
        const double bc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2],
                              b[0] * c[1] - b[1] * c[0]};
        V += a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2];
    }
    if (!(V > 0))
        return fail(err, IBLB_E_MESH, "droplet " + std::to_string(di) +
                                          ": triangles are not counter-clockwise seen from outside");
    return IBLB_OK;
}

void rcb_order(const double *q, int32_t *ids, int n, int nblocks) {
    if (nblocks <= 1) {
        std::sort(ids, ids + n);
        return;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int k = 0; k < n; ++k)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], q[3 * ids[k] + a]);
            hi[a] = std::max(hi[a], q[3 * ids[k] + a]);
        }
    int ax = 0;
    for (int a = 1; a < 3; ++a)
        if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
    std::sort(ids, ids + n, [&](int32_t u, int32_t v) {
        const double qu = q[3 * u + ax], qv = q[3 * v + ax];
        return qu < qv || (qu == qv && u < v);
    });
    const int nl = nblocks / 2;
    rcb_order(q, ids, nl * NB, nl);
    rcb_order(q, ids + nl * NB, n - nl * NB, nblocks - nl);
}

iblb_status build_plan(const iblb_config *cfg, Plan &p, std::string *err) {
    if (!cfg) return fail(err, IBLB_E_INVAL, "config is NULL");
    if (cfg->n_boxes < 1 || !cfg->boxes) return fail(err, IBLB_E_INVAL, "need at least one box");
    if (cfg->n_droplets < 0 || (cfg->n_droplets > 0 && !cfg->droplets))
        return fail(err, IBLB_E_INVAL, "droplet array missing");
    if (cfg->storage < IBLB_F64 || cfg->storage > IBLB_BF16DEV)
        return fail(err, IBLB_E_INVAL, "unknown storage");
    if (cfg->flags & ~(uint32_t)(IBLB_FLAG_GRAPH | IBLB_FLAG_AUTOTUNE | IBLB_FLAG_FULL_U))
        return fail(err, IBLB_E_INVAL, "unknown flag bits");
    p.storage = cfg->storage;
    p.flags = cfg->flags;
    p.real = cfg->storage == IBLB_F64 ? 8 : 4;
    p.scale = 1.0;
    if (cfg->storage == IBLB_F16DEV) {
        int e = 0;
        const double m = std::frexp(cfg->dev_scale, &e);
        if (!(cfg->dev_scale > 0) || !finite(cfg->dev_scale) || m != 0.5 || cfg->dev_scale > 65536.0)
            return fail(err, IBLB_E_INVAL, "dev_scale must be a power of two in (0, 65536]");
        p.scale = cfg->dev_scale;
    }
    const int eb = elem_bytes(cfg->storage);
    p.boxes.resize(cfg->n_boxes);
    for (int b = 0; b < cfg->n_boxes; ++b) {
        const iblb_box &B = cfg->boxes[b];
        const std::string nm = "box " + std::to_string(b);
        if (B.nx < 1 || B.ny < 1 || B.nz < 1) return fail(err, IBLB_E_INVAL, nm + ": sizes must be >= 1");
        if (B.zbc != IBLB_Z_WALLS && B.zbc != IBLB_Z_PERIODIC)
            return fail(err, IBLB_E_INVAL, nm + ": unknown z boundary");
        if (!(B.tau > 0.5) || !finite(B.tau)) return fail(err, IBLB_E_INVAL, nm + ": tau must exceed 1/2");
        if (!(B.tau_in == 0.0 || (B.tau_in > 0.5 && finite(B.tau_in))))
            return fail(err, IBLB_E_INVAL, nm + ": tau_in must be 0 or exceed 1/2");
        for (int a = 0; a < 2; ++a) {
            const double lo = B.wall_lo[a], hi = B.wall_hi[a];
            if (!(finite(lo) && finite(hi) && std::fabs(lo) <= 0.1 && std::fabs(hi) <= 0.1))
                return fail(err, IBLB_E_INVAL, nm + ": wall velocities must be finite with |u| <= 0.1");
            if (B.zbc != IBLB_Z_WALLS && (lo != 0.0 || hi != 0.0))
                return fail(err, IBLB_E_INVAL, nm + ": moving walls need zbc = IBLB_Z_WALLS");
        }
        if (!(B.rho0 > 0) || !finite(B.rho0)) return fail(err, IBLB_E_INVAL, nm + ": rho0 must be > 0");
        for (int a = 0; a < 3; ++a)
            if (!finite(B.body_force[a])) return fail(err, IBLB_E_INVAL, nm + ": body force not finite");
        BoxHost &H = p.boxes[b];
        H.b = B;
        H.sx = (int)round_up((size_t)B.nx, 128 / eb);
        H.plane = (int64_t)round_up((size_t)H.sx * B.ny * B.nz, 64);
        // A plane of a multiple of 65,536 cells (power-of-two boxes) puts
        // the same cell of all 19 planes at one offset modulo a large power
        // of two, and the stream-collide's 38 streams then run slower: at
        // 512x512x256 the bulk kernel took 1.7 % (FP32) and 2.8 % (FP16)
        // longer than with the planes staggered by 1,024 cells, whole steps
        // 1.9 % and 3.9 %.  Staggers of 2,048 cells (and, in FP32, 64) were
        // slower than none; FP64 planes showed no gain, so they keep theirs.
        if (eb <= 4 && H.plane >= (int64_t)1 << 22 && H.plane % 65536 == 0 &&
            10 * (H.plane + 1024) * eb <= (int64_t)BUF_MAX_PLANE_GROUP)
            H.plane += 1024;
        // the stream-collide addresses ten population planes from one base
        // with 32-bit offsets
        if ((int64_t)B.ny * B.nz >= (1LL << 31) || 10 * H.plane * eb > (int64_t)BUF_MAX_PLANE_GROUP)
            return fail(err, IBLB_E_INVAL,
                        nm + ": box too large (ten population planes must fit in 4 GiB: at most " +
                            std::to_string(BUF_MAX_PLANE_GROUP / 10 / eb) + " cells incl. x padding)");
        H.tnx = (B.nx + TX - 1) / TX;
        H.tny = (B.ny + TY - 1) / TY;
        H.tnz = (B.nz + TZ - 1) / TZ;
        H.n_tiles = H.tnx * H.tny * H.tnz;
        H.tile_base = p.total_tiles;
        p.total_tiles += (int)round_up((size_t)H.n_tiles, TILE_CELLS);
        // row segments of at least 64 cells, plus the empty row groups that
        // fill the last group of eight
        p.max_rows += ((size_t)B.ny * B.nz + 7) * ((B.nx + 63) / 64);
    }
    p.drops.resize(cfg->n_droplets);
    // droplets are laid out box by box so each box owns a contiguous block range
    std::vector<int> order(cfg->n_droplets);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return cfg->droplets[a].box < cfg->droplets[b].box; });
    for (int di = 0; di < cfg->n_droplets; ++di) {
        const iblb_droplet &D = cfg->droplets[di];
        const std::string nm = "droplet " + std::to_string(di);
        if (D.box < 0 || D.box >= cfg->n_boxes) return fail(err, IBLB_E_INVAL, nm + ": bad box index");
        if (D.n_nodes < 4 || D.n_tris < 4 || !D.nodes || !D.tris)
            return fail(err, IBLB_E_INVAL, nm + ": mesh arrays missing or too small");
        if (!(D.sigma >= 0) || !finite(D.sigma)) return fail(err, IBLB_E_INVAL, nm + ": sigma must be >= 0");
        if (!(D.theta_eq >= 0 && D.theta_eq <= M_PI))
            return fail(err, IBLB_E_INVAL, nm + ": theta_eq must lie in [0, pi]");
        if (!(D.xi > 0) || !finite(D.xi)) return fail(err, IBLB_E_INVAL, nm + ": xi must be > 0");
        if (!(D.n_exp > D.m_exp && D.m_exp >= 1 && D.n_exp <= 64))
            return fail(err, IBLB_E_INVAL, nm + ": need 64 >= n > m >= 1");
        if (!(D.k_vol >= 0) || !finite(D.k_vol)) return fail(err, IBLB_E_INVAL, nm + ": k_vol must be >= 0");
        const iblb_box &B = cfg->boxes[D.box];
        if (B.nx < 4 || B.ny < 4 || B.nz < 4)
            return fail(err, IBLB_E_INVAL, nm + ": a box holding a droplet needs nx, ny, nz >= 4");
        for (int k = 0; k < 3 * D.n_nodes; ++k)
            if (!finite(D.nodes[k])) return fail(err, IBLB_E_INVAL, nm + ": node coordinate not finite");
        iblb_status st = check_mesh(D, di, err);
        if (st != IBLB_OK) return st;
        if (B.zbc == IBLB_Z_WALLS) {
            for (int j = 0; j < D.n_nodes; ++j)
                if (!(D.nodes[3 * j + 2] > 0.0) || !(D.nodes[3 * j + 2] < B.nz))
                    return fail(err, IBLB_E_MESH, nm + ": node " + std::to_string(j) +
                                                      " is not strictly between the walls");
        }
    }
    int blk = 0, tri = 0, chunk = 0;
    for (int oi = 0; oi < cfg->n_droplets; ++oi) {
        const int di = order[oi];
        const iblb_droplet &D = cfg->droplets[di];
        DropHost &H = p.drops[di];
        H.d = D;
        H.nodes.assign(D.nodes, D.nodes + 3 * (size_t)D.n_nodes);
        H.tris.assign(D.tris, D.tris + 3 * (size_t)D.n_tris);
        H.d.nodes = nullptr;
        H.d.tris = nullptr;
        H.n_blocks = (D.n_nodes + NB - 1) / NB;
        H.blk_off = blk;
        H.node_off = blk * NB;
        blk += H.n_blocks;
        H.tri_off = tri;
        tri += D.n_tris;
        H.n_chunks = (D.n_tris + TRI_CHUNK - 1) / TRI_CHUNK;
        H.chunk_off = chunk;
        chunk += H.n_chunks;
        H.A = D.sigma * (double)((D.m_exp - 1) * (D.n_exp - 1)) / ((double)(D.n_exp - D.m_exp) * D.xi) *
              (1.0 + std::cos(D.theta_eq));  // Eq. 11
        if (D.k_vol > 0) p.any_kvol = true;
        // compact node blocks: recursive coordinate bisection of the initial
        // positions into ceil(N/64) parts of 64 (the last one partial),
        // splitting the longest extent at a multiple of 64 nodes
        H.perm.resize(D.n_nodes);
        std::iota(H.perm.begin(), H.perm.end(), 0);
        rcb_order(D.nodes, H.perm.data(), D.n_nodes, H.n_blocks);
        H.inv.resize(D.n_nodes);
        for (int k = 0; k < D.n_nodes; ++k) H.inv[H.perm[k]] = k;
        double c[3] = {0, 0, 0};
        for (int j = 0; j < D.n_nodes; ++j)
            for (int a = 0; a < 3; ++a) c[a] += D.nodes[3 * j + a];
        for (int a = 0; a < 3; ++a) H.ref[a] = std::floor(c[a] / D.n_nodes);
    }
    p.nblk = blk;
    p.Ntot = blk * NB;
    p.Ttot = tri;
    p.n_chunks = chunk;
    for (int b = 0; b < cfg->n_boxes; ++b) {
        BoxHost &H = p.boxes[b];
        H.blk_begin = H.blk_end = 0;
        bool any = false;
        for (const auto &dh : p.drops)
            if (dh.d.box == b) {
                if (!any) H.blk_begin = dh.blk_off;
                any = true;
                H.blk_end = std::max(H.blk_end, dh.blk_off + dh.n_blocks);
            }
    }

    // workspace layout
    size_t o = 0;
    auto take = [&](size_t bytes, size_t al = ALIGN) {
        o = round_up(o, al);
        const size_t r = o;
        o += std::max<size_t>(bytes, 1);
        return r;
    };
    for (auto &H : p.boxes) {
        for (int k = 0; k < 2; ++k) H.off_f[k] = take((size_t)Q * H.plane * eb, BIG_ALIGN);
        for (int k = 0; k < 2; ++k) H.off_stamp[k] = take((size_t)H.n_tiles * 4);
        H.off_F = take((size_t)H.n_tiles * 3 * TILE_CELLS * p.real);
        H.off_u = take((size_t)H.n_tiles * 3 * TILE_CELLS * p.real);
        if (p.flags & IBLB_FLAG_FULL_U) H.off_ufull = take((size_t)3 * H.plane * p.real);
        if (H.b.tau_in > 0.0) {
            H.nzw = (H.b.nz + 63) / 64;
            for (int k = 0; k < 2; ++k) H.off_mask[k] = take((size_t)H.nzw * H.b.ny * H.b.nx * 8);
        }
    }
    p.off_boxes = take(sizeof(BoxDev) * p.boxes.size());
    p.off_drops = take(sizeof(DropDev) * std::max<size_t>(p.drops.size(), 1));
    const size_t N = (size_t)p.Ntot;
    p.off_qh = take(3 * N * p.real);
    p.off_ql = take(3 * N * p.real);
    p.off_phi = take(3 * N * p.real);
    p.off_wgt = take(12 * N * p.real);
    p.off_trec = take((size_t)TREC * p.Ttot * p.real);
    p.off_tile_list = take((size_t)p.total_tiles * 8);
    p.off_tile_count = take(2 * 4);
    p.off_base = take(3 * N * 4);
    p.off_s0 = take(3 * N * 4);
    p.off_bbox = take(6 * (size_t)p.nblk * 4);
    p.off_breg = take((size_t)BREG * p.nblk * 4);
    p.off_part = take((size_t)3 * MAXP * p.nblk * p.real);
    p.off_blk_drop = take((size_t)p.nblk * 8);
    p.off_tri = take(3 * (size_t)p.Ttot * 4);
    p.off_csr_off = take((N + 1) * 4);
    p.off_csr_ent = take(3 * (size_t)p.Ttot * 4);
    p.off_chunks = take(sizeof(TriChunk) * (size_t)p.n_chunks);
    p.off_tri_part = take(2 * (size_t)p.n_chunks * 8);
    p.off_rows = take(sizeof(RowGroup) * (size_t)p.max_rows);
    p.off_tchunk = take((size_t)(p.total_tiles / TILE_CELLS) * 4);
    p.off_tcand = take((size_t)p.total_tiles * MAXC * 4);
    p.off_tncand = take((size_t)2 * p.total_tiles * 4);
    p.off_scan = take((size_t)2 * p.boxes.size() * 4);
    p.off_ctr = take(4);
    p.off_step_epoch = take(2 * 4);
    p.off_status = take(4);
    p.off_obs_part = take(2 * (size_t)OBS_GROUPS * 8);
    p.off_obs_out = take(((size_t)p.drops.size() * OBS_DROP + p.boxes.size() * OBS_BOX) * 8);
    p.off_uout = take(3 * N * 8);
    p.total = round_up(o, ALIGN);
    o = 0;
    p.st_trec = take((size_t)TREC * p.Ttot * p.real);
    p.st_tri_part = take(2 * (size_t)p.n_chunks * 8);
    p.st_bbox = take(6 * (size_t)p.nblk * 4);
    p.st_breg = take((size_t)BREG * p.nblk * 4);
    p.st_part = take((size_t)3 * MAXP * p.nblk * p.real);
    p.st_tile_list = take((size_t)p.total_tiles * 8);
    p.st_tile_count = take(2 * 4);
    p.st_tcand = take((size_t)p.total_tiles * MAXC * 4);
    p.st_tncand = take((size_t)2 * p.total_tiles * 4);
    p.st_scan = take((size_t)2 * p.boxes.size() * 4);
    p.st_total = round_up(o, ALIGN);
    return IBLB_OK;
}

}  // namespace

struct iblb_ctx {
    Plan plan;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;  // origin stream of graph captures
    hipStream_t ib = nullptr;       // second stream: the mesh chain of a step
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    char *scratch = nullptr;  // this device's fixed scratch (iblb_step_static)
    DevPtrs P{};
    Launch L{};
    hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // [parity][advect first]
    // MULTI_LEN[i] consecutive steps from a pending advection, by starting
    // parity: one launch instead of MULTI_LEN[i] (the host cost of a launch
    // is close to a step's device time at the sizes of the spreading
    // workload)
    hipGraphExec_t multi[N_MULTI][2] = {};
    bool pending = false;  // advection of the last step not yet applied
    int parity = 0;
    int64_t step = 0;
    bool u_valid = false;    // the full u field holds the last step's velocity
    int32_t epoch = 0;       // host mirror of the device step epoch
    int32_t last_step_epoch = -1;
    int last_step_parity = 0;  // buffer parity of the last step (its stamp set)
    hipEvent_t ev_chain = nullptr, ev_bulk = nullptr;  // joins inside a run of steps
    bool unstable = false;
    std::string err = "no error";
    double *host_obs = nullptr;
    uint32_t *host_status = nullptr;
    std::vector<char> init_qh, init_ql;  // initial node positions, kept during init only
};

namespace {

iblb_status set_err(iblb_ctx *c, iblb_status code, const std::string &msg) {
    if (c) c->err = msg;
    g_last_error = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_err(ctx, IBLB_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool is_f64(const iblb_ctx *c) { return c->plan.storage == IBLB_F64; }

// Row groups of the bulk launch: BY * CPT rows each, and, when a row is
// longer than the workgroup's threads along x (a multiple of 64), split into
// segments of that length taken by consecutive workgroups, so that the
// workgroups in flight stream through consecutive stretches of each
// population plane (a workgroup looping along the row instead: 5.46
// against 5.69 TB/s for the stream-collide of a 512x512x256 box, 5.31
// against 5.67 at 1024 cells per row).
iblb_status upload_rows(iblb_ctx *c) {
    std::vector<RowGroup> rows;
    const int R = c->L.by * c->L.cpt, BX = c->L.bx;
    for (int b = 0; b < (int)c->plan.boxes.size(); ++b) {
        const iblb_box &B = c->plan.boxes[b].b;
        const int nr = B.ny * B.nz;
        // rows end in the padding (zeros written with the row's last line,
        // so that no line is written in part) when it is at most an eighth
        // of the row (FP32: 250 -> 256 cells 10 % faster, the batched boxes'
        // 48 -> 64, 80 -> 96, 112 -> 128 slower), and always for two-byte
        // storage (the batched boxes' fluid pass 3.5 % faster)
        const int sx = c->plan.boxes[b].sx;
        const bool two_byte = elem_bytes(c->plan.storage) == 2;
        const int xe = (two_byte || (sx - B.nx) * 8 <= B.nx) ? sx : B.nx;
        const int seg = (BX % 64 == 0 && B.nx > BX) ? BX : B.nx;
        if (seg == B.nx) {
            for (int r = 0; r < nr; r += R) rows.push_back({b, r, std::min(r + R, nr), 0, xe, {0, 0, 0}});
            continue;
        }
        // Rows split into segments: the segments of one row group share the
        // cache lines at their ends (the +-1 shifted pulls, the periodic
        // wrap), so they go to workgroups 8 apart, which the dispatcher
        // places on the same XCD (one L2) at about the same time.  Groups of
        // eight row groups, segment-major within a group; the last group is
        // filled up with empty row groups so that the pattern holds for the
        // whole box.
        for (int r = 0; r < nr; r += 8 * R)
            for (int x0 = 0; x0 < B.nx; x0 += seg)
                for (int k = 0; k < 8; ++k) {
                    const int r0 = std::min(r + k * R, nr), r1 = std::min(r + (k + 1) * R, nr);
                    rows.push_back({b, r0, r1, x0, x0 + seg < B.nx ? x0 + seg : xe, {0, 0, 0}});
                }
    }
    if (rows.size() > c->plan.max_rows)
        return set_err(c, IBLB_E_INVAL, "row table exceeds its reserved size");
    c->P.n_rowgroups = (int)rows.size();
    c->P.pad_rows = 0;
    for (const RowGroup &g : rows)
        if (g.x1 > c->plan.boxes[g.box].b.nx) c->P.pad_rows = 1;
    c->L.grid = (int)rows.size();
    if (c->L.maxg > 0 && c->L.maxg < c->L.grid) c->L.grid = c->L.maxg;
    HIPCHK(c, hipMemcpyAsync(c->P.rows, rows.data(), rows.size() * sizeof(RowGroup),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return IBLB_OK;
}

// Inside bits (boxes with tau_in) of the current node positions into mask
// set `slot`: cleared by a kernel, then toggled by the triangles.
iblb_status compute_masks(iblb_ctx *c, int slot, hipStream_t s) {
    if (!c->P.contrast) return IBLB_OK;
    HIPCHK(c, launch_mask_clear(c->P, slot, s));
    HIPCHK(c, launch_inside(c->P, is_f64(c), slot, s));
    return IBLB_OK;
}

// n consecutive time steps on stream s, the first with buffer parity
// `parity`.  Per step, on the second stream, the mesh chain: [advection of
// the previous step] -> inside bits -> triangle records -> node pass
// (forces, weights, tile stamps, partial spread) -> stamped-tile list.  The
// band kernel gathers the spread force of every stamped tile and does the
// collision of its cells; the bulk stream-collide does the collision of the
// other cells with the body force only.  Two schedules (Launch::after),
// chosen by the autotuner; every cell gets the same arithmetic in both:
//   0 (band beside bulk): the bulk kernel of step k runs on s after the
//     node pass of step k (its stamps and inside bits) and skips the stamped
//     tiles; the band kernel runs on the second stream right after the node
//     pass, once the bulk kernel of step k-1 is done (it overwrites the
//     buffer that kernel read).  The mesh chain of step k+1 follows the band
//     kernel on the second stream, beside the bulk kernel of step k: per
//     step, one queue crossing each way.
//   1 (band after bulk): the bulk kernel of step k runs over every cell on
//     s beside the mesh chain of step k, which forks from s after the band
//     kernel of step k-1; the band kernel then overwrites its tiles on s,
//     after both.  The bulk kernel relaxes with the previous step's inside
//     bits, so this schedule is not used with a viscosity contrast.
// The advection of the last step is left pending (it only needs that step's
// band velocities) and runs first in the next chain, or in flush().  A run
// ends joined into s.
iblb_status enqueue_steps(iblb_ctx *c, hipStream_t s, int parity, bool advect_first, int n) {
    const bool f64 = is_f64(c);
    const int full_u = (c->plan.flags & IBLB_FLAG_FULL_U) ? 1 : 0;
    const float scale = (float)c->plan.scale;
    if (c->plan.nblk == 0) {
        for (int k = 0; k < n; ++k)
            HIPCHK(c, launch_bulk(c->P, c->plan.storage, parity ^ (k & 1), full_u, scale, c->L, false, s));
        return IBLB_OK;
    }
    auto chain = [&](int k, int p) -> iblb_status {
        if (advect_first || k > 0) HIPCHK(c, launch_interp(c->P, f64, 0, nullptr, c->ib));
        const iblb_status st = compute_masks(c, p, c->ib);
        if (st != IBLB_OK) return st;
        HIPCHK(c, launch_tri(c->P, f64, c->ib));
        HIPCHK(c, launch_node(c->P, f64, 0, p, c->ib));
        HIPCHK(c, hipEventRecord(c->ev_chain, c->ib));
        return IBLB_OK;
    };
    if (c->L.after) {
        for (int k = 0; k < n; ++k) {
            const int p = parity ^ (k & 1);
            HIPCHK(c, hipEventRecord(c->ev_fork, s));
            HIPCHK(c, hipStreamWaitEvent(c->ib, c->ev_fork, 0));
            const iblb_status st = chain(k, p);
            if (st != IBLB_OK) return st;
            HIPCHK(c, launch_bulk(c->P, c->plan.storage, p, full_u, scale, c->L, false, s));
            HIPCHK(c, hipStreamWaitEvent(s, c->ev_chain, 0));
            HIPCHK(c, launch_band(c->P, c->plan.storage, p, full_u, scale, true, c->L.nt, s));
        }
        return IBLB_OK;
    }
    HIPCHK(c, hipEventRecord(c->ev_fork, s));
    HIPCHK(c, hipStreamWaitEvent(c->ib, c->ev_fork, 0));
    for (int k = 0; k < n; ++k) {
        const int p = parity ^ (k & 1);
        const iblb_status st = chain(k, p);
        if (st != IBLB_OK) return st;
        HIPCHK(c, hipStreamWaitEvent(s, c->ev_chain, 0));
        HIPCHK(c, launch_bulk(c->P, c->plan.storage, p, full_u, scale, c->L, true, s));
        if (k > 0) HIPCHK(c, hipStreamWaitEvent(c->ib, c->ev_bulk, 0));  // the previous step's bulk kernel
        HIPCHK(c, launch_band(c->P, c->plan.storage, p, full_u, scale, true, c->L.nt, c->ib));
        HIPCHK(c, hipEventRecord(c->ev_bulk, s));
    }
    HIPCHK(c, hipEventRecord(c->ev_join, c->ib));
    HIPCHK(c, hipStreamWaitEvent(s, c->ev_join, 0));
    return IBLB_OK;
}

// Apply a pending advection (positions then correspond to the completed
// steps).  Every call that reads or replaces state starts with it.
iblb_status flush(iblb_ctx *c) {
    if (!c->pending) return IBLB_OK;
    HIPCHK(c, launch_interp(c->P, is_f64(c), 0, nullptr, c->stream));
    c->pending = false;
    ++c->epoch;
    return IBLB_OK;
}

void drop_graphs(iblb_ctx *c) {
    for (auto &row : c->multi)
        for (auto &e : row)
            if (e) {
                (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
    for (auto &row : c->exec)
        for (auto &e : row)
            if (e) {
                (void)hipGraphExecDestroy(e);
                e = nullptr;
            }
}

iblb_status build_graphs(iblb_ctx *c) {
    drop_graphs(c);
    if (!(c->plan.flags & IBLB_FLAG_GRAPH)) return IBLB_OK;
    if (!c->capture) HIPCHK(c, hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
    for (int p = 0; p < 2; ++p)
        for (int a = 0; a < 2; ++a) {
            hipGraph_t g = nullptr;
            HIPCHK(c, hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
            iblb_status st = enqueue_steps(c, c->capture, p, a == 1, 1);
            hipError_t e = hipStreamEndCapture(c->capture, &g);
            if (st != IBLB_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess)
                return set_err(c, IBLB_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&c->exec[p][a], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess)
                return set_err(c, IBLB_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
    if (c->plan.nblk == 0) return IBLB_OK;  // no advection: single steps only
    for (int li = 0; li < N_MULTI; ++li)
        for (int p = 0; p < 2; ++p) {
            hipGraph_t g = nullptr;
            HIPCHK(c, hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
            const iblb_status st = enqueue_steps(c, c->capture, p, true, MULTI_LEN[li]);
            hipError_t e = hipStreamEndCapture(c->capture, &g);
            if (st != IBLB_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess)
                return set_err(c, IBLB_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&c->multi[li][p], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess)
                return set_err(c, IBLB_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
    return IBLB_OK;
}

// Why a bulk launch configuration is not valid (nullptr if it is).
const char *launch_problem(const Launch &L) {
    if (L.bx < 32 || (L.bx & 31) || L.by < 1 || L.bx * L.by > K1_MAX_THREADS || (L.bx * L.by) % 64)
        return "launch shape: threads_x a multiple of 32, threads_x*rows a multiple of 64 and <= 256";
    if (L.cpt != 1 && L.cpt != 2) return "cells_per_thread must be 1 or 2";
    if (L.cpt == 2 && L.bx % 64) return "cells_per_thread 2 needs threads_x a multiple of 64";
    if (L.nt != 0 && L.nt != 1) return "streaming_stores must be 0 or 1";
    if (L.maxg < 0) return "max_workgroups must be >= 0";
    if (L.after != 0 && L.after != 1) return "band_after_bulk must be 0 or 1";
    return nullptr;
}
static_assert(K1_MAX_THREADS == 256, "launch_problem() states the bound");

// Two timing events, destroyed on every return path.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() = default;
    EventPair(const EventPair &) = delete;
    EventPair &operator=(const EventPair &) = delete;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

iblb_status time_k1(iblb_ctx *c, int reps, double *ms) {
    EventPair ev;
    HIPCHK(c, hipEventCreate(&ev.a));
    HIPCHK(c, hipEventCreate(&ev.b));
    HIPCHK(c, hipEventRecord(ev.a, c->stream));
    for (int r = 0; r < reps; ++r) {
        HIPCHK(c, launch_bulk(c->P, c->plan.storage, c->parity, 0, (float)c->plan.scale, c->L, false,
                              c->stream));
        c->parity ^= 1;
    }
    HIPCHK(c, hipEventRecord(ev.b, c->stream));
    HIPCHK(c, hipEventSynchronize(ev.b));
    float t = 0;
    HIPCHK(c, hipEventElapsedTime(&t, ev.a, ev.b));
    *ms = (double)t / reps;
    return IBLB_OK;
}

// Back to the state iblb_init leaves: fluid at rest, initial node positions,
// no pending advection, step 0 (the device epoch keeps counting).
iblb_status reset_state(iblb_ctx *c) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &H : c->plan.boxes)
        for (int k = 0; k < 2; ++k)
            HIPCHK(c, hipMemsetAsync(c->ws + H.off_f[k], 0,
                                     (size_t)Q * H.plane * elem_bytes(c->plan.storage), c->stream));
    if (!c->init_qh.empty()) {
        HIPCHK(c, hipMemcpyAsync(c->P.qh, c->init_qh.data(), c->init_qh.size(), hipMemcpyHostToDevice,
                                 c->stream));
        HIPCHK(c, hipMemcpyAsync(c->P.ql, c->init_ql.data(), c->init_ql.size(), hipMemcpyHostToDevice,
                                 c->stream));
    }
    HIPCHK(c, hipMemsetAsync(c->P.status, 0, 4, c->stream));
    for (int k = 0; k < 2; ++k) {
        const iblb_status st = compute_masks(c, k, c->stream);
        if (st != IBLB_OK) return st;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->pending) {
        // the dropped advection would have started a new epoch: start it here,
        // so that the next stamping pass does not meet the last one's stamps
        HIPCHK(c, launch_epoch(c->P, c->stream));
        ++c->epoch;
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->pending = false;
    c->parity = 0;
    c->step = 0;
    c->last_step_epoch = -1;
    c->unstable = false;
    return IBLB_OK;
}

// Mean device time (ms) of one graph-replayed step, best of three runs.
iblb_status time_steps(iblb_ctx *c, double *ms) {
    EventPair ev;
    HIPCHK(c, hipEventCreate(&ev.a));
    HIPCHK(c, hipEventCreate(&ev.b));
    iblb_status st = iblb_step(c, 20);
    *ms = 1e300;
    for (int rep = 0; rep < 3 && st == IBLB_OK; ++rep) {
        HIPCHK(c, hipEventRecord(ev.a, c->stream));
        st = iblb_step(c, 40);
        HIPCHK(c, hipEventRecord(ev.b, c->stream));
        HIPCHK(c, hipEventSynchronize(ev.b));
        float t = 0;
        HIPCHK(c, hipEventElapsedTime(&t, ev.a, ev.b));
        *ms = std::min(*ms, (double)t / 40);
    }
    return st;
}

iblb_status autotune(iblb_ctx *c) {
    int nxmax = 0;
    for (auto &H : c->plan.boxes) nxmax = std::max(nxmax, H.b.nx);
    const int saved_parity = c->parity;
    auto timed = [&](const Launch &L, double *ms) -> iblb_status {
        c->L = L;
        iblb_status st = upload_rows(c);
        if (st != IBLB_OK) return st;
        double t = 0;
        *ms = 1e300;
        st = time_k1(c, 3, &t);
        for (int rep = 0; rep < 3 && st == IBLB_OK; ++rep) {
            st = time_k1(c, 10, &t);
            *ms = std::min(*ms, t);
        }
        return st;
    };
    // 1. block shape, rows per thread, store policy: fastest bulk kernel
    Launch best = c->L;
    double tbest = 1e300;
    std::vector<std::pair<double, Launch>> tried;
    for (int nt : {0, 1})
        for (int bx : {32, 64, 128, 256}) {
            if (bx > (int)round_up((size_t)nxmax, 32)) continue;
            for (int threads : {64, 128, K1_MAX_THREADS})
                for (int cpt : {1, 2}) {
                    const Launch L{bx, threads / bx, 0, nt, cpt, 0, 0};
                    if (L.by < 1 || launch_problem(L)) continue;
                    double ms = 0;
                    iblb_status st = timed(L, &ms);
                    if (st != IBLB_OK) return st;
                    tried.push_back({ms, L});
                    if (ms < tbest) {
                        tbest = ms;
                        best = L;
                    }
                }
        }
    // Up to three more block shapes whose bulk kernel alone is within 3 % of
    // the fastest go on to whole steps too: skipping the band tiles, beside
    // the band and mesh kernels, the shapes can rank otherwise (at
    // 256x256x128 in FP32 the bulk kernel alone took 128x1, 128x2 and 256x1
    // within 1 % of each other, and whole steps 0.294, 0.257 and 0.251 ms).
    std::stable_sort(tried.begin(), tried.end(),
                     [](const std::pair<double, Launch> &a, const std::pair<double, Launch> &b) {
                         return a.first < b.first;
                     });
    std::vector<Launch> shapes{best};
    for (const auto &t : tried) {
        if (t.first > tbest * 1.03 || shapes.size() >= 4) break;
        bool seen = false;
        for (const Launch &h : shapes)
            seen = seen || (h.bx == t.second.bx && h.by == t.second.by && h.nt == t.second.nt);
        if (!seen) shapes.push_back(t.second);
    }
    // 2. with meshes present and the step replayed as graphs, the schedule
    //    and a cap on the bulk grid are judged by whole steps: the workgroups
    //    the cap does not take leave CU slots to the mesh kernels that run
    //    beside it, at some cost in bulk bandwidth.  Under a cap, two rows per
    //    thread keep more loads in flight per wave, so both are tried.  Each
    //    candidate starts from the initial state.
    if (c->plan.nblk > 0 && (c->plan.flags & IBLB_FLAG_GRAPH)) {
        const int cus = c->P.n_cus;
        double sbest = 1e300;
        Launch chosen = best;
        for (size_t si = 0; si < shapes.size(); ++si) {
            const Launch &shape = shapes[si];
            const int wpg = shape.bx * shape.by / 64;  // waves per workgroup
            for (int after = 0; after < (c->P.contrast ? 1 : 2); ++after)
                for (int waves_per_cu : {0, 16, 12, 8, 6})
                    for (int cpt : {1, 2}) {
                        // the other shapes: uncapped, at their own rows per thread
                        if (si > 0 && (waves_per_cu || cpt != shape.cpt)) continue;
                        Launch L = shape;
                        L.cpt = cpt;
                        L.after = after;
                        if (launch_problem(L)) continue;
                        L.maxg = waves_per_cu ? std::max(1, cus * waves_per_cu / wpg) : 0;
                        c->L = L;
                        iblb_status st = upload_rows(c);
                        if (st != IBLB_OK) return st;
                        if (L.maxg && c->L.grid >= c->P.n_rowgroups) continue;  // no cap at this size
                        double ms = 0;
                        st = reset_state(c);
                        if (st == IBLB_OK) st = build_graphs(c);
                        if (st == IBLB_OK) st = time_steps(c, &ms);
                        if (st != IBLB_OK) return st;
                        if (ms < sbest) {
                            sbest = ms;
                            chosen = L;
                        }
                    }
        }
        best = chosen;
        iblb_status st = reset_state(c);
        if (st != IBLB_OK) return st;
    }
    c->L = best;
    iblb_status st = upload_rows(c);
    if (st != IBLB_OK) return st;
    // the timing runs advanced the fluid without the meshes: back to rest
    c->parity = saved_parity;
    for (auto &H : c->plan.boxes)
        for (int k = 0; k < 2; ++k)
            HIPCHK(c, hipMemsetAsync(c->ws + H.off_f[k], 0,
                                     (size_t)Q * H.plane * elem_bytes(c->plan.storage), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return IBLB_OK;
}

// ---- autotune results kept across contexts ----
// Key: the device (architecture, compute units), storage, graph use,
// viscosity contrast and moving walls, and per box its dimensions, z
// boundary and the node count of its droplets -- what the timed candidates
// depend on.  Kept per process, and in the text file that the environment
// variable IBLB_TUNE_CACHE names (one "key<TAB>launch" line per entry;
// later lines win), so that repeated inits of one configuration time once.
std::mutex g_tune_mu;
std::unordered_map<std::string, Launch> g_tune;

iblb_status tune_key(iblb_ctx *c, std::string *key) {
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIPCHK(c, hipGetDeviceProperties(&prop, dev));
    std::ostringstream k;
    k << prop.gcnArchName << "/cu" << c->P.n_cus << "/st" << c->plan.storage << "/g"
      << ((c->plan.flags & IBLB_FLAG_GRAPH) ? 1 : 0) << "/c" << c->P.contrast << "/m" << c->P.moving;
    for (size_t b = 0; b < c->plan.boxes.size(); ++b) {
        const iblb_box &B = c->plan.boxes[b].b;
        long nodes = 0;
        for (const DropHost &d : c->plan.drops)
            if (d.d.box == (int)b) nodes += d.d.n_nodes;
        k << "/" << B.nx << "x" << B.ny << "x" << B.nz << "z" << B.zbc << "n" << nodes;
    }
    *key = k.str();
    return IBLB_OK;
}

bool tune_lookup(const std::string &key, Launch *L) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
        *L = it->second;
        return true;
    }
    const char *path = std::getenv("IBLB_TUNE_CACHE");
    if (!path || !*path) return false;
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        const size_t tab = line.find('\t');
        if (tab == std::string::npos || line.compare(0, tab, key) != 0 || tab != key.size()) continue;
        std::istringstream v(line.substr(tab + 1));
        Launch t{};
        if (v >> t.bx >> t.by >> t.cpt >> t.nt >> t.maxg >> t.after) {
            *L = t;
            found = true;
        }
    }
    if (found) g_tune[key] = *L;
    return found;
}

void tune_store(const std::string &key, const Launch &L) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = L;
    const char *path = std::getenv("IBLB_TUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream out(path, std::ios::app);
    out << key << '\t' << L.bx << ' ' << L.by << ' ' << L.cpt << ' ' << L.nt << ' ' << L.maxg << ' ' << L.after
        << '\n';
}

// ---- host conversion of stored populations (I/O only) ----
double decode(const iblb_ctx *c, const void *raw, size_t i) {
    switch (c->plan.storage) {
    case IBLB_F64: return ((const double *)raw)[i];
    case IBLB_F32: return ((const float *)raw)[i];
    case IBLB_F16DEV: return (double)(float)((const _Float16 *)raw)[i] / c->plan.scale;
    default: {
        uint32_t bits = (uint32_t)((const uint16_t *)raw)[i] << 16;
        float f;
        std::memcpy(&f, &bits, 4);
        return f;
    }
    }
}

void encode(const iblb_ctx *c, void *raw, size_t i, double v) {
    switch (c->plan.storage) {
    case IBLB_F64: ((double *)raw)[i] = v; break;
    case IBLB_F32: ((float *)raw)[i] = (float)v; break;
    case IBLB_F16DEV: ((_Float16 *)raw)[i] = (_Float16)(float)(v * c->plan.scale); break;
    default: {
        const float f = (float)v;
        uint32_t bits;
        std::memcpy(&bits, &f, 4);
        bits += 0x7fffu + ((bits >> 16) & 1u);  // round to nearest even
        ((uint16_t *)raw)[i] = (uint16_t)(bits >> 16);
    }
    }
}

inline int wrap(int i, int n) { return ((i % n) + n) % n; }

}  // namespace

// =====================================================================  ABI

extern "C" {

iblb_status iblb_velocity_set(int32_t *c, double *w) {
    if (!c || !w) return set_err(nullptr, IBLB_E_INVAL, "NULL output");
    for (int i = 0; i < Q; ++i) {
        c[3 * i] = cx_of(i);
        c[3 * i + 1] = cy_of(i);
        c[3 * i + 2] = cz_of(i);
        w[i] = w_of(i);
    }
    return IBLB_OK;
}

iblb_status iblb_workspace_size(const iblb_config *cfg, size_t *bytes) {
    if (!bytes) return set_err(nullptr, IBLB_E_INVAL, "bytes is NULL");
    Plan p;
    std::string err;
    iblb_status st = build_plan(cfg, p, &err);
    if (st != IBLB_OK) return set_err(nullptr, st, err);
    *bytes = p.total;
    return IBLB_OK;
}

// Device-side set-up of a context whose plan, workspace, streams and events
// are in place: tables, meshes, initial state, launch shape, graphs.  On
// failure the caller destroys the context.
static iblb_status init_device(iblb_ctx *c) {
    Plan &p = c->plan;
    iblb_status st = IBLB_OK;
    auto at = [&](size_t off) { return (void *)(c->ws + off); };
    DevPtrs &P = c->P;
    P.boxes = (BoxDev *)at(p.off_boxes);
    P.drops = (DropDev *)at(p.off_drops);
    P.n_boxes = (int)p.boxes.size();
    P.n_drops = (int)p.drops.size();
    P.qh = at(p.off_qh);
    P.ql = at(p.off_ql);
    P.phi = at(p.off_phi);
    P.wgt = at(p.off_wgt);
    P.trec = at(p.off_trec);
    P.tile_list = (int32_t *)at(p.off_tile_list);
    P.tile_count = (int32_t *)at(p.off_tile_count);
    P.base = (int32_t *)at(p.off_base);
    P.s0 = (int32_t *)at(p.off_s0);
    P.bbox = (int32_t *)at(p.off_bbox);
    P.breg = (int32_t *)at(p.off_breg);
    P.part = at(p.off_part);
    P.blk_drop = (int32_t *)at(p.off_blk_drop);
    P.tri = (int32_t *)at(p.off_tri);
    P.csr_off = (int32_t *)at(p.off_csr_off);
    P.csr_ent = (int32_t *)at(p.off_csr_ent);
    P.chunks = (TriChunk *)at(p.off_chunks);
    P.tri_part = (double *)at(p.off_tri_part);
    P.rows = (RowGroup *)at(p.off_rows);
    P.tchunk_box = (int32_t *)at(p.off_tchunk);
    P.tcand = (int32_t *)at(p.off_tcand);
    P.tncand = (int32_t *)at(p.off_tncand);
    P.scan_all = (int32_t *)at(p.off_scan);
    P.ctr = (int32_t *)at(p.off_ctr);
    P.step_epoch = (int32_t *)at(p.off_step_epoch);
    P.status = (uint32_t *)at(p.off_status);
    P.obs_part = (double *)at(p.off_obs_part);
    P.obs_out = (double *)at(p.off_obs_out);
    P.Ntot = p.Ntot;
    P.nblk = p.nblk;
    P.Ttot = p.Ttot;
    P.n_chunks = p.n_chunks;
    P.total_tiles = p.total_tiles;
    P.obs_groups = OBS_GROUPS;
    {
        int dev = 0, cus = 0;
        HIPCHK(c, hipGetDevice(&dev));
        HIPCHK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        P.n_cus = std::max(cus, 1);
        HIPCHK(c, scratch_address(dev, &c->scratch));
    }

    // host tables
    std::vector<BoxDev> bd(p.boxes.size());
    std::vector<int32_t> tchunk(p.total_tiles / TILE_CELLS, 0);
    for (size_t b = 0; b < p.boxes.size(); ++b) {
        const BoxHost &H = p.boxes[b];
        BoxDev &D = bd[b];
        D.nx = H.b.nx;
        D.ny = H.b.ny;
        D.nz = H.b.nz;
        D.zbc = H.b.zbc;
        D.sx = H.sx;
        D.tnx = H.tnx;
        D.tny = H.tny;
        D.tnz = H.tnz;
        D.plane = H.plane;
        D.n_tiles = H.n_tiles;
        D.tile_base = H.tile_base;
        D.blk_begin = H.blk_begin;
        D.blk_end = H.blk_end;
        D.f[0] = at(H.off_f[0]);
        D.f[1] = at(H.off_f[1]);
        D.Fband = at(H.off_F);
        D.uband = at(H.off_u);
        D.stamp[0] = (int32_t *)at(H.off_stamp[0]);
        D.stamp[1] = (int32_t *)at(H.off_stamp[1]);
        D.ufull = (p.flags & IBLB_FLAG_FULL_U) ? at(H.off_ufull) : nullptr;
        D.tau = H.b.tau;
        D.rho0 = H.b.rho0;
        for (int a = 0; a < 3; ++a) D.g[a] = H.b.body_force[a];
        D.omega = 1.0 / H.b.tau;
        D.guo = 1.0 - 1.0 / (2.0 * H.b.tau);
        D.cells_rho0 = (double)H.b.nx * H.b.ny * H.b.nz * H.b.rho0;
        D.contrast = H.b.tau_in > 0.0 ? 1 : 0;
        D.nzw = H.nzw;
        D.omega_in = D.contrast ? 1.0 / H.b.tau_in : D.omega;
        D.guo_in = D.contrast ? 1.0 - 1.0 / (2.0 * H.b.tau_in) : D.guo;
        for (int k = 0; k < 2; ++k) D.mask[k] = D.contrast ? (uint64_t *)at(H.off_mask[k]) : nullptr;
        D.uw[0] = H.b.wall_lo[0];
        D.uw[1] = H.b.wall_lo[1];
        D.uw[2] = H.b.wall_hi[0];
        D.uw[3] = H.b.wall_hi[1];
        D.moving = (D.uw[0] != 0.0 || D.uw[1] != 0.0 || D.uw[2] != 0.0 || D.uw[3] != 0.0) ? 1 : 0;
        if (D.moving) P.moving = 1;
        if (D.contrast) {
            P.contrast = 1;
            P.mask_words = std::max(P.mask_words, (int32_t)((int64_t)D.nzw * D.ny * D.nx));
        }
        for (int k = 0; k < (int)round_up((size_t)H.n_tiles, TILE_CELLS) / TILE_CELLS; ++k)
            tchunk[H.tile_base / TILE_CELLS + k] = (int32_t)b;
    }
    const int N = p.Ntot;
    const int R = p.real;
    std::vector<char> qh((size_t)3 * N * R, 0), ql((size_t)3 * N * R, 0);
    std::vector<int32_t> tri((size_t)3 * std::max(p.Ttot, 1)), csr_off((size_t)N + 1, 0),
        csr_ent((size_t)3 * std::max(p.Ttot, 1)), blk_drop(2 * (size_t)std::max(p.nblk, 1));
    std::vector<TriChunk> chunks(std::max(p.n_chunks, 1));
    std::vector<DropDev> dd(std::max<size_t>(p.drops.size(), 1));
    for (size_t di = 0; di < p.drops.size(); ++di) {
        const DropHost &H = p.drops[di];
        DropDev &D = dd[di];
        D.box = H.d.box;
        D.n_nodes = H.d.n_nodes;
        D.n_tris = H.d.n_tris;
        D.n_exp = H.d.n_exp;
        D.m_exp = H.d.m_exp;
        D.node_off = H.node_off;
        D.blk_off = H.blk_off;
        D.n_blocks = H.n_blocks;
        D.tri_off = H.tri_off;
        D.chunk_off = H.chunk_off;
        D.n_chunks = H.n_chunks;
        D.sigma = H.d.sigma;
        D.A = H.A;
        D.xi = H.d.xi;
        D.kvol = H.d.k_vol;
        D.V0 = 0.0;
        for (int a = 0; a < 3; ++a) D.ref[a] = H.ref[a];
        for (int k = 0; k < H.n_blocks; ++k) {
            blk_drop[2 * (H.blk_off + k)] = (int32_t)di;
            blk_drop[2 * (H.blk_off + k) + 1] = (int32_t)H.d.box;
        }
        for (int k = 0; k < H.n_chunks; ++k) {
            const int t0 = H.tri_off + k * TRI_CHUNK;
            chunks[H.chunk_off + k] = {(int32_t)di, t0, std::min(t0 + TRI_CHUNK, H.tri_off + H.d.n_tris), 0};
        }
        for (int k = 0; k < H.d.n_nodes; ++k) {
            const int j = H.node_off + k;
            for (int a = 0; a < 3; ++a) {
                const double v = H.nodes[3 * H.perm[k] + a];
                if (R == 8) {
                    ((double *)qh.data())[(size_t)a * N + j] = v;
                } else {
                    const float h = (float)v;
                    ((float *)qh.data())[(size_t)a * N + j] = h;
                    ((float *)ql.data())[(size_t)a * N + j] = (float)(v - (double)h);
                }
            }
        }
        for (int t = 0; t < H.d.n_tris; ++t)
            for (int cc = 0; cc < 3; ++cc)
                tri[3 * (size_t)(H.tri_off + t) + cc] = H.node_off + H.inv[H.tris[3 * t + cc]];
    }
    // node -> incident triangles, ascending triangle id
    for (int t = 0; t < p.Ttot; ++t)
        for (int cc = 0; cc < 3; ++cc) csr_off[tri[3 * t + cc] + 1] += 1;
    for (int j = 0; j < N; ++j) csr_off[j + 1] += csr_off[j];
    {
        std::vector<int32_t> fill(N, 0);
        for (int t = 0; t < p.Ttot; ++t)
            for (int cc = 0; cc < 3; ++cc) {
                const int j = tri[3 * t + cc];
                csr_ent[csr_off[j] + fill[j]++] = 3 * t + cc;
            }
    }
    HIPCHK(c, hipMemcpyAsync(P.boxes, bd.data(), bd.size() * sizeof(BoxDev), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(P.drops, dd.data(), dd.size() * sizeof(DropDev), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(P.qh, qh.data(), qh.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(P.ql, ql.data(), ql.size(), hipMemcpyHostToDevice, c->stream));
    if (p.flags & IBLB_FLAG_AUTOTUNE) {
        c->init_qh = qh;
        c->init_ql = ql;
    }
    HIPCHK(c, hipMemcpyAsync(P.tri, tri.data(), 3 * (size_t)p.Ttot * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(P.csr_off, csr_off.data(), csr_off.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(P.csr_ent, csr_ent.data(), 3 * (size_t)p.Ttot * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(P.blk_drop, blk_drop.data(), (size_t)p.nblk * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(P.chunks, chunks.data(), (size_t)p.n_chunks * sizeof(TriChunk), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(P.tchunk_box, tchunk.data(), tchunk.size() * 4, hipMemcpyHostToDevice, c->stream));
    // fluid at rest: all deviations zero; no tile stamped; band zeroed
    for (auto &H : p.boxes) {
        for (int k = 0; k < 2; ++k)
            HIPCHK(c, hipMemsetAsync(at(H.off_f[k]), 0, (size_t)Q * H.plane * elem_bytes(p.storage), c->stream));
        for (int k = 0; k < 2; ++k)
            HIPCHK(c, hipMemsetAsync(at(H.off_stamp[k]), 0xff, (size_t)H.n_tiles * 4, c->stream));
        HIPCHK(c, hipMemsetAsync(at(H.off_F), 0, (size_t)H.n_tiles * 3 * TILE_CELLS * R, c->stream));
        HIPCHK(c, hipMemsetAsync(at(H.off_u), 0, (size_t)H.n_tiles * 3 * TILE_CELLS * R, c->stream));
        if (p.flags & IBLB_FLAG_FULL_U)
            HIPCHK(c, hipMemsetAsync(at(H.off_ufull), 0, (size_t)3 * H.plane * R, c->stream));
    }
    HIPCHK(c, hipMemsetAsync(P.ctr, 0, 4, c->stream));
    // no epoch yet: 0xfefefefe matches neither an unstamped tile (-1) nor an epoch
    HIPCHK(c, hipMemsetAsync(P.step_epoch, 0xfe, 8, c->stream));
    HIPCHK(c, hipMemsetAsync(P.tile_count, 0, 8, c->stream));
    HIPCHK(c, hipMemsetAsync(P.tncand, 0, (size_t)2 * p.total_tiles * 4, c->stream));
    HIPCHK(c, hipMemsetAsync(P.scan_all, 0, (size_t)2 * p.boxes.size() * 4, c->stream));
    HIPCHK(c, hipMemsetAsync(P.status, 0, 4, c->stream));
    HIPCHK(c, hipMemsetAsync(P.phi, 0, (size_t)3 * N * R, c->stream));
    // reference volumes V0 from the initial mesh (same FP64 sum as the penalty)
    HIPCHK(c, launch_tri(P, is_f64(c), c->stream));
    HIPCHK(c, launch_set_v0(P, is_f64(c), c->stream));
    // inside bits of the initial positions in both sets
    for (int k = 0; k < 2 && st == IBLB_OK; ++k) st = compute_masks(c, k, c->stream);
    if (st != IBLB_OK) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));

    // default launch shape of the stream-collide kernel
    int nxmax = 0;
    for (auto &H : p.boxes) nxmax = std::max(nxmax, H.b.nx);
    c->L.bx = nxmax <= 32 ? 32 : (nxmax <= 64 ? 64 : (nxmax <= 128 ? 128 : 256));
    c->L.by = std::max(1, 256 / c->L.bx);
    // streaming stores once both population buffers exceed the 256 MiB
    // last-level cache
    size_t pop_bytes = 0;
    for (auto &H : p.boxes) pop_bytes += 2 * (size_t)Q * H.plane * elem_bytes(p.storage);
    c->L.nt = pop_bytes > ((size_t)256 << 20) ? 1 : 0;
    c->L.cpt = 1;
    c->L.maxg = 0;
    st = upload_rows(c);
    if (st == IBLB_OK && (p.flags & IBLB_FLAG_AUTOTUNE)) {
        std::string key;
        Launch cached{};
        st = tune_key(c, &key);
        if (st == IBLB_OK && tune_lookup(key, &cached) && !launch_problem(cached) &&
            !(cached.after && c->P.contrast)) {
            c->L = cached;
            st = upload_rows(c);
        } else if (st == IBLB_OK) {
            st = autotune(c);
            if (st == IBLB_OK) tune_store(key, c->L);
        }
    }
    c->init_qh = std::vector<char>();
    c->init_ql = std::vector<char>();
    if (st == IBLB_OK) st = build_graphs(c);
    if (st == IBLB_OK) {
        if (hipHostMalloc((void **)&c->host_obs,
                          ((size_t)P.n_drops * OBS_DROP + (size_t)P.n_boxes * OBS_BOX) * 8 + 64,
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&c->host_status, 64, hipHostMallocDefault) != hipSuccess)
            st = set_err(c, IBLB_E_DEVICE, "pinned host buffer allocation failed");
    }
    return st;
}

iblb_status iblb_init(const iblb_config *cfg, void *dev_workspace, size_t bytes, void *hip_stream,
                      iblb_ctx **out) {
    if (!out) return set_err(nullptr, IBLB_E_INVAL, "out is NULL");
    *out = nullptr;
    iblb_ctx *c = new iblb_ctx();
    std::string err;
    iblb_status st = build_plan(cfg, c->plan, &err);
    if (st != IBLB_OK) {
        delete c;
        return set_err(nullptr, st, err);
    }
    Plan &p = c->plan;
    if (!dev_workspace || ((uintptr_t)dev_workspace % ALIGN) != 0 || bytes < p.total) {
        delete c;
        return set_err(nullptr, IBLB_E_WORKSPACE,
                       "workspace must be 256-byte aligned device memory of at least " +
                           std::to_string(p.total) + " bytes");
    }
    c->ws = (char *)dev_workspace;
    c->stream = (hipStream_t)hip_stream;
    {
        hipError_t e = hipStreamCreateWithFlags(&c->ib, hipStreamNonBlocking);
        const char *what = "hipStreamCreateWithFlags";
        if (e == hipSuccess) {
            e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
            what = "hipEventCreateWithFlags";
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_chain, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_bulk, hipEventDisableTiming);
        if (e != hipSuccess) {
            const std::string m = std::string(what) + ": " + hipGetErrorString(e);
            iblb_destroy(c);
            return set_err(nullptr, IBLB_E_DEVICE, m);
        }
    }
    st = init_device(c);
    if (st != IBLB_OK) {
        g_last_error = c->err;
        iblb_destroy(c);
        return st;
    }
    *out = c;
    return IBLB_OK;
}

iblb_status iblb_step(iblb_ctx *c, int64_t n) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (n < 0) return set_err(c, IBLB_E_INVAL, "n_steps < 0");
    if (c->unstable) return set_err(c, IBLB_E_STATE, "context is unstable; no further steps");
    for (int64_t k = 0; k < n;) {
        const int a = c->pending ? 1 : 0;
        const int p0 = c->parity;
        int64_t m = 0;
        for (int li = 0; a && li < N_MULTI && !m; ++li)
            if (n - k >= MULTI_LEN[li] && c->multi[li][p0]) {
                // MULTI_LEN[li] steps, each starting with the previous
                // step's advection
                HIPCHK(c, hipGraphLaunch(c->multi[li][p0], c->stream));
                m = MULTI_LEN[li];
            }
        if (!m && c->exec[p0][a]) {
            HIPCHK(c, hipGraphLaunch(c->exec[p0][a], c->stream));
            m = 1;
        }
        if (!m) {
            // eager: up to 256 steps as one pipelined run
            m = std::min<int64_t>(n - k, 256);
            iblb_status st = enqueue_steps(c, c->stream, p0, a == 1, (int)m);
            if (st != IBLB_OK) return st;
        }
        c->parity = p0 ^ (int)(m & 1);
        c->step += m;
        c->u_valid = true;
        if (c->plan.nblk > 0) {
            c->epoch += (int32_t)(m - 1 + a);  // one advection at the head of each step but the first
            c->last_step_epoch = c->epoch;
            c->last_step_parity = p0 ^ (int)((m - 1) & 1);
            c->pending = true;
        }
        k += m;
    }
    return IBLB_OK;
}

iblb_status iblb_step_static(iblb_ctx *c, int64_t n) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (n < 0) return set_err(c, IBLB_E_INVAL, "n_steps < 0");
    if (c->unstable) return set_err(c, IBLB_E_STATE, "context is unstable; no further steps");
    const Plan &p = c->plan;
    if (p.st_total > SCRATCH_BYTES)
        return set_err(c, IBLB_E_WORKSPACE,
                       "iblb_step_static: the configuration needs " + std::to_string(p.st_total) +
                           " bytes of step scratch, the fixed scratch holds " + std::to_string(SCRATCH_BYTES));
    if (n == 0) return IBLB_OK;
    {
        iblb_status st = flush(c);  // a pending advection of an iblb_step run
        if (st != IBLB_OK) return st;
    }
    hipStream_t s = c->stream;
    const bool f64 = is_f64(c);
    const int full_u = (p.flags & IBLB_FLAG_FULL_U) ? 1 : 0;
    const float scale = (float)p.scale;
    if (p.nblk == 0) {
        for (int64_t k = 0; k < n; ++k) {
            HIPCHK(c, launch_bulk(c->P, p.storage, c->parity, full_u, scale, c->L, false, s));
            c->parity ^= 1;
            ++c->step;
        }
        c->u_valid = true;
        return IBLB_OK;
    }
    // the step's arrays inside the fixed scratch; the records that must
    // start empty are cleared by a fill kernel (the scratch keeps whatever
    // the last call on this device left)
    DevPtrs V = c->P;
    char *const S = c->scratch;
    V.trec = S + p.st_trec;
    V.tri_part = (double *)(S + p.st_tri_part);
    V.bbox = (int32_t *)(S + p.st_bbox);
    V.breg = (int32_t *)(S + p.st_breg);
    V.part = S + p.st_part;
    V.tile_list = (int32_t *)(S + p.st_tile_list);
    V.tile_count = (int32_t *)(S + p.st_tile_count);
    V.tcand = (int32_t *)(S + p.st_tcand);
    V.tncand = (int32_t *)(S + p.st_tncand);
    V.scan_all = (int32_t *)(S + p.st_scan);
    HIPCHK(c, launch_fill_i32(V.tncand, 0, 2 * (int64_t)p.total_tiles, s));
    HIPCHK(c, launch_fill_i32(V.tile_count, 0, 2, s));
    HIPCHK(c, launch_fill_i32(V.scan_all, 0, 2 * (int64_t)p.boxes.size(), s));
    // one queue, in order: mesh chain, band tiles, every other cell, then the
    // advection (none is left pending)
    for (int64_t k = 0; k < n; ++k) {
        const int par = c->parity;
        const iblb_status st = compute_masks(c, par, s);  // inside bits: workspace arrays only
        if (st != IBLB_OK) return st;
        HIPCHK(c, launch_tri(V, f64, s));
        HIPCHK(c, launch_node(V, f64, 0, par, s));
        HIPCHK(c, launch_band(V, p.storage, par, full_u, scale, true, c->L.nt, s));
        HIPCHK(c, launch_bulk(V, p.storage, par, full_u, scale, c->L, true, s));
        HIPCHK(c, launch_interp(V, f64, 0, nullptr, s));
        c->last_step_epoch = c->epoch;
        c->last_step_parity = par;
        ++c->epoch;  // the advection starts the next epoch
        c->parity ^= 1;
        ++c->step;
    }
    c->u_valid = true;
    // the workspace's records start empty for a later iblb_step
    HIPCHK(c, launch_fill_i32(c->P.tncand, 0, 2 * (int64_t)p.total_tiles, s));
    HIPCHK(c, launch_fill_i32(c->P.tile_count, 0, 2, s));
    HIPCHK(c, launch_fill_i32(c->P.scan_all, 0, 2 * (int64_t)p.boxes.size(), s));
    return IBLB_OK;
}

iblb_status iblb_observables(iblb_ctx *c, iblb_obs *per_drop, int32_t n_drops, iblb_box_obs *per_box,
                             int32_t n_boxes) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if ((per_drop && n_drops != c->P.n_drops) || (per_box && n_boxes != c->P.n_boxes))
        return set_err(c, IBLB_E_INVAL, "output counts do not match the configuration");
    {
        iblb_status st = flush(c);
        if (st != IBLB_OK) return st;
    }
    HIPCHK(c, launch_box_obs(c->P, c->plan.storage, c->parity, (float)(1.0 / c->plan.scale), c->stream));
    HIPCHK(c, launch_drop_obs(c->P, is_f64(c), c->stream));
    const size_t nobs = (size_t)c->P.n_drops * OBS_DROP + (size_t)c->P.n_boxes * OBS_BOX;
    HIPCHK(c, hipMemcpyAsync(c->host_obs, c->P.obs_out, nobs * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->host_status, c->P.status, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const uint32_t bits = *c->host_status;
    if (per_drop)
        for (int d = 0; d < c->P.n_drops; ++d) {
            const double *o = c->host_obs + (size_t)d * OBS_DROP;
            iblb_obs &r = per_drop[d];
            r.step = c->step;
            r.volume = o[0];
            r.area = o[1];
            r.z_min = o[2];
            r.z_max = o[3];
            r.height = o[3] - o[2];
            r.centroid[0] = o[4];
            r.centroid[1] = o[5];
            r.centroid[2] = o[6];
            r.n_crossings = (int32_t)o[8];
            r.contact_radius = o[8] > 0 ? o[7] / o[8] : 0.0;
            r.theta_app = r.contact_radius > 0 ? 2.0 * std::atan(r.height / r.contact_radius) : 0.0;
            // second moments about the volume centroid, x-z block; its
            // eigenvalues are r^2 / 5 of the equivalent ellipsoid's semi-axes
            {
                const double V = o[9], cx = o[10] / V, cz = o[12] / V;
                const double sxx = o[13] / V - cx * cx, szz = o[15] / V - cz * cz, sxz = o[17] / V - cx * cz;
                const double h = 0.5 * (sxx + szz), d = std::sqrt(0.25 * (sxx - szz) * (sxx - szz) + sxz * sxz);
                const double r1 = std::sqrt(5.0 * (h + d)), r3 = std::sqrt(std::max(5.0 * (h - d), 0.0));
                r.deformation = (r1 - r3) / (r1 + r3);
                r.inclination = 0.5 * std::atan2(2.0 * sxz, sxx - szz);
            }
            r.status_bits = bits;
        }
    if (per_box)
        for (int b = 0; b < c->P.n_boxes; ++b) {
            const double *o = c->host_obs + (size_t)c->P.n_drops * OBS_DROP + (size_t)b * OBS_BOX;
            per_box[b].step = c->step;
            per_box[b].mass = o[0];
            per_box[b].max_u = o[1];
            per_box[b].status_bits = bits;
            per_box[b].reserved = 0;
        }
    if (bits) {
        c->unstable = true;
        return set_err(c, IBLB_E_UNSTABLE, "device status bits 0x" + std::to_string(bits) +
                                               " (1 rho, 2 Mach, 4 wall, 8 jump)");
    }
    return IBLB_OK;
}

// Moving-wall term of population i reflected at the lower (z = 0) or upper
// wall: 6 w_i rho0 (c_i . u_w).
double wall_term(const iblb_box &b, int i, bool lower) {
    const double *u = lower ? b.wall_lo : b.wall_hi;
    return 6.0 * w_of(i) * b.rho0 * (cx_of(i) * u[0] + cy_of(i) * u[1]);
}

iblb_status iblb_read_window(iblb_ctx *c, int32_t box, const int32_t *lo, const int32_t *ext, double *f_out,
                             double *u_out) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (box < 0 || box >= c->P.n_boxes || (!f_out && !u_out) || !lo || !ext)
        return set_err(c, IBLB_E_INVAL, "bad box, window or outputs");
    const BoxHost &H = c->plan.boxes[box];
    const int nx = H.b.nx, ny = H.b.ny, nz = H.b.nz;
    const bool zper = H.b.zbc == IBLB_Z_PERIODIC;
    if (ext[0] < 1 || ext[1] < 1 || ext[2] < 1 || ext[0] > nx || ext[1] > ny || ext[2] > nz ||
        (!zper && (lo[2] < 0 || lo[2] + ext[2] > nz)))
        return set_err(c, IBLB_E_INVAL, "window outside the box (1 <= extent <= size; z inside a walled box)");
    {
        iblb_status fst = flush(c);
        if (fst != IBLB_OK) return fst;
    }
    const int ex = ext[0], ey = ext[1], ez = ext[2];
    const size_t wcells = (size_t)ex * ey * ez;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (f_out) {
        // the planes' rows from one cell below the window to one above it
        // (every row when a periodic window touches the z ends)
        const size_t eb = elem_bytes(c->plan.storage);
        int za = lo[2] - 1, zb = lo[2] + ez;
        if (zper && (za < 0 || zb >= nz)) {
            za = 0;
            zb = nz - 1;
        }
        za = std::max(za, 0);
        zb = std::min(zb, nz - 1);
        const size_t row = (size_t)H.sx * eb, slab = (size_t)(zb - za + 1) * ny * row;
        std::vector<char> raw((size_t)Q * slab);
        for (int i = 0; i < Q; ++i)
            HIPCHK(c, hipMemcpy(raw.data() + (size_t)i * slab,
                                c->ws + H.off_f[c->parity] + ((size_t)i * H.plane + (size_t)za * ny * H.sx) * eb, slab,
                                hipMemcpyDeviceToHost));
        const size_t pstride = slab / eb;  // elements per plane in raw
        for (int wz = 0; wz < ez; ++wz)
            for (int wy = 0; wy < ey; ++wy)
                for (int wx = 0; wx < ex; ++wx) {
                    const int z = zper ? wrap(lo[2] + wz, nz) : lo[2] + wz;
                    const int y = wrap(lo[1] + wy, ny), x = wrap(lo[0] + wx, nx);
                    const size_t cell = ((size_t)wz * ey + wy) * ex + wx;
                    for (int i = 0; i < Q; ++i) {
                        const int zs = z - cz_of(i);
                        size_t src;
                        double wall = 0.0;
                        if (!zper && (zs < 0 || zs >= nz)) {
                            src = (size_t)opp_of(i) * pstride + ((size_t)(z - za) * ny + y) * H.sx + x;
                            wall = wall_term(H.b, i, zs < 0);
                        } else {
                            src = (size_t)i * pstride +
                                  ((size_t)(wrap(zs, nz) - za) * ny + wrap(y - cy_of(i), ny)) * H.sx +
                                  wrap(x - cx_of(i), nx);
                        }
                        f_out[(size_t)i * wcells + cell] = w_of(i) * H.b.rho0 + (decode(c, raw.data(), src) + wall);
                    }
                }
    }
    if (u_out && (c->plan.flags & IBLB_FLAG_FULL_U)) {
        const int R = c->plan.real;
        std::vector<char> uf((size_t)3 * H.plane * R);
        HIPCHK(c, hipMemcpy(uf.data(), c->ws + H.off_ufull, uf.size(), hipMemcpyDeviceToHost));
        for (int a = 0; a < 3; ++a)
            for (int wz = 0; wz < ez; ++wz)
                for (int wy = 0; wy < ey; ++wy)
                    for (int wx = 0; wx < ex; ++wx) {
                        const int z = wrap(lo[2] + wz, nz), y = wrap(lo[1] + wy, ny), x = wrap(lo[0] + wx, nx);
                        const size_t k = (size_t)a * H.plane + ((size_t)z * ny + y) * H.sx + x;
                        const double v = R == 8 ? ((double *)uf.data())[k] : ((float *)uf.data())[k];
                        u_out[(size_t)a * wcells + ((size_t)wz * ey + wy) * ex + wx] = c->u_valid ? v : NAN;
                    }
    } else if (u_out) {
        const int R = c->plan.real;
        std::vector<char> ub((size_t)H.n_tiles * 3 * TILE_CELLS * R);
        std::vector<int32_t> stamp(H.n_tiles);
        HIPCHK(c, hipMemcpy(ub.data(), c->ws + H.off_u, ub.size(), hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(stamp.data(), c->ws + H.off_stamp[c->last_step_parity], stamp.size() * 4,
                            hipMemcpyDeviceToHost));
        for (int wz = 0; wz < ez; ++wz)
            for (int wy = 0; wy < ey; ++wy)
                for (int wx = 0; wx < ex; ++wx) {
                    const int z = wrap(lo[2] + wz, nz), y = wrap(lo[1] + wy, ny), x = wrap(lo[0] + wx, nx);
                    const size_t cell = ((size_t)wz * ey + wy) * ex + wx;
                    const size_t tile = (size_t)band_tile(x, y, z, H.tnx, H.tny);
                    const int loc = band_loc(x, y, z);
                    const bool ok = c->last_step_epoch >= 0 && stamp[tile] == c->last_step_epoch;
                    for (int a = 0; a < 3; ++a) {
                        const size_t k = (tile * 3 + a) * TILE_CELLS + loc;
                        const double v = R == 8 ? ((const double *)ub.data())[k] : ((const float *)ub.data())[k];
                        u_out[(size_t)a * wcells + cell] = ok ? v : NAN;
                    }
                }
    }
    return IBLB_OK;
}

iblb_status iblb_read_state(iblb_ctx *c, int32_t box, double *f_out, double *u_out) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (box < 0 || box >= c->P.n_boxes) return set_err(c, IBLB_E_INVAL, "bad box or outputs");
    const iblb_box &B = c->plan.boxes[box].b;
    const int32_t lo[3] = {0, 0, 0}, ext[3] = {B.nx, B.ny, B.nz};
    return iblb_read_window(c, box, lo, ext, f_out, u_out);
}

iblb_status iblb_write_state(iblb_ctx *c, int32_t box, const double *f_in) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (box < 0 || box >= c->P.n_boxes || !f_in) return set_err(c, IBLB_E_INVAL, "bad box or input");
    {
        iblb_status fst = flush(c);
        if (fst != IBLB_OK) return fst;
    }
    const BoxHost &H = c->plan.boxes[box];
    const int nx = H.b.nx, ny = H.b.ny, nz = H.b.nz;
    const size_t cells = (size_t)nx * ny * nz;
    for (size_t k = 0; k < (size_t)Q * cells; ++k)
        if (!std::isfinite(f_in[k])) return set_err(c, IBLB_E_INVAL, "populations not finite");
    const size_t eb = elem_bytes(c->plan.storage);
    std::vector<char> raw((size_t)Q * H.plane * eb, 0);
    const bool zper = H.b.zbc == IBLB_Z_PERIODIC;
    // inverse of the pull: the stored value at (i, y) is f_i(y + c_i), or,
    // where y + c_i lies in a wall, f_opp(i)(y)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                for (int i = 0; i < Q; ++i) {
                    const int zt = z + cz_of(i);
                    double v;
                    if (!zper && (zt < 0 || zt >= nz))
                        v = f_in[(size_t)opp_of(i) * cells + ((size_t)z * ny + y) * nx + x] -
                            wall_term(H.b, opp_of(i), zt < 0);
                    else
                        v = f_in[(size_t)i * cells +
                                 ((size_t)wrap(zt, nz) * ny + wrap(y + cy_of(i), ny)) * nx +
                                 wrap(x + cx_of(i), nx)];
                    encode(c, raw.data(), (size_t)i * H.plane + ((size_t)z * ny + y) * H.sx + x,
                           v - w_of(i) * H.b.rho0);
                }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->ws + H.off_f[c->parity], raw.data(), raw.size(), hipMemcpyHostToDevice));
    return IBLB_OK;
}

iblb_status iblb_read_nodes(iblb_ctx *c, int32_t d, double *nodes_out) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (d < 0 || d >= c->P.n_drops || !nodes_out) return set_err(c, IBLB_E_INVAL, "bad droplet or output");
    {
        iblb_status fst = flush(c);
        if (fst != IBLB_OK) return fst;
    }
    const DropHost &H = c->plan.drops[d];
    const int N = c->P.Ntot, R = c->plan.real;
    std::vector<char> qh((size_t)3 * N * R), ql((size_t)3 * N * R);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(qh.data(), c->P.qh, qh.size(), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(ql.data(), c->P.ql, ql.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < H.d.n_nodes; ++k)
        for (int a = 0; a < 3; ++a) {
            const size_t idx = (size_t)a * N + H.node_off + k;
            nodes_out[3 * (size_t)H.perm[k] + a] =
                R == 8 ? ((double *)qh.data())[idx] + ((double *)ql.data())[idx]
                       : (double)((float *)qh.data())[idx] + (double)((float *)ql.data())[idx];
        }
    return IBLB_OK;
}

iblb_status iblb_write_nodes(iblb_ctx *c, int32_t d, const double *nodes_in) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (d < 0 || d >= c->P.n_drops || !nodes_in) return set_err(c, IBLB_E_INVAL, "bad droplet or input");
    {
        iblb_status fst = flush(c);
        if (fst != IBLB_OK) return fst;
    }
    const DropHost &H = c->plan.drops[d];
    const iblb_box &B = c->plan.boxes[H.d.box].b;
    for (int k = 0; k < 3 * H.d.n_nodes; ++k)
        if (!std::isfinite(nodes_in[k])) return set_err(c, IBLB_E_INVAL, "node coordinate not finite");
    if (B.zbc == IBLB_Z_WALLS)
        for (int k = 0; k < H.d.n_nodes; ++k)
            if (!(nodes_in[3 * k + 2] > 0.0 && nodes_in[3 * k + 2] < B.nz))
                return set_err(c, IBLB_E_MESH, "node not strictly between the walls");
    const int N = c->P.Ntot, R = c->plan.real;
    std::vector<char> qh((size_t)3 * N * R), ql((size_t)3 * N * R);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(qh.data(), c->P.qh, qh.size(), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(ql.data(), c->P.ql, ql.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < H.d.n_nodes; ++k)
        for (int a = 0; a < 3; ++a) {
            const size_t idx = (size_t)a * N + H.node_off + k;
            const double v = nodes_in[3 * (size_t)H.perm[k] + a];
            if (R == 8) {
                ((double *)qh.data())[idx] = v;
                ((double *)ql.data())[idx] = 0.0;
            } else {
                const float h = (float)v;
                ((float *)qh.data())[idx] = h;
                ((float *)ql.data())[idx] = (float)(v - (double)h);
            }
        }
    HIPCHK(c, hipMemcpy(c->P.qh, qh.data(), qh.size(), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->P.ql, ql.data(), ql.size(), hipMemcpyHostToDevice));
    // the next step's bulk collision reads the other set of inside bits
    const iblb_status st = compute_masks(c, c->parity ^ 1, c->stream);
    if (st != IBLB_OK) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return IBLB_OK;
}

iblb_status iblb_compute_forces(iblb_ctx *c, int32_t d, double *phi_out) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (d < 0 || d >= c->P.n_drops || !phi_out) return set_err(c, IBLB_E_INVAL, "bad droplet or output");
    {
        iblb_status fst = flush(c);
        if (fst != IBLB_OK) return fst;
    }
    const bool f64 = is_f64(c);
    HIPCHK(c, launch_tri(c->P, f64, c->stream));
    HIPCHK(c, launch_node(c->P, f64, 1, c->parity, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const DropHost &H = c->plan.drops[d];
    const int N = c->P.Ntot, R = c->plan.real;
    std::vector<char> phi((size_t)3 * N * R);
    HIPCHK(c, hipMemcpy(phi.data(), c->P.phi, phi.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < H.d.n_nodes; ++k)
        for (int a = 0; a < 3; ++a) {
            const size_t idx = (size_t)a * N + H.node_off + k;
            phi_out[3 * (size_t)H.perm[k] + a] =
                R == 8 ? ((double *)phi.data())[idx] : (double)((float *)phi.data())[idx];
        }
    return IBLB_OK;
}

iblb_status iblb_compute_spread(iblb_ctx *c, int32_t b, double *F_out, uint8_t *flags_out) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (b < 0 || b >= c->P.n_boxes || (!F_out && !flags_out)) return set_err(c, IBLB_E_INVAL, "bad box or outputs");
    {
        iblb_status fst = flush(c);
        if (fst != IBLB_OK) return fst;
    }
    const bool f64 = is_f64(c);
    HIPCHK(c, launch_tri(c->P, f64, c->stream));
    HIPCHK(c, launch_node(c->P, f64, 0, c->parity, c->stream));
    HIPCHK(c, launch_band(c->P, c->plan.storage, c->parity, 0, (float)c->plan.scale, false, 0, c->stream));
    HIPCHK(c, launch_epoch(c->P, c->stream));
    const int32_t used = c->epoch;
    ++c->epoch;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const BoxHost &H = c->plan.boxes[b];
    const int R = c->plan.real;
    std::vector<char> Fb(F_out ? (size_t)H.n_tiles * 3 * TILE_CELLS * R : 0);
    std::vector<int32_t> stamp(H.n_tiles);
    if (F_out) HIPCHK(c, hipMemcpy(Fb.data(), c->ws + H.off_F, Fb.size(), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(stamp.data(), c->ws + H.off_stamp[c->parity], stamp.size() * 4, hipMemcpyDeviceToHost));
    const int nx = H.b.nx, ny = H.b.ny, nz = H.b.nz;
    const size_t cells = (size_t)nx * ny * nz;
    if (flags_out)
        for (int t = 0; t < H.n_tiles; ++t) flags_out[t] = stamp[t] == used ? 1 : 0;
    if (F_out)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const size_t cell = ((size_t)z * ny + y) * nx + x;
                    const size_t tile = (size_t)band_tile(x, y, z, H.tnx, H.tny);
                    const int loc = band_loc(x, y, z);
                    for (int a = 0; a < 3; ++a) {
                        const size_t k = (tile * 3 + a) * TILE_CELLS + loc;
                        const double v = R == 8 ? ((double *)Fb.data())[k] : ((float *)Fb.data())[k];
                        F_out[(size_t)a * cells + cell] = stamp[tile] == used ? v : 0.0;
                    }
                }
    return IBLB_OK;
}

iblb_status iblb_interpolate(iblb_ctx *c, int32_t d, const double *u_in, double *U_out) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (d < 0 || d >= c->P.n_drops || !u_in || !U_out) return set_err(c, IBLB_E_INVAL, "bad droplet or arrays");
    {
        iblb_status fst = flush(c);
        if (fst != IBLB_OK) return fst;
    }
    const DropHost &Dh = c->plan.drops[d];
    const BoxHost &H = c->plan.boxes[Dh.d.box];
    const int nx = H.b.nx, ny = H.b.ny, nz = H.b.nz, R = c->plan.real;
    const size_t cells = (size_t)nx * ny * nz;
    std::vector<char> ub((size_t)H.n_tiles * 3 * TILE_CELLS * R, 0);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t cell = ((size_t)z * ny + y) * nx + x;
                const size_t tile = (size_t)band_tile(x, y, z, H.tnx, H.tny);
                const int loc = band_loc(x, y, z);
                for (int a = 0; a < 3; ++a) {
                    const size_t k = (tile * 3 + a) * TILE_CELLS + loc;
                    if (R == 8) ((double *)ub.data())[k] = u_in[(size_t)a * cells + cell];
                    else ((float *)ub.data())[k] = (float)u_in[(size_t)a * cells + cell];
                }
            }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->ws + H.off_u, ub.data(), ub.size(), hipMemcpyHostToDevice));
    const bool f64 = is_f64(c);
    double *Udev = (double *)(c->ws + c->plan.off_uout);
    HIPCHK(c, launch_tri(c->P, f64, c->stream));
    HIPCHK(c, launch_node(c->P, f64, 1, c->parity, c->stream));
    HIPCHK(c, launch_interp(c->P, f64, 1, Udev, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<double> U((size_t)3 * c->P.Ntot);
    HIPCHK(c, hipMemcpy(U.data(), Udev, U.size() * 8, hipMemcpyDeviceToHost));
    for (int k = 0; k < Dh.d.n_nodes; ++k)
        for (int a = 0; a < 3; ++a) U_out[3 * (size_t)Dh.perm[k] + a] = U[3 * (size_t)(Dh.node_off + k) + a];
    return IBLB_OK;
}

iblb_status iblb_read_bins(iblb_ctx *c, int32_t d, int32_t *base_out) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (d < 0 || d >= c->P.n_drops || !base_out) return set_err(c, IBLB_E_INVAL, "bad droplet or output");
    {
        iblb_status fst = flush(c);
        if (fst != IBLB_OK) return fst;
    }
    HIPCHK(c, launch_tri(c->P, is_f64(c), c->stream));
    HIPCHK(c, launch_node(c->P, is_f64(c), 1, c->parity, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const DropHost &H = c->plan.drops[d];
    const iblb_box &B = c->plan.boxes[H.d.box].b;
    const int N = c->P.Ntot;
    std::vector<int32_t> base((size_t)3 * N);
    HIPCHK(c, hipMemcpy(base.data(), c->P.base, base.size() * 4, hipMemcpyDeviceToHost));
    for (int k = 0; k < H.d.n_nodes; ++k) {
        const size_t u = 3 * (size_t)H.perm[k];
        base_out[u] = wrap(base[H.node_off + k], B.nx);
        base_out[u + 1] = wrap(base[(size_t)N + H.node_off + k], B.ny);
        base_out[u + 2] = base[2 * (size_t)N + H.node_off + k];
    }
    return IBLB_OK;
}

iblb_status iblb_read_inside(iblb_ctx *c, int32_t b, uint8_t *inside_out) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (b < 0 || b >= c->P.n_boxes || !inside_out) return set_err(c, IBLB_E_INVAL, "bad box or output");
    const BoxHost &H = c->plan.boxes[b];
    if (!(H.b.tau_in > 0.0)) return set_err(c, IBLB_E_INVAL, "box has no tau_in");
    {
        iblb_status fst = flush(c);
        if (fst != IBLB_OK) return fst;
    }
    // the next step recomputes this set before any kernel reads it
    {
        iblb_status st = compute_masks(c, c->parity, c->stream);
        if (st != IBLB_OK) return st;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int nx = H.b.nx, ny = H.b.ny, nz = H.b.nz;
    std::vector<uint64_t> m((size_t)H.nzw * ny * nx);
    HIPCHK(c, hipMemcpy(m.data(), c->ws + H.off_mask[c->parity], m.size() * 8, hipMemcpyDeviceToHost));
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x)
                inside_out[((size_t)z * ny + y) * nx + x] =
                    (uint8_t)((m[((size_t)(z >> 6) * ny + y) * nx + x] >> (z & 63)) & 1u);
    return IBLB_OK;
}

// ---------------------------------------------------------- checkpoints
// Blob: header, then per box its dimensions and the stored populations of
// the current time (raw storage bytes, padding included), the node
// positions as stored (hi and lo arrays), and per droplet its counts and
// reference volume V0.  A fingerprint of the configuration (box fields,
// storage, droplet parameters, node order and triangles) ties a blob to
// contexts built from the same configuration.
namespace {
struct StateHeader {
    char magic[8];
    uint64_t fingerprint;
    int64_t step;
    int32_t storage, n_boxes, n_drops, Ntot;
    uint32_t status;
    int32_t real;
};
constexpr char STATE_MAGIC[8] = {'I', 'B', 'L', 'B', 'S', 'T', '0', '1'};

uint64_t fnv(uint64_t h, const void *p, size_t n) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

uint64_t fingerprint(const iblb_ctx *c) {
    const Plan &p = c->plan;
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, &p.storage, sizeof p.storage);
    h = fnv(h, &p.scale, sizeof p.scale);
    for (const BoxHost &H : p.boxes) {
        const iblb_box &b = H.b;
        const int32_t dims[4] = {b.nx, b.ny, b.nz, b.zbc};
        const double prm[10] = {b.tau,    b.rho0,       b.body_force[0], b.body_force[1], b.body_force[2],
                                b.tau_in, b.wall_lo[0], b.wall_lo[1],    b.wall_hi[0],    b.wall_hi[1]};
        h = fnv(h, dims, sizeof dims);
        h = fnv(h, prm, sizeof prm);
    }
    for (const DropHost &D : p.drops) {
        const int32_t cnt[5] = {D.d.box, D.d.n_nodes, D.d.n_tris, D.d.n_exp, D.d.m_exp};
        const double prm[4] = {D.d.sigma, D.d.theta_eq, D.d.xi, D.d.k_vol};
        h = fnv(h, cnt, sizeof cnt);
        h = fnv(h, prm, sizeof prm);
        h = fnv(h, D.perm.data(), D.perm.size() * 4);
        h = fnv(h, D.tris.data(), D.tris.size() * 4);
    }
    return h;
}

size_t state_bytes(const iblb_ctx *c) {
    const Plan &p = c->plan;
    size_t n = sizeof(StateHeader);
    for (const BoxHost &H : p.boxes) n += 16 + (size_t)Q * H.plane * elem_bytes(p.storage);
    n += (size_t)2 * 3 * p.Ntot * p.real;
    n += (size_t)p.drops.size() * 16;
    return n;
}
}  // namespace

iblb_status iblb_state_size(const iblb_ctx *c, size_t *bytes) {
    if (!c || !bytes) return set_err(nullptr, IBLB_E_INVAL, "ctx or bytes is NULL");
    *bytes = state_bytes(c);
    return IBLB_OK;
}

iblb_status iblb_save_state(iblb_ctx *c, void *blob, size_t n) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (!blob || n != state_bytes(c)) return set_err(c, IBLB_E_INVAL, "blob is NULL or not iblb_state_size bytes");
    {
        iblb_status st = flush(c);
        if (st != IBLB_OK) return st;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const Plan &p = c->plan;
    char *o = (char *)blob;
    StateHeader hd{};
    std::memcpy(hd.magic, STATE_MAGIC, 8);
    hd.fingerprint = fingerprint(c);
    hd.step = c->step;
    hd.storage = p.storage;
    hd.n_boxes = (int32_t)p.boxes.size();
    hd.n_drops = (int32_t)p.drops.size();
    hd.Ntot = p.Ntot;
    hd.real = p.real;
    HIPCHK(c, hipMemcpy(&hd.status, c->P.status, 4, hipMemcpyDeviceToHost));
    std::memcpy(o, &hd, sizeof hd);
    o += sizeof hd;
    for (const BoxHost &H : p.boxes) {
        const int32_t dims[4] = {H.b.nx, H.b.ny, H.b.nz, H.b.zbc};
        std::memcpy(o, dims, 16);
        o += 16;
        const size_t bytes = (size_t)Q * H.plane * elem_bytes(p.storage);
        HIPCHK(c, hipMemcpy(o, c->ws + H.off_f[c->parity], bytes, hipMemcpyDeviceToHost));
        o += bytes;
    }
    const size_t qb = (size_t)3 * p.Ntot * p.real;
    HIPCHK(c, hipMemcpy(o, c->P.qh, qb, hipMemcpyDeviceToHost));
    o += qb;
    HIPCHK(c, hipMemcpy(o, c->P.ql, qb, hipMemcpyDeviceToHost));
    o += qb;
    std::vector<DropDev> dd(p.drops.size());
    if (!dd.empty())
        HIPCHK(c, hipMemcpy(dd.data(), c->P.drops, dd.size() * sizeof(DropDev), hipMemcpyDeviceToHost));
    for (size_t d = 0; d < p.drops.size(); ++d) {
        const int32_t cnt[2] = {p.drops[d].d.n_nodes, p.drops[d].d.n_tris};
        std::memcpy(o, cnt, 8);
        std::memcpy(o + 8, &dd[d].V0, 8);
        o += 16;
    }
    return IBLB_OK;
}

iblb_status iblb_load_state(iblb_ctx *c, const void *blob, size_t n) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (!blob || n != state_bytes(c)) return set_err(c, IBLB_E_INVAL, "blob is NULL or not iblb_state_size bytes");
    const Plan &p = c->plan;
    const char *o = (const char *)blob;
    StateHeader hd;
    std::memcpy(&hd, o, sizeof hd);
    o += sizeof hd;
    if (std::memcmp(hd.magic, STATE_MAGIC, 8) != 0) return set_err(c, IBLB_E_INVAL, "not an iblb state blob");
    if (hd.fingerprint != fingerprint(c) || hd.storage != p.storage || hd.n_boxes != (int32_t)p.boxes.size() ||
        hd.n_drops != (int32_t)p.drops.size() || hd.Ntot != p.Ntot || hd.real != p.real || hd.step < 0)
        return set_err(c, IBLB_E_INVAL, "the blob was saved from a different configuration");
    {
        iblb_status st = flush(c);  // no advection may be left pending
        if (st != IBLB_OK) return st;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (const BoxHost &H : p.boxes) {
        int32_t dims[4];
        std::memcpy(dims, o, 16);
        o += 16;
        if (dims[0] != H.b.nx || dims[1] != H.b.ny || dims[2] != H.b.nz || dims[3] != H.b.zbc)
            return set_err(c, IBLB_E_INVAL, "the blob was saved from a different configuration");
        const size_t bytes = (size_t)Q * H.plane * elem_bytes(p.storage);
        HIPCHK(c, hipMemcpy(c->ws + H.off_f[c->parity], o, bytes, hipMemcpyHostToDevice));
        o += bytes;
    }
    const size_t qb = (size_t)3 * p.Ntot * p.real;
    HIPCHK(c, hipMemcpy(c->P.qh, o, qb, hipMemcpyHostToDevice));
    o += qb;
    HIPCHK(c, hipMemcpy(c->P.ql, o, qb, hipMemcpyHostToDevice));
    o += qb;
    for (size_t d = 0; d < p.drops.size(); ++d) {
        double V0;
        std::memcpy(&V0, o + 8, 8);
        o += 16;
        HIPCHK(c, hipMemcpy((char *)c->P.drops + d * sizeof(DropDev) + offsetof(DropDev, V0), &V0, 8,
                            hipMemcpyHostToDevice));
    }
    HIPCHK(c, hipMemcpy(c->P.status, &hd.status, 4, hipMemcpyHostToDevice));
    // both sets of inside bits from the loaded positions
    for (int k = 0; k < 2; ++k) {
        const iblb_status st = compute_masks(c, k, c->stream);
        if (st != IBLB_OK) return st;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->step = hd.step;
    c->pending = false;
    c->last_step_epoch = -1;
    c->u_valid = false;
    c->unstable = false;
    return IBLB_OK;
}

iblb_status iblb_read_csr(iblb_ctx *c, int32_t d, int32_t *offsets, int32_t *entries) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (d < 0 || d >= c->P.n_drops || !offsets || !entries) return set_err(c, IBLB_E_INVAL, "bad droplet or outputs");
    const DropHost &H = c->plan.drops[d];
    const int N = c->P.Ntot;
    std::vector<int32_t> off((size_t)N + 1), ent((size_t)3 * c->P.Ttot);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(off.data(), c->P.csr_off, off.size() * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(ent.data(), c->P.csr_ent, ent.size() * 4, hipMemcpyDeviceToHost));
    offsets[0] = 0;
    for (int u = 0; u < H.d.n_nodes; ++u) {
        const int k = H.node_off + H.inv[u];
        offsets[u + 1] = offsets[u] + (off[k + 1] - off[k]);
        for (int e = off[k]; e < off[k + 1]; ++e) {
            const int code = ent[e], t = code / 3;
            entries[offsets[u] + (e - off[k])] = 3 * (t - H.tri_off) + (code - 3 * t);
        }
    }
    return IBLB_OK;
}

iblb_status iblb_set_launch(iblb_ctx *c, int32_t bx, int32_t by, int32_t cpt, int32_t nt, int32_t maxg,
                            int32_t after) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    const Launch L{bx, by, 0, nt, cpt, maxg, after};
    if (const char *why = launch_problem(L)) return set_err(c, IBLB_E_INVAL, why);
    if (L.after && c->P.contrast)
        return set_err(c, IBLB_E_INVAL, "band_after_bulk needs a configuration without tau_in");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->L = L;
    iblb_status st = upload_rows(c);
    if (st == IBLB_OK) st = build_graphs(c);
    return st;
}

iblb_status iblb_get_launch(const iblb_ctx *c, int32_t *bx, int32_t *by, int32_t *cpt, int32_t *nt,
                            int32_t *maxg, int32_t *after) {
    if (!c || !bx || !by || !cpt || !nt || !maxg || !after) return set_err(nullptr, IBLB_E_INVAL, "NULL argument");
    *bx = c->L.bx;
    *by = c->L.by;
    *cpt = c->L.cpt;
    *nt = c->L.nt;
    *maxg = c->L.maxg;
    *after = c->L.after;
    return IBLB_OK;
}

iblb_status iblb_band_tile(int32_t *shape) {
    if (!shape) return set_err(nullptr, IBLB_E_INVAL, "NULL argument");
    shape[0] = TX;
    shape[1] = TY;
    shape[2] = TZ;
    return IBLB_OK;
}

iblb_status iblb_time_stream_collide(iblb_ctx *c, int32_t reps, double *ms) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (reps < 1 || !ms) return set_err(c, IBLB_E_INVAL, "reps >= 1 and an output are required");
    return time_k1(c, reps, ms);
}

iblb_status iblb_time_mesh_chain(iblb_ctx *c, int32_t reps, double *ms) {
    if (!c) return set_err(nullptr, IBLB_E_INVAL, "ctx is NULL");
    if (reps < 1 || !ms) return set_err(c, IBLB_E_INVAL, "reps >= 1 and an output are required");
    *ms = 0.0;
    if (c->plan.nblk == 0) return IBLB_OK;
    {
        iblb_status st = flush(c);
        if (st != IBLB_OK) return st;
    }
    const bool f64 = is_f64(c);
    double *Udev = (double *)(c->ws + c->plan.off_uout);
    EventPair ev;
    HIPCHK(c, hipEventCreate(&ev.a));
    HIPCHK(c, hipEventCreate(&ev.b));
    c->last_step_epoch = -1;  // the band velocities no longer match the stamps
    HIPCHK(c, hipEventRecord(ev.a, c->stream));
    for (int r = 0; r < reps; ++r) {
        // a fresh epoch each time, as the advection at the head of a step
        // starts one; the nodes do not move (interpolation into a scratch U)
        HIPCHK(c, launch_epoch(c->P, c->stream));
        ++c->epoch;
        iblb_status st = compute_masks(c, c->parity, c->stream);
        if (st != IBLB_OK) return st;
        HIPCHK(c, launch_tri(c->P, f64, c->stream));
        HIPCHK(c, launch_node(c->P, f64, 0, c->parity, c->stream));
        HIPCHK(c, launch_interp(c->P, f64, 1, Udev, c->stream));
    }
    HIPCHK(c, hipEventRecord(ev.b, c->stream));
    HIPCHK(c, hipEventSynchronize(ev.b));
    float t = 0;
    HIPCHK(c, hipEventElapsedTime(&t, ev.a, ev.b));
    *ms = (double)t / reps;
    return IBLB_OK;
}

iblb_status iblb_destroy(iblb_ctx *c) {
    if (!c) return IBLB_OK;
    drop_graphs(c);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    if (c->ib) (void)hipStreamDestroy(c->ib);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ev_chain) (void)hipEventDestroy(c->ev_chain);
    if (c->ev_bulk) (void)hipEventDestroy(c->ev_bulk);
    if (c->host_obs) (void)hipHostFree(c->host_obs);
    if (c->host_status) (void)hipHostFree(c->host_status);
    delete c;
    return IBLB_OK;
}

const char *iblb_last_error(const iblb_ctx *c) { return c ? c->err.c_str() : g_last_error.c_str(); }

}  // extern "C"
