// Mesh kernels of the IBLB wetting step (gfx950): per-triangle records,
// the node pass (interface forces, Peskin weights, tile stamps and the
// block-partial spread), the stamped-tile list, interpolation with forward
// Euler advection, the inside bits of the viscosity contrast, and the
// per-droplet observables.
#include "iblb_device.h"

namespace iblb {

// ------------------------------------------------------- per-triangle pass
// One thread per triangle (a,b,c): N = (q_b - q_a) x (q_c - q_a), area
// A_t = |N|/2, unit normal n_t, the volume-gradient share N/6 and the three
// corner forces -sigma dA_t/dq = (sigma/2)(q_prev - q_next) x n_t, stored as
// a record of five four-vectors per triangle for the node gather.  Also the FP64 volume
// sum_t (a-r).((b-r)x(c-r))/6 and area per chunk of 256 triangles
// (positions relative to the droplet's reference point r), fixed tree.

template <typename R>
__global__ void __launch_bounds__(256) k_tri(DevPtrs P) {
    __shared__ double sv[256], sa[256];
    const int ci = xcd_item(blockIdx.x, gridDim.x);
    const TriChunk ch = P.chunks[ci];
    const DropDev &D = P.drops[ch.drop];
    const R *qh = (const R *)P.qh, *ql = (const R *)P.ql;
    const int t = ch.t0 + threadIdx.x;
    const int N = P.Ntot;
    double v = 0.0, ar = 0.0;
    if (t < ch.t1) {
        const Node3<R> a = load_node(qh, ql, N, P.tri[3 * t]);
        const Node3<R> b = load_node(qh, ql, N, P.tri[3 * t + 1]);
        const Node3<R> c = load_node(qh, ql, N, P.tri[3 * t + 2]);
        R e1[3], e2[3], Nt[3], cb[3], ac[3], ba[3], f0[3], f1[3], f2[3];
        diff(b, a, e1);
        diff(c, a, e2);
        cross3(e1, e2, Nt);
        const R len = sqrt(Nt[0] * Nt[0] + Nt[1] * Nt[1] + Nt[2] * Nt[2]);
        const R il = R(1) / len;
        const R nt[3] = {Nt[0] * il, Nt[1] * il, Nt[2] * il};
        const R hs = R(0.5) * (R)D.sigma;
        diff(c, b, cb);
        diff(a, c, ac);
        diff(b, a, ba);
        cross3(cb, nt, f0);
        cross3(ac, nt, f1);
        cross3(ba, nt, f2);
        using V4 = typename Vec4<R>::T;
        V4 *tr = (V4 *)P.trec + (int64_t)t * (TREC / 4);
        tr[0] = V4{R(0.5) * len, nt[0], nt[1], nt[2]};
        tr[1] = V4{Nt[0] / R(6), Nt[1] / R(6), Nt[2] / R(6), R(0)};
        tr[2] = V4{hs * f0[0], hs * f0[1], hs * f0[2], R(0)};
        tr[3] = V4{hs * f1[0], hs * f1[1], hs * f1[2], R(0)};
        tr[4] = V4{hs * f2[0], hs * f2[1], hs * f2[2], R(0)};
        double p[3][3];
        const Node3<R> *abc[3] = {&a, &b, &c};
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                p[cc][k] = ((double)abc[cc]->h[k] + (double)abc[cc]->l[k]) - D.ref[k];
        const double bc0 = p[1][1] * p[2][2] - p[1][2] * p[2][1];
        const double bc1 = p[1][2] * p[2][0] - p[1][0] * p[2][2];
        const double bc2 = p[1][0] * p[2][1] - p[1][1] * p[2][0];
        v = (p[0][0] * bc0 + p[0][1] * bc1 + p[0][2] * bc2) / 6.0;
        double d1[3], d2[3];
        for (int k = 0; k < 3; ++k) {
            d1[k] = p[1][k] - p[0][k];
            d2[k] = p[2][k] - p[0][k];
        }
        const double n0 = d1[1] * d2[2] - d1[2] * d2[1];
        const double n1 = d1[2] * d2[0] - d1[0] * d2[2];
        const double n2 = d1[0] * d2[1] - d1[1] * d2[0];
        ar = 0.5 * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    }
    sv[threadIdx.x] = v;
    sa[threadIdx.x] = ar;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            sv[threadIdx.x] += sv[threadIdx.x + k];
            sa[threadIdx.x] += sa[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        P.tri_part[ci] = sv[0];
        P.tri_part[P.n_chunks + ci] = sa[0];
    }
}

// V0 of each droplet = the same fixed-order sum the volume penalty uses.
__global__ void __launch_bounds__(64) k_set_v0(DevPtrs P) {
    DropDev *D = P.drops + blockIdx.x;
    const double V = droplet_partial_sum(P.tri_part, D->chunk_off, D->n_chunks, threadIdx.x);
    if (threadIdx.x == 0) D->V0 = V;
}

// -------------------------------------------------------------- node pass
// One wavefront (workgroup) per block of 64 nodes.  Per node: gather over
// its incident triangles (CSR, ascending triangle id) the corner
// surface-tension forces, the 1-ring area chi, the sum of unit face normals
// and the volume gradient; then the wetting force -chi Pi(d) n/3 with Pi
// from integer powers (Eq. 10) and the optional volume penalty.  Also: base
// cell floor(q - 1/2) (decided exactly from the hi/lo pair), the four
// Peskin weights per axis and the block's stencil bounding box.  Mode 0
// (a time step) also stamps every tile holding a stencil cell with the
// epoch and spreads the block's forces (Eq. 8) into an LDS copy of its
// stencil box, node by node in ascending order (each lane one of the 64
// stencil points, so no two lanes touch the same cell; node data are read
// from LDS as broadcasts), then writes that partial region out for the tile
// gather.
template <typename R, int NR>
__global__ void __launch_bounds__(64 * NR) k_node(DevPtrs P, int mode, int parity) {
    // NR waves spread NB / NR nodes each into their own LDS copy of the
    // region (NR = 1 keeps the LDS small when there are many more blocks
    // than compute units, NR > 1 shortens a block when there are few)
    constexpr int NT = 64 * NR;
    __shared__ R reg[NR][3 * MAXP];
    __shared__ R nw[12][NB], nf[3][NB];
    __shared__ int nbs[3][NB];
    __shared__ int sreg[5];  // ex, ey, ez, overflow, nodes in the block
    __shared__ int tlist[3][64];  // distinct tiles per axis of the block's stencil box
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int blk = xcd_item(blockIdx.x, gridDim.x);
    // droplet and box in one load, so their records load side by side
    const int d = P.blk_drop[2 * blk], bi = P.blk_drop[2 * blk + 1];
    const DropDev &D = P.drops[d];
    if (wave == 0) {  // the node pass: one lane per node
        const BoxDev &B = P.boxes[bi];
        // every constant of the droplet and its box is read here, before the
        // first store (a scalar load behind vector stores waits for them)
        const int nx = B.nx, ny = B.ny, nz = B.nz, tnx = B.tnx, tny = B.tny, tile_base = B.tile_base;
        const bool records = box_records(B.blk_begin, B.blk_end);
        const bool zper = B.zbc == 1;
        IBLB_GLOBAL int32_t *const stamp = (IBLB_GLOBAL int32_t *)B.stamp[parity];
        const int node_off = D.node_off, n_nodes = D.n_nodes, n_exp = D.n_exp, m_exp = D.m_exp;
        const int chunk_off = D.chunk_off, n_chunks = D.n_chunks;
        const double kvol = D.kvol, V0 = D.V0, Aw = D.A, xi = D.xi;
        const int N = P.Ntot;
        const R *qh = (const R *)P.qh, *ql = (const R *)P.ql;
        using V4 = typename Vec4<R>::T;
        const V4 *tr = (const V4 *)P.trec;
        const int j = blk * NB + lane;
        const bool valid = (j - node_off) < n_nodes;
        const int dims[3] = {nx, ny, nz};
        const int ctr = mode == 0 ? *P.ctr : 0;
        // the stream-collide of this step skips the tiles stamped with this
        // epoch (the band kernel owns them); it finds the epoch here
        if (mode == 0 && blk == 0 && lane == 0) P.step_epoch[parity] = ctr;
        double dV = 0.0;
        if (kvol > 0.0) {
            const double V = droplet_partial_sum(P.tri_part, chunk_off, n_chunks, lane);
            dV = (V - V0) / V0;
        }
        int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
        R w[12], f[3];
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] = 0;
        f[0] = f[1] = f[2] = 0;
        int b[3] = {0, 0, 0};
        if (valid) {
            const Node3<R> qj = load_node(qh, ql, N, j);
            R st[3] = {0, 0, 0}, ns[3] = {0, 0, 0}, gv[3] = {0, 0, 0};
            R chi = 0;
            // batches of incident records: every load of a batch is issued
            // (entries past the degree read triangle 0 and are not added)
            // before the first is added, in ascending triangle order
            constexpr int GB = sizeof(R) == 4 ? 8 : 4;
            const int e0 = P.csr_off[j], e1 = P.csr_off[j + 1];
            for (int e = e0; e < e1; e += GB) {
                int code[GB];
#pragma unroll
                for (int k = 0; k < GB; ++k) code[k] = e + k < e1 ? P.csr_ent[e + k] : -1;
                V4 r0[GB], r1[GB], rf[GB];
#pragma unroll
                for (int k = 0; k < GB; ++k) {
                    const int cd = code[k] < 0 ? 0 : code[k];
                    const int t = cd / 3, c = cd - 3 * t;
                    r0[k] = tr[(int64_t)t * (TREC / 4)];
                    r1[k] = tr[(int64_t)t * (TREC / 4) + 1];
                    rf[k] = tr[(int64_t)t * (TREC / 4) + 2 + c];
                }
#pragma unroll
                for (int k = 0; k < GB; ++k) {
                    if (code[k] < 0) continue;
                    chi += r0[k].x;
                    ns[0] += r0[k].y;
                    ns[1] += r0[k].z;
                    ns[2] += r0[k].w;
                    gv[0] += r1[k].x;
                    gv[1] += r1[k].y;
                    gv[2] += r1[k].z;
                    st[0] += rf[k].x;
                    st[1] += rf[k].y;
                    st[2] += rf[k].z;
                }
            }
            const R nl = R(1) / sqrt(ns[0] * ns[0] + ns[1] * ns[1] + ns[2] * ns[2]);
            const R dist = qj.h[2] + qj.l[2];
            if (!(dist > R(0))) atomicOr(P.status, BIT_WALL);
            const R rr = (R)xi / dist;
            R pn = 1, pm = 1;
            for (int k = 0; k < n_exp; ++k) pn *= rr;
            for (int k = 0; k < m_exp; ++k) pm *= rr;
            const R Pi = (R)Aw * (pn - pm);
            const R kw = chi * Pi / R(3) * nl;
            const R kv = (R)(-kvol * dV);
            R *phi = (R *)P.phi;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                f[k] = st[k] - kw * ns[k] + kv * gv[k];
                phi[k * N + j] = f[k];
            }

            // base cell and Peskin 4-point weights per axis.  With t = q - b - 1/2
            // in [0,1] all four weights share s = sqrt(1 + 4t(1-t)):
            //   b-1: (3 - 2t - s)/8, b: (3 - 2t + s)/8, b+1: (1 + 2t + s)/8,
            //   b+2: (1 + 2t - s)/8.
            R *wg = (R *)P.wgt;
            int s0[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                R qa = qj.h[a], la = qj.l[a];
                if (!(fabs(qa) < R(1.0e7))) {  // non-finite or absurd: flag, keep indices sane
                    atomicOr(P.status, BIT_JUMP);
                    qa = R(0.5);
                    la = R(0);
                }
                const R fl = floor(qa);
                const R rf = (qa - fl - R(0.5)) + la;
                const bool neg = rf < R(0);
                b[a] = (int)fl - (neg ? 1 : 0);
                const R t = neg ? rf + R(1) : rf;
                const R s = sqrt(R(1) + R(4) * t * (R(1) - t));
                w[4 * a + 0] = (R(3) - R(2) * t - s) * R(0.125);
                w[4 * a + 1] = (R(3) - R(2) * t + s) * R(0.125);
                w[4 * a + 2] = (R(1) + R(2) * t + s) * R(0.125);
                w[4 * a + 3] = (R(1) + R(2) * t - s) * R(0.125);
#pragma unroll
                for (int o = 0; o < 4; ++o) wg[(4 * a + o) * N + j] = w[4 * a + o];
                P.base[a * N + j] = b[a];
                const bool per = a < 2 || zper;
                s0[a] = per ? wrapn(b[a] - 1, dims[a]) : b[a] - 1;
                P.s0[a * N + j] = s0[a];
                lo[a] = b[a] - 1;
                hi[a] = b[a] + 2;
            }
            if (mode == 0) {
                // epoch stamp of every tile holding a stencil cell (same value
                // from every writer, so plain stores).  Per axis the four
                // stencil cells from s0 (wrapped on a periodic axis; cells in
                // a wall are left out) and the tile of each, kept where it
                // differs from the tiles of the cells before it
                int t3[3][4];
                bool u3[3][4];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int sh = a == 0 ? TXS : (a == 1 ? TYS : TZS);
                    const bool per = a < 2 || zper;
#pragma unroll
                    for (int o = 0; o < 4; ++o) {
                        int c = s0[a] + o;
                        if (per && c >= dims[a]) c -= dims[a];
                        const bool v = c >= 0 && c < dims[a];
                        t3[a][o] = c >> sh;
                        bool fresh = v;
#pragma unroll
                        for (int k = 0; k < o; ++k) fresh = fresh && !(u3[a][k] && t3[a][k] == t3[a][o]);
                        u3[a][o] = fresh;
                    }
                }
#pragma unroll
                for (int iz = 0; iz < 4; ++iz)
#pragma unroll
                    for (int iy = 0; iy < 4; ++iy)
#pragma unroll
                        for (int ix = 0; ix < 4; ++ix)
                            if (u3[2][iz] && u3[1][iy] && u3[0][ix])
                                stamp[((int64_t)t3[2][iz] * tny + t3[1][iy]) * tnx + t3[0][ix]] = ctr;
            }
        }
        // stencil bounding box of the block (unwrapped cell indices)
        int bl[3], bh[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            bl[a] = wave_min(lo[a]);
            bh[a] = wave_max(hi[a]);
            if (lane == 0) {
                P.bbox[(2 * a) * P.nblk + blk] = bl[a];
                P.bbox[(2 * a + 1) * P.nblk + blk] = bh[a];
            }
        }
        if (mode != 0) return;
        // partial spread over the block's stencil box
        int zl = bl[2], zh = bh[2];
        if (!zper) {
            zl = max(zl, 0);
            zh = min(zh, nz - 1);
        }
        const int ex = bh[0] - bl[0] + 1, ey = bh[1] - bl[1] + 1, ez = zh - zl + 1;
        const bool ovf = ex > nx || ey > ny || (zper && ez > nz) || ez < 1 ||
                         (int64_t)ex * ey * ez > MAXP;
        // every band tile that the stencil box covers records the block (slot
        // from an integer counter; the gather sorts the ids, so the order of
        // the records does not matter, but each tile must list a block once);
        // a box covering more than 64 tiles on an axis, or none (all stencil
        // cells in a wall), makes its box's gather scan
        if (mode == 0 && records) {
            const int slot = ctr & 1;
            const int lo3[3] = {bl[0], bl[1], zl}, hi3[3] = {bh[0], bh[1], zh};
            int ntl[3];
            bool ok = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const bool per = a < 2 || zper;
                const int sh = a == 0 ? TXS : (a == 1 ? TYS : TZS);
                const int nta = (dims[a] + (1 << sh) - 1) >> sh;
                const TileRun run = tile_run(per ? wrapn(lo3[a], dims[a]) : lo3[a], hi3[a] - lo3[a] + 1,
                                             dims[a], sh, per);
                ntl[a] = run.count;
                if (run.count < 1 || run.count > 64) {
                    ok = false;
                    continue;
                }
                if (lane < run.count) {
                    const int t = run.first + lane;
                    tlist[a][lane] = t >= nta ? t - nta : t;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (ok) {
                const int nt = ntl[0] * ntl[1] * ntl[2];
                for (int k = lane; k < nt; k += 64) {
                    const int ix = k % ntl[0], iy = (k / ntl[0]) % ntl[1], iz = k / (ntl[0] * ntl[1]);
                    const int gt = tile_base + (tlist[2][iz] * tny + tlist[1][iy]) * tnx + tlist[0][ix];
                    const int pos = atomicAdd(P.tncand + (int64_t)slot * P.total_tiles + gt, 1);
                    if (pos < MAXC) P.tcand[(int64_t)gt * MAXC + pos] = blk;
                }
            } else if (lane == 0) {
                P.scan_all[slot * P.n_boxes + bi] = 1;
            }
        }
        if (lane == 0) {
            int32_t *br = P.breg + (int64_t)blk * BREG;
            br[0] = wrapn(bl[0], nx);
            br[1] = wrapn(bl[1], ny);
            br[2] = zper ? wrapn(zl, nz) : zl;
            br[3] = ex;
            br[4] = ey;
            br[5] = ez;
            br[6] = ovf ? 1 : 0;
            br[7] = 0;
            sreg[0] = ex;
            sreg[1] = ey;
            sreg[2] = ez;
            sreg[3] = ovf ? 1 : 0;
            sreg[4] = min(NB, n_nodes - (blk * NB - node_off));
        }
        // the block's node data, read back by the spreading waves as broadcasts
#pragma unroll
        for (int k = 0; k < 12; ++k) nw[k][lane] = w[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            nf[k][lane] = f[k];
            nbs[k][lane] = b[k] - 1 - (k == 0 ? bl[0] : (k == 1 ? bl[1] : zl));
        }
    }  // wave 0
    if (mode != 0) return;
    __syncthreads();
    const int ex = sreg[0], ey = sreg[1], ez = sreg[2];
    if (sreg[3]) return;
    const int ncell = ex * ey * ez, nvalid = sreg[4];
    for (int c = tid; c < ncell; c += NT)
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            reg[r][c] = R(0);
            reg[r][MAXP + c] = R(0);
            reg[r][2 * MAXP + c] = R(0);
        }
    __syncthreads();
    // wave r < NR adds nodes [r NB/NR, (r+1) NB/NR) in ascending order; each
    // lane is one of a node's 64 stencil points, so no two lanes of a wave
    // touch the same cell
    if (wave < NR) {
        const int ox = lane & 3, oy = (lane >> 2) & 3, oz = lane >> 4;
        R *rg = reg[wave];
        const int n1 = min((wave + 1) * (NB / NR), nvalid);
        for (int nl = wave * (NB / NR); nl < n1; ++nl) {
            const int rz = nbs[2][nl] + oz;  // region coordinates of this lane's stencil cell
            const int ry = nbs[1][nl] + oy;
            const int rx = nbs[0][nl] + ox;
            const R wv = nw[ox][nl] * nw[4 + oy][nl] * nw[8 + oz][nl];
            if (rz >= 0 && rz < ez) {  // outside only for wall layers (dropped)
                const int c = (rz * ey + ry) * ex + rx;
                rg[c] += nf[0][nl] * wv;
                rg[MAXP + c] += nf[1][nl] * wv;
                rg[2 * MAXP + c] += nf[2][nl] * wv;
            }
        }
    }
    __syncthreads();
    // block partial = region 0 + region 1 + ... (fixed order), written with
    // the three components of a cell side by side: the band gather reads a
    // run of a region row as one contiguous stretch of lines
    IBLB_GLOBAL R *out = (IBLB_GLOBAL R *)P.part + (int64_t)blk * 3 * MAXP;
    for (int c = tid; c < ncell; c += NT)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            R v = reg[0][k * MAXP + c];
#pragma unroll
            for (int r = 1; r < NR; ++r) v += reg[r][k * MAXP + c];
            out[3 * c + k] = v;
        }
}

// ----------------------------------------------------- stamped-tile list
// One wavefront per chunk of 64 tiles appends the chunk's stamped tiles to
// the list of this epoch (one integer atomic per chunk; the order of the
// list does not affect any result).  Also clears the other epoch's count.
__global__ void __launch_bounds__(256) k_compact(DevPtrs P, int parity) {
    const int lane = threadIdx.x & 63;
    const int c = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int ctr = *P.ctr;
    const int slot = ctr & 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P.tile_count[slot ^ 1] = 0;
        for (int b = 0; b < P.n_boxes; ++b) P.scan_all[(slot ^ 1) * P.n_boxes + b] = 0;
    }
    if (c >= P.total_tiles / TILE_CELLS) return;
    // the next epoch's tile records start empty
    P.tncand[(int64_t)(slot ^ 1) * P.total_tiles + c * TILE_CELLS + lane] = 0;
    const int box = P.tchunk_box[c];
    const BoxDev &B = P.boxes[box];
    const int lt = c * TILE_CELLS + lane - B.tile_base;
    const bool st = lt < B.n_tiles && ((const IBLB_GLOBAL int32_t *)B.stamp[parity])[lt] == ctr;
    const uint64_t m = __ballot(st);
    if (m == 0) return;
    int base = 0;
    if (lane == 0) base = atomicAdd(P.tile_count + slot, __popcll(m));
    base = __shfl(base, 0, 64);
    const int k = base + __popcll(m & ((1ull << lane) - 1ull));
    if (st && k < P.total_tiles) {  // one entry per tile and epoch: k < total_tiles always
        P.tile_list[2 * k] = c * TILE_CELLS + lane;
        P.tile_list[2 * k + 1] = box;
    }
}

// ---------------------------------------------------- interpolate + advect
// One workgroup (4 wavefronts) per node block.  The velocity over the
// block's stencil box is staged in LDS when it fits; wavefront w sums the
// z-slab w of every node's 4x4x4 stencil (Eq. 7, u = 0 on wall cells), the
// four slab sums are added in slab order, and wavefront 0 advances q by
// forward Euler with a compensated (hi, lo) sum.  mode 1 writes U to Uout
// instead of moving the nodes.  Block 0 advances the step epoch.
template <typename R>
__global__ void __launch_bounds__(256) k_interp(DevPtrs P, int mode, double *Uout) {
    constexpr int MAXR = 36864 / (3 * (int)sizeof(R));
    __shared__ R su[3 * MAXR];
    __shared__ R red[3][3][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int blk = xcd_item(blockIdx.x, gridDim.x);
    const DropDev &D = P.drops[P.blk_drop[2 * blk]];
    const BoxDev &B = P.boxes[P.blk_drop[2 * blk + 1]];
    const int N = P.Ntot, nb = P.nblk;
    const bool zper = B.zbc == 1;
    const IBLB_GLOBAL R *ub = (const IBLB_GLOBAL R *)B.uband;
    const int bx0 = P.bbox[0 * nb + blk], bx1 = P.bbox[1 * nb + blk];
    const int by0 = P.bbox[2 * nb + blk], by1 = P.bbox[3 * nb + blk];
    int bz0 = P.bbox[4 * nb + blk], bz1 = P.bbox[5 * nb + blk];
    if (!zper) {
        bz0 = max(bz0, 0);
        bz1 = min(bz1, B.nz - 1);
    }
    const int ex = bx1 - bx0 + 1, ey = by1 - by0 + 1, ez = bz1 - bz0 + 1;
    const bool staged = ex > 0 && ey > 0 && ez > 0 && (int64_t)ex * ey * ez <= MAXR;
    // the node's own data load before the staging, so that they arrive
    // beside it (j < Ntot: nodes are padded to whole blocks)
    const int j = blk * NB + lane;
    const R *wg = (const R *)P.wgt;
    const int bx = P.base[j], by = P.base[N + j], bz = P.base[2 * N + j];
    const R wz = wg[(8 + wave) * N + j];
    R wx[4], wy[4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
        wx[o] = wg[o * N + j];
        wy[o] = wg[(4 + o) * N + j];
    }
    auto gidx = [&](int x, int y, int z) -> int64_t {
        return band_tile(x, y, z, B.tnx, B.tny) * 3 * TILE_CELLS + band_loc(x, y, z);
    };
    if (staged) {
        // the region's cells in order, four per thread and pass with all
        // their loads issued before the first LDS store
        const int x0w = wrapn(bx0, B.nx), y0w = wrapn(by0, B.ny), z0w = zper ? wrapn(bz0, B.nz) : bz0;
        const int ncell = ex * ey * ez;
        for (int c0 = 0; c0 < ncell; c0 += 4 * 256) {
            R v[4][3];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int c = c0 + k * 256 + tid;
                if (c < ncell) {
                    const int r = c / ex, ix = c - r * ex;
                    const int iz = r / ey, iy = r - iz * ey;
                    int x = x0w + ix, y = y0w + iy, z = z0w + iz;
                    while (x >= B.nx) x -= B.nx;
                    while (y >= B.ny) y -= B.ny;
                    if (zper)
                        while (z >= B.nz) z -= B.nz;
                    const int64_t g = gidx(x, y, z);
                    v[k][0] = ub[g];
                    v[k][1] = ub[g + TILE_CELLS];
                    v[k][2] = ub[g + 2 * TILE_CELLS];
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int c = c0 + k * 256 + tid;
                if (c < ncell) {
                    su[c] = v[k][0];
                    su[MAXR + c] = v[k][1];
                    su[2 * MAXR + c] = v[k][2];
                }
            }
        }
    }
    __syncthreads();
    const bool valid = j - D.node_off < D.n_nodes;
    R U0 = 0, U1 = 0, U2 = 0;
    if (valid) {
        const int z = bz - 1 + wave;
        if (zper || (z >= 0 && z < B.nz)) {
            if (staged) {
#pragma unroll
                for (int oy = 0; oy < 4; ++oy) {
                    const int c0 = ((z - bz0) * ey + (by - 1 + oy - by0)) * ex + (bx - 1 - bx0);
#pragma unroll
                    for (int ox = 0; ox < 4; ++ox) {
                        const R w = wx[ox] * wy[oy] * wz;
                        U0 += su[c0 + ox] * w;
                        U1 += su[MAXR + c0 + ox] * w;
                        U2 += su[2 * MAXR + c0 + ox] * w;
                    }
                }
            } else {
                const int zw = zper ? wrapn(z, B.nz) : z;
                for (int oy = 0; oy < 4; ++oy) {
                    const int y = wrapn(by - 1 + oy, B.ny);
                    for (int ox = 0; ox < 4; ++ox) {
                        const R w = wx[ox] * wy[oy] * wz;
                        const int64_t g = gidx(wrapn(bx - 1 + ox, B.nx), y, zw);
                        U0 += ub[g] * w;
                        U1 += ub[g + TILE_CELLS] * w;
                        U2 += ub[g + 2 * TILE_CELLS] * w;
                    }
                }
            }
        }
    }
    if (wave > 0) {
        red[wave - 1][0][lane] = U0;
        red[wave - 1][1][lane] = U1;
        red[wave - 1][2][lane] = U2;
    }
    __syncthreads();
    if (wave == 0 && valid) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            U0 += red[k][0][lane];
            U1 += red[k][1][lane];
            U2 += red[k][2][lane];
        }
        if (mode == 1) {
            Uout[3 * j + 0] = U0;
            Uout[3 * j + 1] = U1;
            Uout[3 * j + 2] = U2;
        } else {
            R *qh = (R *)P.qh, *ql = (R *)P.ql;
            const R U[3] = {U0, U1, U2};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const R h = qh[a * N + j], l = ql[a * N + j];
                // two-sum h + U, fold the error into the low part, renormalise
                const R s = h + U[a];
                const R bb = s - h;
                const R err = (h - (s - bb)) + (U[a] - bb);
                const R l2 = l + err;
                const R h2 = s + l2;
                qh[a * N + j] = h2;
                ql[a * N + j] = l2 - (h2 - s);
            }
            if (fabs(U0) > R(1) || fabs(U1) > R(1) || fabs(U2) > R(1)) atomicOr(P.status, BIT_JUMP);
        }
    }
    if (mode == 0 && blk == 0 && tid == 0) *P.ctr = *P.ctr + 1;
}

__global__ void k_epoch(DevPtrs P) {
    if (threadIdx.x == 0) *P.ctr = *P.ctr + 1;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------ observables
__device__ __forceinline__ double block_sum256(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}
__device__ __forceinline__ double block_minmax256(double v, double *sh, bool mx) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            sh[threadIdx.x] = mx ? fmax(sh[threadIdx.x], sh[threadIdx.x + s])
                                 : fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Per droplet (one workgroup): z range, FP64 area, volume and area-weighted
// centroid, then the edge crossings of z = z_min + xi, and the moments of
// the enclosed volume about the node mean m (for the deformation index):
// over the tetrahedron (m, a, b, c) of each triangle, with p the corners
// relative to m, s = p_a + p_b + p_c and v = p_a . (p_b x p_c) / 6,
//   int dV = v,  int x dV = v s / 4,  int x x^T dV = v (sum p p^T + s s^T) / 20.
template <typename R>
__global__ void __launch_bounds__(256) k_drop_obs(DevPtrs P) {
    __shared__ double sh[256];
    const DropDev &D = P.drops[blockIdx.x];
    const R *qh = (const R *)P.qh, *ql = (const R *)P.ql;
    const int N = P.Ntot;
    auto pos = [&](int j, int a) { return (double)qh[a * N + j] + (double)ql[a * N + j]; };
    double zmin = DBL_MAX, zmax = -DBL_MAX;
    for (int k = threadIdx.x; k < D.n_nodes; k += 256) {
        const double z = pos(D.node_off + k, 2);
        zmin = fmin(zmin, z);
        zmax = fmax(zmax, z);
    }
    zmin = block_minmax256(zmin, sh, false);
    zmax = block_minmax256(zmax, sh, true);
    double mean[3];
    for (int a = 0; a < 3; ++a) {
        double s = 0;
        for (int k = threadIdx.x; k < D.n_nodes; k += 256) s += pos(D.node_off + k, a);
        mean[a] = block_sum256(s, sh) / (double)max(D.n_nodes, 1);
    }
    double mom[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    double vol = 0, area = 0, c0 = 0, c1 = 0, c2 = 0;
    for (int t = D.tri_off + threadIdx.x; t < D.tri_off + D.n_tris; t += 256) {
        double p[3][3];
        for (int c = 0; c < 3; ++c)
            for (int a = 0; a < 3; ++a) p[c][a] = pos(P.tri[3 * t + c], a) - D.ref[a];
        const double bc0 = p[1][1] * p[2][2] - p[1][2] * p[2][1];
        const double bc1 = p[1][2] * p[2][0] - p[1][0] * p[2][2];
        const double bc2 = p[1][0] * p[2][1] - p[1][1] * p[2][0];
        vol += (p[0][0] * bc0 + p[0][1] * bc1 + p[0][2] * bc2) / 6.0;
        double e1[3], e2[3];
        for (int a = 0; a < 3; ++a) {
            e1[a] = p[1][a] - p[0][a];
            e2[a] = p[2][a] - p[0][a];
        }
        const double n0 = e1[1] * e2[2] - e1[2] * e2[1];
        const double n1 = e1[2] * e2[0] - e1[0] * e2[2];
        const double n2 = e1[0] * e2[1] - e1[1] * e2[0];
        const double At = 0.5 * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        area += At;
        c0 += At * (p[0][0] + p[1][0] + p[2][0]) / 3.0;
        c1 += At * (p[0][1] + p[1][1] + p[2][1]) / 3.0;
        c2 += At * (p[0][2] + p[1][2] + p[2][2]) / 3.0;
        double r[3][3];
        for (int c = 0; c < 3; ++c)
            for (int a = 0; a < 3; ++a) r[c][a] = pos(P.tri[3 * t + c], a) - mean[a];
        const double v = (r[0][0] * (r[1][1] * r[2][2] - r[1][2] * r[2][1]) +
                          r[0][1] * (r[1][2] * r[2][0] - r[1][0] * r[2][2]) +
                          r[0][2] * (r[1][0] * r[2][1] - r[1][1] * r[2][0])) / 6.0;
        const double s[3] = {r[0][0] + r[1][0] + r[2][0], r[0][1] + r[1][1] + r[2][1],
                             r[0][2] + r[1][2] + r[2][2]};
        mom[0] += v;
        for (int a = 0; a < 3; ++a) mom[1 + a] += v * s[a] / 4.0;
        constexpr int I[6] = {0, 1, 2, 0, 0, 1}, J[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int e = 0; e < 6; ++e)
            mom[4 + e] += v * (r[0][I[e]] * r[0][J[e]] + r[1][I[e]] * r[1][J[e]] + r[2][I[e]] * r[2][J[e]] +
                               s[I[e]] * s[J[e]]) / 20.0;
    }
    for (int e = 0; e < 10; ++e) mom[e] = block_sum256(mom[e], sh);
    vol = block_sum256(vol, sh);
    area = block_sum256(area, sh);
    c0 = block_sum256(c0, sh) / area + D.ref[0];
    c1 = block_sum256(c1, sh) / area + D.ref[1];
    c2 = block_sum256(c2, sh) / area + D.ref[2];
    const double zc = zmin + D.xi;
    double rs = 0, cnt = 0;
    for (int t = D.tri_off + threadIdx.x; t < D.tri_off + D.n_tris; t += 256) {
        for (int c = 0; c < 3; ++c) {
            const int a = P.tri[3 * t + c], b = P.tri[3 * t + (c + 1) % 3];
            if (a > b) continue;
            const double za = pos(a, 2), zb = pos(b, 2);
            if ((za < zc) == (zb < zc)) continue;
            const double s = (zc - za) / (zb - za);
            const double px = pos(a, 0) + s * (pos(b, 0) - pos(a, 0)) - c0;
            const double py = pos(a, 1) + s * (pos(b, 1) - pos(a, 1)) - c1;
            rs += sqrt(px * px + py * py);
            cnt += 1.0;
        }
    }
    rs = block_sum256(rs, sh);
    cnt = block_sum256(cnt, sh);
    if (threadIdx.x == 0) {
        double *o = P.obs_out + blockIdx.x * OBS_DROP;
        o[0] = vol;
        o[1] = area;
        o[2] = zmin;
        o[3] = zmax;
        o[4] = c0;
        o[5] = c1;
        o[6] = c2;
        o[7] = rs;
        o[8] = cnt;
        for (int e = 0; e < 10; ++e) o[9 + e] = mom[e];
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_tri(const DevPtrs &P, bool f64, hipStream_t s) {
    if (P.n_chunks == 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(k_tri<double>, dim3(P.n_chunks), dim3(256), 0, s, P);
    else hipLaunchKernelGGL(k_tri<float>, dim3(P.n_chunks), dim3(256), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_set_v0(const DevPtrs &P, bool, hipStream_t s) {
    if (P.n_drops == 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_v0, dim3(P.n_drops), dim3(64), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_node(const DevPtrs &P, bool f64, int mode, int parity, hipStream_t s) {
    if (P.nblk == 0) return hipSuccess;
    // few blocks: several waves per block share its spread; many blocks:
    // one wave per block, so that more blocks fit in a compute unit's LDS
    const bool many = P.nblk > P.n_cus;
    if (f64) {
        if (many) hipLaunchKernelGGL((k_node<double, 1>), dim3(P.nblk), dim3(64), 0, s, P, mode, parity);
        else hipLaunchKernelGGL((k_node<double, 2>), dim3(P.nblk), dim3(128), 0, s, P, mode, parity);
    } else {
        if (many) hipLaunchKernelGGL((k_node<float, 1>), dim3(P.nblk), dim3(64), 0, s, P, mode, parity);
        else hipLaunchKernelGGL((k_node<float, 4>), dim3(P.nblk), dim3(256), 0, s, P, mode, parity);
    }
    if (mode == 0 && P.total_tiles > 0) {
        const int chunks = P.total_tiles / TILE_CELLS;
        hipLaunchKernelGGL(k_compact, dim3((chunks + 3) / 4), dim3(256), 0, s, P, parity);
    }
    return hipGetLastError();
}

hipError_t launch_interp(const DevPtrs &P, bool f64, int mode, double *Uout, hipStream_t s) {
    if (P.nblk == 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(k_interp<double>, dim3(P.nblk), dim3(256), 0, s, P, mode, Uout);
    else hipLaunchKernelGGL(k_interp<float>, dim3(P.nblk), dim3(256), 0, s, P, mode, Uout);
    return hipGetLastError();
}


// ------------------------------------------------------------ inside bits
// Cells inside the droplets of boxes with tau_in (Sec. 2, below Eq. 13).  A
// cell is inside when the vertical ray below its centre crosses the closed
// meshes an odd number of times.  Every triangle toggles, in each column
// whose vertical line crosses it, the bits of the cells whose centre lies at
// or above the crossing; XOR does not depend on the order of the toggles,
// so the result is exact and the same in every run.
//   - Coordinates are rounded to the grid of 2^-18 lattice units (half away
//     from zero); the cell centre (i + 1/2) is i 2^18 + 2^17 on that grid.
//   - The line through column point p crosses the triangle when the signs
//     of the three edge functions e_uv(p) = (v_x - u_x)(p_y - u_y) -
//     (v_y - u_y)(p_x - u_x) agree; a zero takes the sign it would have with
//     p moved by (+e, +e^2): that of -(v_y - u_y), else of (v_x - u_x).
//   - With D = e_ab + e_bc + e_ca and N = e_bc a_z + e_ca b_z + e_ab c_z the
//     crossing lies at or below the centre z_c when sign(D) (z_c D - N) >= 0.
// Edge functions and their products are exact in 128-bit integers.
namespace {
constexpr int64_t QS = 1 << 18, QH = 1 << 17;

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {  // b > 0
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}
__device__ __forceinline__ int sos_sign(__int128 e, int64_t dx, int64_t dy) {
    if (e > 0) return 1;
    if (e < 0) return -1;
    if (dy != 0) return dy > 0 ? -1 : 1;
    if (dx != 0) return dx > 0 ? 1 : -1;
    return 0;
}
__device__ __forceinline__ __int128 edge_fn(int64_t ux, int64_t uy, int64_t vx, int64_t vy, int64_t px,
                                            int64_t py) {
    return (__int128)(vx - ux) * (py - uy) - (__int128)(vy - uy) * (px - ux);
}
}  // namespace

template <typename R>
__global__ void __launch_bounds__(256) k_inside(DevPtrs P, int slot) {
    const TriChunk ch = P.chunks[blockIdx.x];
    const DropDev &D = P.drops[ch.drop];
    const BoxDev &B = P.boxes[D.box];
    if (!B.contrast) return;
    const int t = ch.t0 + threadIdx.x;
    if (t >= ch.t1) return;
    const R *qh = (const R *)P.qh, *ql = (const R *)P.ql;
    const int N = P.Ntot, nx = B.nx, ny = B.ny, nz = B.nz, nzw = B.nzw;
    uint64_t *mask = B.mask[slot];
    int64_t X[3], Y[3], Z[3];
    bool sane = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int j = P.tri[3 * t + c];
        const double x = (double)qh[j] + (double)ql[j];
        const double y = (double)qh[N + j] + (double)ql[N + j];
        const double z = (double)qh[2 * N + j] + (double)ql[2 * N + j];
        // |coordinate| < 2^20 keeps every product below in 128 bits (NaN fails too)
        sane = sane && fabs(x) < 0x1p20 && fabs(y) < 0x1p20 && fabs(z) < 0x1p20;
        X[c] = sane ? llround(x * (double)QS) : 0;
        Y[c] = sane ? llround(y * (double)QS) : 0;
        Z[c] = sane ? llround(z * (double)QS) : 0;
    }
    // columns whose point lies in the triangle's xy bounding box
    const int64_t xmin = min(X[0], min(X[1], X[2])), xmax = max(X[0], max(X[1], X[2]));
    const int64_t ymin = min(Y[0], min(Y[1], Y[2])), ymax = max(Y[0], max(Y[1], Y[2]));
    const int64_t iu0 = -floor_div(-(xmin - QH), QS), iu1 = floor_div(xmax - QH, QS);
    const int64_t ju0 = -floor_div(-(ymin - QH), QS), ju1 = floor_div(ymax - QH, QS);
    // a triangle wider than the box (a blown-up mesh; the step reports the
    // instability) is left out rather than looped over
    if (!sane || iu1 - iu0 >= nx || ju1 - ju0 >= ny) return;
    for (int64_t ju = ju0; ju <= ju1; ++ju)
        for (int64_t iu = iu0; iu <= iu1; ++iu) {
            const int64_t px = iu * QS + QH, py = ju * QS + QH;
            const __int128 eab = edge_fn(X[0], Y[0], X[1], Y[1], px, py);
            const __int128 ebc = edge_fn(X[1], Y[1], X[2], Y[2], px, py);
            const __int128 eca = edge_fn(X[2], Y[2], X[0], Y[0], px, py);
            const int s1 = sos_sign(eab, X[1] - X[0], Y[1] - Y[0]);
            const int s2 = sos_sign(ebc, X[2] - X[1], Y[2] - Y[1]);
            const int s3 = sos_sign(eca, X[0] - X[2], Y[0] - Y[2]);
            if (s1 == 0 || s1 != s2 || s2 != s3) continue;
            const __int128 Dt = eab + ebc + eca;
            if (Dt == 0) continue;
            const __int128 Nt = ebc * Z[0] + eca * Z[1] + eab * Z[2];
            auto below = [&](int k) {  // crossing at or below the centre of cell k
                const __int128 d = ((__int128)k * QS + QH) * Dt - Nt;
                return Dt > 0 ? d >= 0 : d <= 0;
            };
            // first cell above the crossing: an estimate in FP64, then exact steps
            const double ea = (double)(X[1] - X[0]) * (double)(py - Y[0]) - (double)(Y[1] - Y[0]) * (double)(px - X[0]);
            const double eb = (double)(X[2] - X[1]) * (double)(py - Y[1]) - (double)(Y[2] - Y[1]) * (double)(px - X[1]);
            const double ec = (double)(X[0] - X[2]) * (double)(py - Y[2]) - (double)(Y[0] - Y[2]) * (double)(px - X[2]);
            const double zs = (eb * (double)Z[0] + ec * (double)Z[1] + ea * (double)Z[2]) / (ea + eb + ec);
            int k0 = (int)fmin(fmax(ceil(zs / (double)QS - 0.5), 0.0), (double)nz);
            while (k0 > 0 && below(k0 - 1)) --k0;
            while (k0 < nz && !below(k0)) ++k0;
            if (k0 >= nz) continue;
            const int i = (int)(iu % nx + (iu % nx < 0 ? nx : 0));
            const int j = (int)(ju % ny + (ju % ny < 0 ? ny : 0));
            for (int w = k0 >> 6; w < nzw; ++w) {
                const uint64_t bits = w == (k0 >> 6) ? (~0ull << (k0 & 63)) : ~0ull;
                atomicXor((unsigned long long *)&mask[((int64_t)w * ny + j) * nx + i], (unsigned long long)bits);
            }
        }
}

// Grid (chunks, boxes): every thread walks mask words of box blockIdx.y.
__global__ void __launch_bounds__(256) k_mask_clear(DevPtrs P, int slot) {
    const BoxDev &B = P.boxes[blockIdx.y];
    if (!B.contrast) return;
    const int64_t n = (int64_t)B.nzw * B.ny * B.nx;
    uint64_t *m = B.mask[slot];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m[i] = 0;
}

namespace {
dim3 mask_grid(const DevPtrs &P) {
    const int64_t g = ((int64_t)P.mask_words + 255) / 256;
    return dim3((unsigned)(g < 1024 ? (g > 0 ? g : 1) : 1024), (unsigned)P.n_boxes);
}
}  // namespace

hipError_t launch_mask_clear(const DevPtrs &P, int slot, hipStream_t s) {
    if (!P.contrast) return hipSuccess;
    hipLaunchKernelGGL(k_mask_clear, mask_grid(P), dim3(256), 0, s, P, slot);
    return hipGetLastError();
}

hipError_t launch_inside(const DevPtrs &P, bool f64, int slot, hipStream_t s) {
    if (P.n_chunks == 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(k_inside<double>, dim3(P.n_chunks), dim3(TRI_CHUNK), 0, s, P, slot);
    else hipLaunchKernelGGL(k_inside<float>, dim3(P.n_chunks), dim3(TRI_CHUNK), 0, s, P, slot);
    return hipGetLastError();
}

hipError_t launch_epoch(const DevPtrs &P, hipStream_t s) {
    hipLaunchKernelGGL(k_epoch, dim3(1), dim3(64), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t g = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_drop_obs(const DevPtrs &P, bool f64, hipStream_t s) {
    if (P.n_drops == 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(k_drop_obs<double>, dim3(P.n_drops), dim3(256), 0, s, P);
    else hipLaunchKernelGGL(k_drop_obs<float>, dim3(P.n_drops), dim3(256), 0, s, P);
    return hipGetLastError();
}

}  // namespace iblb
