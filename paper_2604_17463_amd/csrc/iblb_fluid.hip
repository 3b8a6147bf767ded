// Fluid kernels of the IBLB wetting step (gfx950): the bulk fused
// pull-stream / moments / BGK-Guo collision with the body force only, over
// every cell outside this step's stamped band tiles; the band kernel, which
// gathers the spread interface force for each stamped tile and does the
// collision of its 64 cells with it; and the per-box observables.  The two
// step kernels write disjoint cells and run side by side.
#include "iblb_device.h"

namespace iblb {

// ------------------------------------------------------------------- bulk
// Every cell of every box with F = body force, except (SKIP) the cells of
// the band tiles this step's node pass stamped: the band kernel owns those
// (it adds the spread force) and runs beside this kernel, so each cell is
// pulled, collided and stored once per step.  A workgroup takes a row group
// (rows, or one segment of threads_x cells of rows longer than that; the
// segments of a row go to workgroups on one XCD, so the lines at their ends
// are fetched once); threads stride along x so the +-1 shifted loads of a
// row stay inside the workgroup or its XCD.  UROW: each wavefront lies in one row
// (threads_x a multiple of 64), so the row addressing is wave-uniform and
// lives in scalar registers.  NT: the populations are written with
// streaming stores (they are read again only in the next step; pays off
// once the two population buffers exceed the last-level cache).  EXT: some
// box has a viscosity contrast or a moving wall (the plain variant carries
// none of their registers).  Without SKIP the kernel is the plain
// stream-collide of every cell (boxes without droplets, timing).
template <int ST, bool UROW, bool NT, int CPT, bool EXT, bool SKIP, bool PADW>
__global__ void __launch_bounds__(K1_MAX_THREADS)
    k_bulk(DevPtrs P, int parity, int full_u, float scale, float inv) {
    using S = Stor<ST>;
    using R = typename S::R;
    constexpr uint32_t EB = sizeof(typename S::T);
    // 2-byte storage goes through buffer resources (scalar row offsets, one
    // per-lane offset per access); 4- and 8-byte storage measured faster with
    // plain global addressing
    constexpr bool BUF = UROW && EB == 2;
    const int tx = threadIdx.x, ty = threadIdx.y, BX = blockDim.x, BY = blockDim.y;
    const IBLB_CONST RowGroup *rows = (const IBLB_CONST RowGroup *)P.rows;
    // epoch of this step's stamps (written by the node pass, which this
    // kernel follows); -2 never matches a stamp
    const int epoch = SKIP ? ((const IBLB_GLOBAL int32_t *)P.step_epoch)[parity] : -2;
    for (int gi = blockIdx.x; gi < P.n_rowgroups; gi += gridDim.x) {
        const IBLB_CONST RowGroup &rg = rows[gi];
        const IBLB_CONST BoxDev *B = (const IBLB_CONST BoxDev *)P.boxes + rg.box;
        const int nx = B->nx, ny = B->ny, nz = B->nz, sx = B->sx;
        const bool zper = B->zbc == 1;
        const uint64_t pb = (uint64_t)B->plane * EB;
        const IBLB_GLOBAL char *__restrict__ src = (const IBLB_GLOBAL char *)B->f[parity];
        IBLB_GLOBAL char *__restrict__ dst = (IBLB_GLOBAL char *)B->f[parity ^ 1];
        const R omega = (R)B->omega, guo = (R)B->guo, rho0 = (R)B->rho0;
        const R omega_in = (R)B->omega_in, guo_in = (R)B->guo_in;
        const bool contrast = B->contrast != 0, moving = B->moving != 0;
        const IBLB_GLOBAL uint64_t *mask = (const IBLB_GLOBAL uint64_t *)B->mask[parity];
        const IBLB_GLOBAL int32_t *stamp = (const IBLB_GLOBAL int32_t *)B->stamp[parity];
        const int tnx = B->tnx, tny = B->tny;
        const bool skip_box = SKIP && B->blk_end > B->blk_begin;  // only boxes holding droplets
        R kw[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) kw[a] = (R)(6.0 * B->rho0 * (double)scale * B->uw[a]);
        const R gx = (R)B->g[0], gy = (R)B->g[1], gz = (R)B->g[2];
        IBLB_GLOBAL R *__restrict__ uf = (IBLB_GLOBAL R *)B->ufull;
        const uint64_t plane = (uint64_t)B->plane;
        const PopRes rs = pop_res((const void *)src, pb), rd = pop_res((const void *)dst, pb);
        // row r = z * ny + y, stepped by BY without a division per row; a
        // thread takes CPT rows (BY apart) at a time, with the loads of all
        // of them issued before the first collision
        int r = rg.r0 + ty;
        int z = r / ny, y = r - z * ny;
        for (; r < rg.r1; r += BY * CPT) {
            RowAddr ra[CPT];
            bool on[CPT];
            int ryk[CPT], rzk[CPT];
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                on[k] = r + k * BY < rg.r1;
                const int ry = UROW ? __builtin_amdgcn_readfirstlane(y) : y;
                const int rz = UROW ? __builtin_amdgcn_readfirstlane(z) : z;
                ryk[k] = ry;
                rzk[k] = rz;
                ra[k] = row_addr(ry, rz, ny, nz, sx, zper, EB);
                y += BY;
                while (y >= ny) {
                    y -= ny;
                    ++z;
                }
            }
            // PADW: some row group's x range reaches into its row's padding
            // (x1 > nx: the row table asks for it where the padding is a
            // small part of the row): the lanes x in [nx, sx) redo the row's
            // last cell and store zeros (the padding's value since init) in
            // the same store instructions as their neighbours, so that every
            // line of the row is written whole (a line written in part made
            // rows of 250 cells 10 % slower than rows of 256).  A separate
            // instantiation, so that workloads without it carry none of it.
            for (int x = rg.x0 + tx; x < rg.x1; x += BX) {
                R g[CPT][Q];
                const bool pad = PADW && x >= nx;
                const int xs = pad ? nx - 1 : x;  // the cell computed
                const XOff xo = x_off<EB>(xs, nx);
                const uint32_t xst = PADW ? (uint32_t)x * EB : xo.c;  // the cell stored
                bool mine[CPT];
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    mine[k] = on[k];
                    if (skip_box && on[k])
                        mine[k] = stamp[((int64_t)(rzk[k] >> TZS) * tny + (ryk[k] >> TYS)) * tnx + (xs >> TXS)] != epoch;
                }
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if (!mine[k]) continue;
                    if constexpr (BUF)
                        pull_buf<ST>(rs, (uint32_t)pb, ra[k], xo, g[k]);
                    else
                        pull_raw<ST>(src, pb, ra[k], xo, g[k]);
                }
#pragma unroll
                for (int k = 0; k < CPT; ++k) {
                    if (!mine[k]) continue;
                    R out[Q], u[3], rho;
                    const uint32_t own = ra[k].ro[1][1] + xst;
                    R om = omega, gu = guo;
                    if (EXT && moving && (ra[k].wlo || ra[k].whi)) wall_shift<R>(g[k], ra[k].wlo, ra[k].whi, kw);
                    if (EXT && contrast) {
                        // this step's inside bits (computed by the mesh
                        // chain, which this kernel follows)
                        const uint64_t w = mask[((int64_t)(rzk[k] >> 6) * ny + ryk[k]) * nx + xs];
                        if ((w >> (rzk[k] & 63)) & 1ull) {
                            om = omega_in;
                            gu = guo_in;
                        }
                    }
                    collide<ST>(g[k], gx, gy, gz, rho0, om, gu, scale, inv, out, u, rho);
                    if constexpr (PADW) {
#pragma unroll
                        for (int i = 0; i < Q; ++i) out[i] = pad ? R(0) : out[i];
                    }
                    if constexpr (BUF)
                        store_buf<ST, NT>(rd, (uint32_t)pb, ra[k].ro[1][1], xst, out);
                    else
                        store_ptr<ST, NT>(dst, pb, own, out);
                    if (PADW && pad) continue;
                    if (full_u) {
                        const uint64_t e = own / EB;
                        uf[e] = u[0];
                        uf[plane + e] = u[1];
                        uf[2 * plane + e] = u[2];
                    }
                    if (!(rho > R(0) && rho < R(FLT_MAX))) atomicOr(P.status, BIT_RHO);
                    if (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] > R(1) / R(3)) atomicOr(P.status, BIT_MACH);
                }
            }
        }
    }
}

// ------------------------------------------------------------ spread gather
// Spread force density (Eq. 8) at cell (cx,cy,cz) of band tile gt ([x0..x1]
// x [y0..y1] x [z0..z1]) of box `box`, for the calling lane.  The node
// blocks whose stencil box covers the tile contribute in ascending block
// order; a block's own contribution is the partial sum its node pass
// accumulated over its nodes (read from the block's partial region), or,
// for a block whose region did not fit, the nodes summed here one by one in
// ascending order.  No atomics: the sum order per cell is fixed.
//
// The candidate blocks are the ones the node pass recorded for the tile
// (sorted here); when the records are incomplete the bounding boxes of all
// blocks of the box are tested, GATHER_GROUP x 64 at a time, their hits
// going to a wave-private LDS list in ascending order.  Either way the
// region descriptors and partial values of GATHER_BATCH blocks load side by
// side.
constexpr int GATHER_GROUP = SCAN_GROUP / 64;
constexpr int GATHER_BATCH = 4;

template <typename R>
__device__ __forceinline__ void gather_F(const DevPtrs &P, const IBLB_CONST BoxDev *B, int box, int gt,
                                         int slot, int x0, int x1, int y0, int y1, int z0, int z1, int cx,
                                         int cy, int cz, int *hits, R &F0, R &F1, R &F2) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    const int nb = P.nblk, N = P.Ntot;
    const bool zper = B->zbc == 1;
    const int nx = B->nx, ny = B->ny, nz = B->nz;
    const int b0 = B->blk_begin, b1 = B->blk_end;
    const IBLB_GLOBAL R *part = (const IBLB_GLOBAL R *)P.part;
    const IBLB_CONST int32_t *breg = (const IBLB_CONST int32_t *)P.breg;

    // add the contributions of blocks id(0..n) (ascending) to F: the blocks
    // with a partial region in order, then those without one (their nodes
    // one by one), also in order
    auto add_blocks = [&](auto id, int n) {
        R v[GATHER_BATCH][3];
        bool ovf[GATHER_BATCH];
        bool any_ovf = false;
#pragma unroll
        for (int k = 0; k < GATHER_BATCH; ++k) {
            v[k][0] = v[k][1] = v[k][2] = R(0);
            ovf[k] = false;
            if (k < n) {
                const int blk = id(k);
                const IBLB_CONST int32_t *br = breg + (int64_t)blk * BREG;
                ovf[k] = br[6] != 0;
                any_ovf |= ovf[k];
                if (!ovf[k]) {
                    int dx = cx - br[0], dy = cy - br[1], dz = cz - br[2];
                    if (dx < 0) dx += nx;
                    if (dy < 0) dy += ny;
                    if (zper && dz < 0) dz += nz;
                    const int ex = br[3], ey = br[4], ez = br[5];
                    if (dx < ex && dy < ey && dz >= 0 && dz < ez) {
                        const int64_t c = (int64_t)blk * 3 * MAXP + 3 * ((dz * ey + dy) * ex + dx);
                        v[k][0] = part[c];
                        v[k][1] = part[c + 1];
                        v[k][2] = part[c + 2];
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < GATHER_BATCH; ++k) {
            if (k < n && !ovf[k]) {
                F0 += v[k][0];
                F1 += v[k][1];
                F2 += v[k][2];
            }
        }
        if (!any_ovf) return;
#pragma unroll 1
        for (int k = 0; k < n; ++k) {
            const int blk = id(k);
            if (breg[(int64_t)blk * BREG + 6] == 0) continue;
            const DropDev &D = P.drops[P.blk_drop[2 * blk]];
            const int j = blk * NB + lane;
            bool nh = false;
            if (j - D.node_off < D.n_nodes) {
                const int bx = P.base[j], by = P.base[N + j], bz = P.base[2 * N + j];
                nh = meets(bx - 1, bx + 2, x0, x1, nx, true) && meets(by - 1, by + 2, y0, y1, ny, true) &&
                     meets(bz - 1, bz + 2, z0, z1, nz, zper);
            }
            uint64_t nmask = __ballot(nh);
            if (!nmask) continue;
            const R *wgt = (const R *)P.wgt, *phi = (const R *)P.phi;
            int s0x = 0, s0y = 0, s0z = 0;
            R w[12], f[3];
#pragma unroll
            for (int q = 0; q < 12; ++q) w[q] = 0;
            f[0] = f[1] = f[2] = 0;
            if (nh) {
                s0x = P.s0[j];
                s0y = P.s0[N + j];
                s0z = P.s0[2 * N + j];
#pragma unroll
                for (int q = 0; q < 12; ++q) w[q] = wgt[q * N + j];
#pragma unroll
                for (int q = 0; q < 3; ++q) f[q] = phi[q * N + j];
            }
            while (nmask) {
                const int nl = __builtin_ctzll(nmask);
                nmask &= nmask - 1;
                int ox = cx - bcast_i(s0x, nl), oy = cy - bcast_i(s0y, nl), oz = cz - bcast_i(s0z, nl);
                if (ox < 0) ox += nx;
                if (oy < 0) oy += ny;
                if (zper && oz < 0) oz += nz;
                const R ax = pick4(ox, bcast(w[0], nl), bcast(w[1], nl), bcast(w[2], nl), bcast(w[3], nl));
                const R ay = pick4(oy, bcast(w[4], nl), bcast(w[5], nl), bcast(w[6], nl), bcast(w[7], nl));
                const R az = pick4(oz, bcast(w[8], nl), bcast(w[9], nl), bcast(w[10], nl), bcast(w[11], nl));
                const R wv = ax * ay * az;
                F0 += bcast(f[0], nl) * wv;
                F1 += bcast(f[1], nl) * wv;
                F2 += bcast(f[2], nl) * wv;
            }
        }
    };

    // the recorded candidates: count, flag and the MAXC slots (lane k holds
    // slot k) in one round trip
    const int ncand = ((const IBLB_CONST int32_t *)P.tncand)[(int64_t)slot * P.total_tiles + gt];
    const bool scan = !box_records(b0, b1) ||
                      ((const IBLB_CONST int32_t *)P.scan_all)[slot * P.n_boxes + box] != 0;
    int mine = lane < MAXC ? P.tcand[(int64_t)gt * MAXC + lane] : INT_MAX;
    if (!scan && ncand <= MAXC) {
        mine = lane < ncand ? mine : INT_MAX;
        // rank of each lane's block among the candidates (the ids are distinct)
        int rank = 0;
        for (int k = 0; k < ncand; ++k) rank += __builtin_amdgcn_readlane(mine, k) < mine ? 1 : 0;
        for (int r0 = 0; r0 < ncand; r0 += GATHER_BATCH) {
            auto id = [&](int k) {
                const uint64_t m = __ballot(lane < ncand && rank == r0 + k);
                return m ? __builtin_amdgcn_readlane(mine, __builtin_ctzll(m)) : 0;
            };
            add_blocks(id, min(GATHER_BATCH, ncand - r0));
        }
        return;
    }
    for (int kb = b0; kb < b1; kb += 64 * GATHER_GROUP) {
        bool hit[GATHER_GROUP];
#pragma unroll
        for (int g = 0; g < GATHER_GROUP; ++g) {
            const int mb = kb + 64 * g + lane;
            hit[g] = mb < b1 &&
                     meets(P.bbox[0 * nb + mb], P.bbox[1 * nb + mb], x0, x1, nx, true) &&
                     meets(P.bbox[2 * nb + mb], P.bbox[3 * nb + mb], y0, y1, ny, true) &&
                     meets(P.bbox[4 * nb + mb], P.bbox[5 * nb + mb], z0, z1, nz, zper);
        }
        int total = 0;
#pragma unroll
        for (int g = 0; g < GATHER_GROUP; ++g) {
            const uint64_t m = __ballot(hit[g]);
            if (hit[g]) hits[total + __popcll(m & below)] = kb + 64 * g + lane;
            total += __popcll(m);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int k0 = 0; k0 < total; k0 += GATHER_BATCH) {
            auto id = [&](int k) { return __builtin_amdgcn_readfirstlane(hits[k0 + k]); };
            add_blocks(id, min(GATHER_BATCH, total - k0));
        }
        __builtin_amdgcn_wave_barrier();  // the list is rewritten by the next group
    }
}

// ------------------------------------------------------------------- band
// Largest band grid (workgroups of four waves, one wave per listed tile);
// a multiple of eight.
constexpr int BAND_GRID = 8192;
// One wavefront per stamped tile of this epoch, one lane per cell: gather
// the spread force, then (COLLIDE) pull, collide with F = body force +
// spread force, store the populations (the bulk kernel leaves these cells
// alone) and write u to the band; or (!COLLIDE, inspection) store F in the
// band.
// ONE_BOX: a single box, whose descriptor is read beside the list entry
// rather than after it.  xcd: the grid (BAND_GRID workgroups) takes the
// list in one contiguous eighth per XCD instead of interleaved.
template <int ST, bool COLLIDE, bool ONE_BOX>
__global__ void __launch_bounds__(256)
    k_band(DevPtrs P, int parity, int full_u, float scale, float inv, int xcd, int nt) {
    using S = Stor<ST>;
    using R = typename S::R;
    constexpr uint32_t EB = sizeof(typename S::T);
    __shared__ int hits[4][64 * GATHER_GROUP];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int nwaves = gridDim.x * 4;
    const IBLB_CONST int32_t *tl = (const IBLB_CONST int32_t *)P.tile_list;
    // the epoch counter, both list lengths and the wave's first list entry
    // in one round trip (the entry lies in the list whatever the count; the
    // count decides whether it is used)
    const int ctr = *P.ctr, n0 = P.tile_count[0], n1 = P.tile_count[1];
    const int first = min(wave, P.total_tiles - 1);
    const int first_gt = tl[2 * first], first_box = ONE_BOX ? 0 : tl[2 * first + 1];
    // the descriptor fields the tile's addressing needs (box 0's when there
    // is one box: then they load beside the entry)
    struct Geo {
        int tile_base, tnx, tny, nx, ny, nz, sx, zbc;
        uint64_t plane;
        const void *src;
    };
    auto geo = [&](const IBLB_CONST BoxDev *B) {
        return Geo{B->tile_base, B->tnx, B->tny, B->nx, B->ny, B->nz, B->sx, B->zbc, (uint64_t)B->plane,
                   B->f[parity]};
    };
    Geo g0{};
    if constexpr (ONE_BOX) g0 = geo((const IBLB_CONST BoxDev *)P.boxes);
    // keep these loads beside the counter's (not after the count test)
    asm volatile("" ::"s"(ctr), "s"(n0), "s"(n1), "s"(first_gt), "s"(first_box), "s"(g0.tile_base),
                 "s"(g0.tnx), "s"(g0.tny), "s"(g0.nx), "s"(g0.ny), "s"(g0.nz), "s"(g0.sx), "s"(g0.zbc),
                 "s"(g0.plane), "s"(g0.src));
    const int count = min((ctr & 1) ? n1 : n0, P.total_tiles);
    // list positions of this wave: every nwaves-th from its index, or (xcd,
    // a grid of whole groups of eight workgroups) a contiguous eighth of the
    // list per XCD, so that neighbouring tiles, which read the same partial
    // regions and share population lines, are taken on one L2 at about the
    // same time
    int i0 = wave, i1 = count, di = nwaves;
    if (xcd) {
        const ListRange lr = xcd_list_range(blockIdx.x, threadIdx.x >> 6, gridDim.x, count);
        i0 = __builtin_amdgcn_readfirstlane(lr.first);
        i1 = lr.end;
        di = lr.stride;
    }
    for (int i = i0; i < i1; i += di) {
        // global tile id and its box
        const int gt = (!xcd && i == wave) ? first_gt : tl[2 * i];
        const int box = ONE_BOX ? 0 : ((!xcd && i == wave) ? first_box : tl[2 * i + 1]);
        const IBLB_CONST BoxDev *B = (const IBLB_CONST BoxDev *)P.boxes + box;
        const Geo G = ONE_BOX ? g0 : geo(B);
        const int lt = gt - G.tile_base;
        const int tx = lt % G.tnx, ty = (lt / G.tnx) % G.tny, tz = lt / (G.tnx * G.tny);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
        const int x1 = min(x0 + TX - 1, G.nx - 1), y1 = min(y0 + TY - 1, G.ny - 1),
                  z1 = min(z0 + TZ - 1, G.nz - 1);
        const int cx = x0 + (lane & (TX - 1)), cy = y0 + ((lane >> TXS) & (TY - 1)),
                  cz = z0 + (lane >> (TXS + TYS));
        const bool inside = cx < G.nx && cy < G.ny && cz < G.nz;
        // the populations are pulled first so that their loads are in flight
        // during the force gather
        const uint64_t pb = G.plane * EB;
        const PopRes rs = pop_res(G.src, pb);
        RowAddr ra{};
        XOff xo{};
        R g[Q];
        if (COLLIDE && inside) {
            ra = row_addr(cy, cz, G.ny, G.nz, G.sx, G.zbc == 1, EB);
            xo = x_off<EB>(cx, G.nx);
            pull_buf<ST, true>(rs, (uint32_t)pb, ra, xo, g);
        }
        R F0 = 0, F1 = 0, F2 = 0;
        gather_F<R>(P, B, box, gt, ctr & 1, x0, x1, y0, y1, z0, z1, cx, cy, cz, hits[threadIdx.x >> 6], F0,
                    F1, F2);
        if (!COLLIDE) {
            IBLB_GLOBAL R *Fb = (IBLB_GLOBAL R *)B->Fband + (int64_t)lt * 3 * TILE_CELLS;
            Fb[lane] = F0;
            Fb[TILE_CELLS + lane] = F1;
            Fb[2 * TILE_CELLS + lane] = F2;
            continue;
        }
        if (!inside) continue;
        R out[Q], u[3], rho;
        const uint32_t own = ra.ro[1][1] + xo.c;
        if (B->moving && (ra.wlo || ra.whi)) {
            R kw[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) kw[a] = (R)(6.0 * B->rho0 * (double)scale * B->uw[a]);
            wall_shift<R>(g, ra.wlo, ra.whi, kw);
        }
        R om = (R)B->omega, gu = (R)B->guo;
        if (B->contrast) {  // this step's inside bits
            const uint64_t w = ((const IBLB_GLOBAL uint64_t *)B->mask[parity])[((int64_t)(cz >> 6) * B->ny + cy) * B->nx + cx];
            if ((w >> (cz & 63)) & 1ull) {
                om = (R)B->omega_in;
                gu = (R)B->guo_in;
            }
        }
        collide<ST>(g, (R)B->g[0] + F0, (R)B->g[1] + F1, (R)B->g[2] + F2, (R)B->rho0, om, gu, scale, inv,
                    out, u, rho);
        // streaming stores where the bulk kernel uses them (the populations
        // exceed the last-level cache)
        if (nt)
            store_buf<ST, true, true>(pop_res(B->f[parity ^ 1], pb), (uint32_t)pb, ra.ro[1][1], xo.c, out);
        else
            store_buf<ST, false, true>(pop_res(B->f[parity ^ 1], pb), (uint32_t)pb, ra.ro[1][1], xo.c, out);
        IBLB_GLOBAL R *ub = (IBLB_GLOBAL R *)B->uband + (int64_t)lt * 3 * TILE_CELLS;
        ub[lane] = u[0];
        ub[TILE_CELLS + lane] = u[1];
        ub[2 * TILE_CELLS + lane] = u[2];
        if (full_u) {
            IBLB_GLOBAL R *uf = (IBLB_GLOBAL R *)B->ufull;
            const uint64_t e = own / EB, plane = (uint64_t)B->plane;
            uf[e] = u[0];
            uf[plane + e] = u[1];
            uf[2 * plane + e] = u[2];
        }
        if (!(rho > R(0) && rho < R(FLT_MAX))) atomicOr(P.status, BIT_RHO);
        if (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] > R(1) / R(3)) atomicOr(P.status, BIT_MACH);
    }
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
__device__ __forceinline__ double block_max256(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// Mass and largest bare velocity of one box's current populations: fixed
// partition of the rows over OBS_GROUPS workgroups, then a fixed-order
// final sum.
template <int ST>
__global__ void __launch_bounds__(256) k_box_obs(DevPtrs P, int box, int parity, float inv) {
    using S = Stor<ST>;
    using R = typename S::R;
    __shared__ double sh[256];
    const BoxDev &B = P.boxes[box];
    const int rows = B.ny * B.nz;
    const int r0 = (int)((int64_t)rows * blockIdx.x / gridDim.x);
    const int r1 = (int)((int64_t)rows * (blockIdx.x + 1) / gridDim.x);
    const IBLB_GLOBAL char *src = (const IBLB_GLOBAL char *)B.f[parity];
    const uint64_t pb = (uint64_t)B.plane * sizeof(typename S::T);
    double m = 0.0, umax = 0.0;
    for (int r = r0; r < r1; ++r) {
        const int z = r / B.ny, y = r - z * B.ny;
        const RowAddr ra = row_addr(y, z, B.ny, B.nz, B.sx, B.zbc == 1, sizeof(typename S::T));
        for (int x = threadIdx.x; x < B.nx; x += 256) {
            R g[Q];
            pull<ST>(src, pb, ra, x, B.nx, inv, g);
            if (B.moving && (ra.wlo || ra.whi)) {  // g holds unscaled deviations
                R kw[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) kw[a] = (R)(6.0 * B.rho0 * B.uw[a]);
                wall_shift<R>(g, ra.wlo, ra.whi, kw);
            }
            double dr = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                dr += (double)g[i];
                jx += cx_of(i) * (double)g[i];
                jy += cy_of(i) * (double)g[i];
                jz += cz_of(i) * (double)g[i];
            }
            m += dr;
            umax = fmax(umax, sqrt(jx * jx + jy * jy + jz * jz) / (B.rho0 + dr));
        }
    }
    m = block_sum256(m, sh);
    umax = block_max256(umax, sh);
    if (threadIdx.x == 0) {
        P.obs_part[2 * blockIdx.x] = m;
        P.obs_part[2 * blockIdx.x + 1] = umax;
    }
}

__global__ void __launch_bounds__(256) k_box_obs_final(DevPtrs P, int box, int groups) {
    __shared__ double sh[256];
    double m = 0.0, umax = 0.0;
    for (int k = threadIdx.x; k < groups; k += 256) {
        m += P.obs_part[2 * k];
        umax = fmax(umax, P.obs_part[2 * k + 1]);
    }
    m = block_sum256(m, sh);
    umax = block_max256(umax, sh);
    if (threadIdx.x == 0) {
        double *o = P.obs_out + P.n_drops * OBS_DROP + box * OBS_BOX;
        o[0] = P.boxes[box].cells_rho0 + m;
        o[1] = umax;
    }
}

// ---------------------------------------------------------------- launchers
template <int ST, bool UROW, bool NT, bool SKIP, bool PADW>
static void launch_bulk_p(const DevPtrs &P, int parity, int full_u, float scale, float inv, const Launch &L,
                          dim3 grid, dim3 block, hipStream_t s) {
    if (P.contrast || P.moving) {
        if (UROW && L.cpt == 2)
            hipLaunchKernelGGL((k_bulk<ST, UROW, NT, 2, true, SKIP, PADW>), grid, block, 0, s, P, parity, full_u,
                               scale, inv);
        else
            hipLaunchKernelGGL((k_bulk<ST, UROW, NT, 1, true, SKIP, PADW>), grid, block, 0, s, P, parity, full_u,
                               scale, inv);
    } else if (UROW && L.cpt == 2) {
        hipLaunchKernelGGL((k_bulk<ST, UROW, NT, 2, false, SKIP, PADW>), grid, block, 0, s, P, parity, full_u, scale,
                           inv);
    } else {
        hipLaunchKernelGGL((k_bulk<ST, UROW, NT, 1, false, SKIP, PADW>), grid, block, 0, s, P, parity, full_u, scale,
                           inv);
    }
}

template <int ST, bool UROW, bool NT, bool SKIP>
static void launch_bulk_c(const DevPtrs &P, int parity, int full_u, float scale, float inv, const Launch &L,
                          dim3 grid, dim3 block, hipStream_t s) {
    if (P.pad_rows)
        launch_bulk_p<ST, UROW, NT, SKIP, true>(P, parity, full_u, scale, inv, L, grid, block, s);
    else
        launch_bulk_p<ST, UROW, NT, SKIP, false>(P, parity, full_u, scale, inv, L, grid, block, s);
}

template <int ST, bool SKIP>
static hipError_t launch_bulk_t(const DevPtrs &P, int parity, int full_u, float scale, const Launch &L,
                                hipStream_t s) {
    // never launch a shape the kernel was not compiled for
    if (L.bx < 1 || L.by < 1 || L.bx * L.by > K1_MAX_THREADS || L.grid < 1 || L.cpt < 1 || L.cpt > 2)
        return hipErrorInvalidValue;
    const dim3 block(L.bx, L.by), grid(L.grid);
    const float inv = 1.0f / scale;
    if (L.bx % 64 == 0) {
        if (L.nt)
            launch_bulk_c<ST, true, true, SKIP>(P, parity, full_u, scale, inv, L, grid, block, s);
        else
            launch_bulk_c<ST, true, false, SKIP>(P, parity, full_u, scale, inv, L, grid, block, s);
    } else {
        if (L.nt)
            launch_bulk_c<ST, false, true, SKIP>(P, parity, full_u, scale, inv, L, grid, block, s);
        else
            launch_bulk_c<ST, false, false, SKIP>(P, parity, full_u, scale, inv, L, grid, block, s);
    }
    return hipGetLastError();
}

template <int ST>
static hipError_t launch_bulk_s(const DevPtrs &P, int parity, int full_u, float scale, const Launch &L,
                                bool skip_band, hipStream_t s) {
    return skip_band ? launch_bulk_t<ST, true>(P, parity, full_u, scale, L, s)
                     : launch_bulk_t<ST, false>(P, parity, full_u, scale, L, s);
}

hipError_t launch_bulk(const DevPtrs &P, int storage, int parity, int full_u, float scale,
                       const Launch &L, bool skip_band, hipStream_t s) {
    switch (storage) {
    case 0: return launch_bulk_s<0>(P, parity, full_u, scale, L, skip_band, s);
    case 1: return launch_bulk_s<1>(P, parity, full_u, scale, L, skip_band, s);
    case 2: return launch_bulk_s<2>(P, parity, full_u, scale, L, skip_band, s);
    default: return launch_bulk_s<3>(P, parity, full_u, scale, L, skip_band, s);
    }
}

template <int ST, bool C>
static void launch_band_t(const DevPtrs &P, int parity, int full_u, float scale, int nt, hipStream_t s) {
    // one wave per tile up to 32,768 waves (workgroups of four); large
    // bands (many boxes or droplets) loop over the rest of the list
    const int grid = min((P.total_tiles + 3) / 4, BAND_GRID);
    // a full grid (a multiple of eight workgroups) takes the list in XCD
    // ranges; a small one keeps the interleaved order, whose first entry
    // loads beside the list count (latency decides there)
    const int xcd = grid == BAND_GRID ? 1 : 0;
    if (P.n_boxes == 1)
        hipLaunchKernelGGL((k_band<ST, C, true>), dim3(grid), dim3(256), 0, s, P, parity, full_u, scale,
                           1.0f / scale, xcd, nt);
    else
        hipLaunchKernelGGL((k_band<ST, C, false>), dim3(grid), dim3(256), 0, s, P, parity, full_u, scale,
                           1.0f / scale, xcd, nt);
}

hipError_t launch_band(const DevPtrs &P, int storage, int parity, int full_u, float scale, bool collide,
                       int nt, hipStream_t s) {
    if (P.nblk == 0 || P.total_tiles == 0) return hipSuccess;
    if (collide) {
        switch (storage) {
        case 0: launch_band_t<0, true>(P, parity, full_u, scale, nt, s); break;
        case 1: launch_band_t<1, true>(P, parity, full_u, scale, nt, s); break;
        case 2: launch_band_t<2, true>(P, parity, full_u, scale, nt, s); break;
        default: launch_band_t<3, true>(P, parity, full_u, scale, nt, s); break;
        }
    } else if (storage == 0) {
        launch_band_t<0, false>(P, parity, full_u, scale, 0, s);
    } else {
        launch_band_t<1, false>(P, parity, full_u, scale, 0, s);
    }
    return hipGetLastError();
}

hipError_t launch_box_obs(const DevPtrs &P, int storage, int parity, float inv, hipStream_t s) {
    for (int b = 0; b < P.n_boxes; ++b) {
        const dim3 grid(OBS_GROUPS), block(256);
        switch (storage) {
        case 0: hipLaunchKernelGGL(k_box_obs<0>, grid, block, 0, s, P, b, parity, inv); break;
        case 1: hipLaunchKernelGGL(k_box_obs<1>, grid, block, 0, s, P, b, parity, inv); break;
        case 2: hipLaunchKernelGGL(k_box_obs<2>, grid, block, 0, s, P, b, parity, inv); break;
        default: hipLaunchKernelGGL(k_box_obs<3>, grid, block, 0, s, P, b, parity, inv); break;
        }
        hipLaunchKernelGGL(k_box_obs_final, dim3(1), dim3(256), 0, s, P, b, OBS_GROUPS);
    }
    return hipGetLastError();
}

}  // namespace iblb
