// gfx950 kernels of the IBLB wetting step.
//
// Per step (paper Sec. 2): nodal forces at q^t (Eqs. 9-11) -> spreading to
// the lattice (Eq. 8) -> fused pull-stream / moments / BGK collision with
// the Guo source (Eqs. 1-6) -> interpolation of u^t at q^t (Eq. 7) and
// forward Euler advection.  No floating-point atomics anywhere: spreading is
// a per-tile gather in a fixed node order, and every FP64 sum is a fixed tree.
#include "iblb_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cfloat>
#include <climits>

namespace iblb {

// ---------------------------------------------------------------- storage
template <int ST> struct Stor;
template <> struct Stor<0> {  // FP64 deviations
    using T = double;
    using R = double;
    static __device__ __forceinline__ R ld(const T *p, float) { return *p; }
    static __device__ __forceinline__ void st(T *p, R v, float) { *p = v; }
};
template <> struct Stor<1> {  // FP32 deviations
    using T = float;
    using R = float;
    static __device__ __forceinline__ R ld(const T *p, float) { return *p; }
    static __device__ __forceinline__ void st(T *p, R v, float) { *p = v; }
};
template <> struct Stor<2> {  // binary16, scaled deviations
    using T = __half;
    using R = float;
    static __device__ __forceinline__ R ld(const T *p, float inv) { return __half2float(*p) * inv; }
    static __device__ __forceinline__ void st(T *p, R v, float s) { *p = __float2half_rn(v * s); }
};
template <> struct Stor<3> {  // bfloat16 deviations
    using T = __hip_bfloat16;
    using R = float;
    static __device__ __forceinline__ R ld(const T *p, float) { return __bfloat162float(*p); }
    static __device__ __forceinline__ void st(T *p, R v, float) { *p = __float2bfloat16(v); }
};

__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
__device__ __forceinline__ int wrapn(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

// ------------------------------------------------------- pulled populations
// Pre-collision deviations of cell (x,y,z) at the current time: the value
// stored at x - c_i, or, where x - c_i lies in a wall, the opposite
// population stored at x itself (halfway bounce-back).
template <int ST>
__device__ __forceinline__ void pull(const typename Stor<ST>::T *__restrict__ src, int64_t plane,
                                     int nx, int ny, int nz, int sx, bool zper, int x, int y, int z,
                                     float inv, typename Stor<ST>::R (&g)[Q]) {
    using S = Stor<ST>;
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    int zm = z - 1, zp = z + 1;
    if (zper) {
        zm = z == 0 ? nz - 1 : zm;
        zp = z == nz - 1 ? 0 : zp;
    }
    const bool wlo = !zper && z == 0, whi = !zper && z == nz - 1;
    const int64_t own = ((int64_t)z * ny + y) * sx + x;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
        const bool bb = (cz == 1 && wlo) || (cz == -1 && whi);
        if (bb) {
            g[i] = S::ld(src + opp_of(i) * plane + own, inv);
        } else {
            const int xs = cx == 1 ? xm : (cx == -1 ? xp : x);
            const int ys = cy == 1 ? ym : (cy == -1 ? yp : y);
            const int zs = cz == 1 ? zm : (cz == -1 ? zp : z);
            g[i] = S::ld(src + i * plane + (((int64_t)zs * ny + ys) * sx + xs), inv);
        }
    }
}

// ------------------------------------------------------- stream + collide
// One launch advances every cell of every box by one step.  A workgroup
// takes whole x-rows (a row group); threads stride along x, so the ±1
// shifted loads of a row stay inside one workgroup.
template <int ST>
__global__ void __launch_bounds__(1024)
    k_stream_collide(DevPtrs P, int parity, int full_u, float scale, float inv) {
    using S = Stor<ST>;
    using T = typename S::T;
    using R = typename S::R;
    const int tx = threadIdx.x, ty = threadIdx.y, BX = blockDim.x, BY = blockDim.y;
    const int ctr = *P.ctr;
    for (int gi = blockIdx.x; gi < P.n_rowgroups; gi += gridDim.x) {
        const RowGroup rg = P.rows[gi];
        const BoxDev *B = P.boxes + rg.box;
        const int nx = B->nx, ny = B->ny, nz = B->nz, sx = B->sx;
        const bool zper = B->zbc == 1;
        const int64_t plane = B->plane;
        const T *__restrict__ src = (const T *)B->f[parity];
        T *__restrict__ dst = (T *)B->f[parity ^ 1];
        const R omega = (R)B->omega, guo = (R)B->guo, rho0 = (R)B->rho0;
        const R gx = (R)B->g[0], gy = (R)B->g[1], gz = (R)B->g[2];
        const int32_t *__restrict__ stamp = B->stamp;
        const R *__restrict__ Fb = (const R *)B->Fband;
        R *__restrict__ ub = (R *)B->uband;
        const int tnx = B->tnx, tny = B->tny;
        for (int r = rg.r0 + ty; r < rg.r1; r += BY) {
            const int z = r / ny, y = r - z * ny;
            for (int x = tx; x < nx; x += BX) {
                R g[Q];
                pull<ST>(src, plane, nx, ny, nz, sx, zper, x, y, z, inv, g);
                const int64_t tile = ((int64_t)(z >> 2) * tny + (y >> 2)) * tnx + (x >> 2);
                const int loc = ((z & 3) << 4) | ((y & 3) << 2) | (x & 3);
                const bool stamped = stamp[tile] == ctr;
                R Fx = gx, Fy = gy, Fz = gz;
                if (stamped) {
                    const R *fp = Fb + tile * 3 * TILE_CELLS + loc;
                    Fx += fp[0];
                    Fy += fp[TILE_CELLS];
                    Fz += fp[2 * TILE_CELLS];
                }
                // moments (Eqs. 5-6) in deviation form: rho = rho0 + sum g
                R drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    drho += g[i];
                    jx += (R)cx_of(i) * g[i];
                    jy += (R)cy_of(i) * g[i];
                    jz += (R)cz_of(i) * g[i];
                }
                const R rho = rho0 + drho;
                const R irho = R(1) / rho;
                const R ux = (jx + R(0.5) * Fx) * irho;
                const R uy = (jy + R(0.5) * Fy) * irho;
                const R uz = (jz + R(0.5) * Fz) * irho;
                const R usq = ux * ux + uy * uy + uz * uz;
                const R uF = ux * Fx + uy * Fy + uz * Fz;
                const int64_t own = ((int64_t)z * ny + y) * sx + x;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const R w = (R)w_of(i);
                    const R cu = (R)cx_of(i) * ux + (R)cy_of(i) * uy + (R)cz_of(i) * uz;
                    const R cF = (R)cx_of(i) * Fx + (R)cy_of(i) * Fy + (R)cz_of(i) * Fz;
                    // f_eq - w rho0 (Eq. 3) and the Guo source (Eq. 4), cs^2 = 1/3
                    const R geq = w * (drho + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq));
                    const R src_i = guo * w * (R(3) * (cF - uF) + R(9) * cu * cF);
                    S::st(dst + i * plane + own, g[i] + omega * (geq - g[i]) + src_i, scale);
                }
                if (stamped || full_u) {
                    R *up = ub + tile * 3 * TILE_CELLS + loc;
                    up[0] = ux;
                    up[TILE_CELLS] = uy;
                    up[2 * TILE_CELLS] = uz;
                }
                if (!(rho > R(0) && rho < R(FLT_MAX))) atomicOr(P.status, BIT_RHO);
                if (usq > R(1) / R(3)) atomicOr(P.status, BIT_MACH);
            }
        }
    }
}

// ------------------------------------------------------------ wave helpers
template <typename V> __device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Fixed-order FP64 sum of a droplet's per-chunk partials; every lane of the
// wave returns the same value, identical in every wave that calls it.
__device__ __forceinline__ double droplet_partial_sum(const double *part, int off, int n, int lane) {
    double s = 0.0;
    for (int k = lane; k < n; k += 64) s += part[off + k];
    return wave_sum(s);
}

// Position helpers: a node coordinate is hi + lo (lo carries what the
// advection increments lose in hi; exact zero for FP64 in practice).
template <typename R> struct Node3 {
    R h[3], l[3];
};
template <typename R>
__device__ __forceinline__ Node3<R> load_node(const R *qh, const R *ql, int Ntot, int j) {
    Node3<R> n;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        n.h[a] = qh[a * Ntot + j];
        n.l[a] = ql[a * Ntot + j];
    }
    return n;
}
template <typename R> __device__ __forceinline__ void diff(const Node3<R> &b, const Node3<R> &a, R (&d)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = (b.h[k] - a.h[k]) + (b.l[k] - a.l[k]);
}
template <typename R> __device__ __forceinline__ void cross3(const R (&a)[3], const R (&b)[3], R (&c)[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// ------------------------------------------------- triangle FP64 partials
// Volume sum_t (a-r).((b-r)x(c-r))/6 and area, per chunk of 256 triangles,
// positions relative to the droplet's reference point r, in FP64.
template <typename R>
__global__ void __launch_bounds__(256) k_tri_sums(DevPtrs P) {
    __shared__ double sv[256], sa[256];
    const TriChunk ch = P.chunks[blockIdx.x];
    const DropDev &D = P.drops[ch.drop];
    const R *qh = (const R *)P.qh, *ql = (const R *)P.ql;
    const int t = ch.t0 + threadIdx.x;
    double v = 0.0, ar = 0.0;
    if (t < ch.t1) {
        double p[3][3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int j = P.tri[3 * t + c];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                p[c][a] = ((double)qh[a * P.Ntot + j] + (double)ql[a * P.Ntot + j]) - D.ref[a];
        }
        const double bc0 = p[1][1] * p[2][2] - p[1][2] * p[2][1];
        const double bc1 = p[1][2] * p[2][0] - p[1][0] * p[2][2];
        const double bc2 = p[1][0] * p[2][1] - p[1][1] * p[2][0];
        v = (p[0][0] * bc0 + p[0][1] * bc1 + p[0][2] * bc2) / 6.0;
        double e1[3], e2[3];
        for (int a = 0; a < 3; ++a) {
            e1[a] = p[1][a] - p[0][a];
            e2[a] = p[2][a] - p[0][a];
        }
        const double n0 = e1[1] * e2[2] - e1[2] * e2[1];
        const double n1 = e1[2] * e2[0] - e1[0] * e2[2];
        const double n2 = e1[0] * e2[1] - e1[1] * e2[0];
        ar = 0.5 * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    }
    sv[threadIdx.x] = v;
    sa[threadIdx.x] = ar;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sv[threadIdx.x] += sv[threadIdx.x + s];
            sa[threadIdx.x] += sa[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        P.tri_part[blockIdx.x] = sv[0];
        P.tri_part[P.n_chunks + blockIdx.x] = sa[0];
    }
}

// V0 of each droplet = the same fixed-order sum the volume penalty uses.
__global__ void __launch_bounds__(64) k_set_v0(DevPtrs P) {
    DropDev *D = P.drops + blockIdx.x;
    const double V = droplet_partial_sum(P.tri_part, D->chunk_off, D->n_chunks, threadIdx.x);
    if (threadIdx.x == 0) D->V0 = V;
}

// -------------------------------------------------------------- node pass
// One wavefront per block of 64 nodes.  Per node: gather over its incident
// triangles (CSR, ascending triangle id) the surface-tension corner forces
// -sigma dA_t/dq = (sigma/2)(q_prev - q_next) x n_t, the 1-ring area chi,
// the sum of unit face normals and the volume gradient; then the wetting
// force -chi Pi(d) n/3 with Pi from integer powers (Eq. 10) and the optional
// volume penalty.  Also: base cell floor(q - 1/2) (decided exactly from the
// hi/lo pair), the four Peskin weights per axis, the block's stencil
// bounding box, and (mode 0) the epoch stamps of every tile holding a
// stencil cell.
template <typename R>
__global__ void __launch_bounds__(256) k_node(DevPtrs P, int mode) {
    const int lane = threadIdx.x & 63;
    const int blk = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (blk >= P.nblk) return;
    const int d = P.blk_drop[blk];
    const DropDev &D = P.drops[d];
    const BoxDev &B = P.boxes[D.box];
    const int N = P.Ntot;
    const R *qh = (const R *)P.qh, *ql = (const R *)P.ql;
    const int j = blk * NB + lane;
    const bool valid = (j - D.node_off) < D.n_nodes;
    double dV = 0.0;
    if (D.kvol > 0.0) {
        const double V = droplet_partial_sum(P.tri_part, D.chunk_off, D.n_chunks, lane);
        dV = (V - D.V0) / D.V0;
    }
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
    if (valid) {
        const Node3<R> qj = load_node(qh, ql, N, j);
        R st[3] = {0, 0, 0}, ns[3] = {0, 0, 0}, gv[3] = {0, 0, 0};
        R chi = 0;
        const R hs = R(0.5) * (R)D.sigma;
        const int e0 = P.csr_off[j], e1 = P.csr_off[j + 1];
        for (int e = e0; e < e1; ++e) {
            const int code = P.csr_ent[e];
            const int t = code / 3, c = code - 3 * t;
            const int nxt = P.tri[3 * t + (c == 2 ? 0 : c + 1)];
            const int prv = P.tri[3 * t + (c == 0 ? 2 : c - 1)];
            const Node3<R> qn = load_node(qh, ql, N, nxt), qp = load_node(qh, ql, N, prv);
            R a[3], b[3], Nt[3], ed[3], f[3];
            diff(qn, qj, a);
            diff(qp, qj, b);
            cross3(a, b, Nt);
            const R len = sqrt(Nt[0] * Nt[0] + Nt[1] * Nt[1] + Nt[2] * Nt[2]);
            const R il = R(1) / len;
            R nt[3] = {Nt[0] * il, Nt[1] * il, Nt[2] * il};
            diff(qp, qn, ed);
            cross3(ed, nt, f);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                st[k] += hs * f[k];
                ns[k] += nt[k];
                gv[k] += Nt[k] / R(6);
            }
            chi += R(0.5) * len;
        }
        const R nl = R(1) / sqrt(ns[0] * ns[0] + ns[1] * ns[1] + ns[2] * ns[2]);
        const R dist = qj.h[2] + qj.l[2];
        if (!(dist > R(0))) atomicOr(P.status, BIT_WALL);
        const R rr = (R)D.xi / dist;
        R pn = 1, pm = 1;
        for (int k = 0; k < D.n_exp; ++k) pn *= rr;
        for (int k = 0; k < D.m_exp; ++k) pm *= rr;
        const R Pi = (R)D.A * (pn - pm);
        const R kw = chi * Pi / R(3) * nl;
        const R kv = (R)(-D.kvol * dV);
        R *phi = (R *)P.phi;
#pragma unroll
        for (int k = 0; k < 3; ++k) phi[k * N + j] = st[k] - kw * ns[k] + kv * gv[k];

        // base cell and Peskin 4-point weights per axis.  With t = q - b - 1/2
        // in [0,1] all four weights share s = sqrt(1 + 4t(1-t)):
        //   b-1: (3 - 2t - s)/8, b: (3 - 2t + s)/8, b+1: (1 + 2t + s)/8,
        //   b+2: (1 + 2t - s)/8.
        R *wg = (R *)P.wgt;
        const int dims[3] = {B.nx, B.ny, B.nz};
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
            const int b = (int)fl - (neg ? 1 : 0);
            const R t = neg ? rf + R(1) : rf;
            const R s = sqrt(R(1) + R(4) * t * (R(1) - t));
            wg[(4 * a + 0) * N + j] = (R(3) - R(2) * t - s) * R(0.125);
            wg[(4 * a + 1) * N + j] = (R(3) - R(2) * t + s) * R(0.125);
            wg[(4 * a + 2) * N + j] = (R(1) + R(2) * t + s) * R(0.125);
            wg[(4 * a + 3) * N + j] = (R(1) + R(2) * t - s) * R(0.125);
            P.base[a * N + j] = b;
            const bool per = a < 2 || B.zbc == 1;
            P.s0[a * N + j] = per ? wrapn(b - 1, dims[a]) : b - 1;
            lo[a] = b - 1;
            hi[a] = b + 2;
        }
        if (mode == 0) {
            // epoch stamp of every tile holding a stencil cell (same value
            // from every writer, so plain stores)
            int tl[3][4], tn[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                tn[a] = 0;
                const bool per = a < 2 || B.zbc == 1;
                for (int o = 0; o < 4; ++o) {
                    int c = lo[a] + o;
                    if (per) c = wrapn(c, dims[a]);
                    else if (c < 0 || c >= dims[a]) continue;
                    const int tt = c >> 2;
                    if (tn[a] == 0 || tl[a][tn[a] - 1] != tt) tl[a][tn[a]++] = tt;
                }
            }
            for (int iz = 0; iz < tn[2]; ++iz)
                for (int iy = 0; iy < tn[1]; ++iy)
                    for (int ix = 0; ix < tn[0]; ++ix)
                        B.stamp[((int64_t)tl[2][iz] * B.tny + tl[1][iy]) * B.tnx + tl[0][ix]] =
                            *P.ctr;
        }
    }
    // stencil bounding box of the block (unwrapped cell indices)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int l = wave_min(lo[a]), h = wave_max(hi[a]);
        if (lane == 0) {
            P.bbox[(2 * a) * P.nblk + blk] = l;
            P.bbox[(2 * a + 1) * P.nblk + blk] = h;
        }
    }
}

// Does the periodic interval [lo, hi] (unwrapped) meet cells [t0, t1] of an
// axis of n cells?  Non-periodic axes compare directly.
__device__ __forceinline__ bool meets(int lo, int hi, int t0, int t1, int n, bool per) {
    if (!per) return lo <= t1 && hi >= t0;
    if (hi - lo + 1 >= n) return true;
    const int l = wrapn(lo, n), h = l + (hi - lo);
    return (l <= t1 && h >= t0) || (l <= t1 + n && h >= t0 + n);
}

// ----------------------------------------------------------------- spread
// Eq. 8 as a gather: one wavefront per stamped tile, one lane per cell.
// Candidate node blocks (those whose stencil box meets the tile) are taken
// in ascending block order and, inside a block, nodes whose own stencil
// meets the tile in ascending node order, so every cell sums its
// contributions in one fixed order.  Writes all 64 cells of the tile.
template <typename R>
__global__ void __launch_bounds__(256) k_spread(DevPtrs P) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * 4;
    const int ctr = *P.ctr;
    const int N = P.Ntot;
    const R *phi = (const R *)P.phi, *wg = (const R *)P.wgt;
    const int nchunk = P.total_tiles / TILE_CELLS;
    for (int c = wave; c < nchunk; c += nwaves) {
        const BoxDev &B = P.boxes[P.tchunk_box[c]];
        const int lt_lane = c * TILE_CELLS + lane - B.tile_base;
        const bool st = lt_lane < B.n_tiles && B.stamp[lt_lane] == ctr;
        uint64_t tmask = __ballot(st);
        while (tmask) {
            const int l = __builtin_ctzll(tmask);
            tmask &= tmask - 1;
            const int lt = c * TILE_CELLS + l - B.tile_base;
            const int tx = lt % B.tnx, ty = (lt / B.tnx) % B.tny, tz = lt / (B.tnx * B.tny);
            const int x0 = tx * TILE, y0 = ty * TILE, z0 = tz * TILE;
            const int x1 = min(x0 + TILE - 1, B.nx - 1), y1 = min(y0 + TILE - 1, B.ny - 1),
                      z1 = min(z0 + TILE - 1, B.nz - 1);
            const int cxl = x0 + (lane & 3), cyl = y0 + ((lane >> 2) & 3), czl = z0 + (lane >> 4);
            const bool zper = B.zbc == 1;
            R acc0 = 0, acc1 = 0, acc2 = 0;
            for (int kb = B.blk_begin; kb < B.blk_end; kb += 64) {
                const int mb = kb + lane;
                bool hit = false;
                if (mb < B.blk_end) {
                    const int nb = P.nblk;
                    hit = meets(P.bbox[0 * nb + mb], P.bbox[1 * nb + mb], x0, x1, B.nx, true) &&
                          meets(P.bbox[2 * nb + mb], P.bbox[3 * nb + mb], y0, y1, B.ny, true) &&
                          meets(P.bbox[4 * nb + mb], P.bbox[5 * nb + mb], z0, z1, B.nz, zper);
                }
                uint64_t bmask = __ballot(hit);
                while (bmask) {
                    const int bl = __builtin_ctzll(bmask);
                    bmask &= bmask - 1;
                    const int blk = kb + bl;
                    const DropDev &D = P.drops[P.blk_drop[blk]];
                    const int j = blk * NB + lane;
                    bool nh = false;
                    if (j - D.node_off < D.n_nodes) {
                        const int bx = P.base[j], by = P.base[N + j], bz = P.base[2 * N + j];
                        nh = meets(bx - 1, bx + 2, x0, x1, B.nx, true) &&
                             meets(by - 1, by + 2, y0, y1, B.ny, true) &&
                             meets(bz - 1, bz + 2, z0, z1, B.nz, zper);
                    }
                    uint64_t nmask = __ballot(nh);
                    while (nmask) {
                        const int nl = __builtin_ctzll(nmask);
                        nmask &= nmask - 1;
                        const int n = blk * NB + nl;
                        int ox = cxl - P.s0[n], oy = cyl - P.s0[N + n], oz = czl - P.s0[2 * N + n];
                        if (ox < 0) ox += B.nx;
                        if (oy < 0) oy += B.ny;
                        if (zper && oz < 0) oz += B.nz;
                        R w = 0;
                        if (ox < 4 && oy < 4 && oz >= 0 && oz < 4)
                            w = wg[(0 + ox) * N + n] * wg[(4 + oy) * N + n] * wg[(8 + oz) * N + n];
                        acc0 += phi[n] * w;
                        acc1 += phi[N + n] * w;
                        acc2 += phi[2 * N + n] * w;
                    }
                }
            }
            R *Fb = (R *)B.Fband + (int64_t)lt * 3 * TILE_CELLS;
            Fb[lane] = acc0;
            Fb[TILE_CELLS + lane] = acc1;
            Fb[2 * TILE_CELLS + lane] = acc2;
        }
    }
}

// ---------------------------------------------------- interpolate + advect
// One wavefront per node block.  The velocity over the block's stencil box
// is staged in LDS when it fits, then each lane sums its node's 4x4x4
// stencil (Eq. 7, u = 0 on wall cells) and advances q by forward Euler with
// a compensated (hi, lo) sum.  mode 1 writes U to Uout instead of moving
// the nodes.  Block 0 advances the step epoch once the step is done.
template <typename R>
__global__ void __launch_bounds__(64) k_interp(DevPtrs P, int mode, double *Uout) {
    constexpr int MAXR = 49152 / (3 * (int)sizeof(R));
    __shared__ R su[3 * MAXR];
    const int lane = threadIdx.x;
    const int blk = blockIdx.x;
    const DropDev &D = P.drops[P.blk_drop[blk]];
    const BoxDev &B = P.boxes[D.box];
    const int N = P.Ntot, nb = P.nblk;
    const bool zper = B.zbc == 1;
    const R *ub = (const R *)B.uband;
    int bx0 = P.bbox[0 * nb + blk], bx1 = P.bbox[1 * nb + blk];
    int by0 = P.bbox[2 * nb + blk], by1 = P.bbox[3 * nb + blk];
    int bz0 = P.bbox[4 * nb + blk], bz1 = P.bbox[5 * nb + blk];
    if (!zper) {
        bz0 = max(bz0, 0);
        bz1 = min(bz1, B.nz - 1);
    }
    const int ex = bx1 - bx0 + 1, ey = by1 - by0 + 1, ez = bz1 - bz0 + 1;
    const bool staged = ex > 0 && ey > 0 && ez > 0 && (int64_t)ex * ey * ez <= MAXR;
    auto gidx = [&](int x, int y, int z) -> int64_t {
        x = wrapn(x, B.nx);
        y = wrapn(y, B.ny);
        if (zper) z = wrapn(z, B.nz);
        const int64_t tile = ((int64_t)(z >> 2) * B.tny + (y >> 2)) * B.tnx + (x >> 2);
        return tile * 3 * TILE_CELLS + (((z & 3) << 4) | ((y & 3) << 2) | (x & 3));
    };
    if (staged) {
        const int n = ex * ey * ez;
        for (int c = lane; c < n; c += 64) {
            const int ix = c % ex, iy = (c / ex) % ey, iz = c / (ex * ey);
            const int64_t g = gidx(bx0 + ix, by0 + iy, bz0 + iz);
            su[c] = ub[g];
            su[MAXR + c] = ub[g + TILE_CELLS];
            su[2 * MAXR + c] = ub[g + 2 * TILE_CELLS];
        }
    }
    __syncthreads();
    const int j = blk * NB + lane;
    if (j - D.node_off < D.n_nodes) {
        const R *wg = (const R *)P.wgt;
        const int bx = P.base[j], by = P.base[N + j], bz = P.base[2 * N + j];
        R U0 = 0, U1 = 0, U2 = 0;
        for (int oz = 0; oz < 4; ++oz) {
            const int z = bz - 1 + oz;
            if (!zper && (z < 0 || z >= B.nz)) continue;
            const R wz = wg[(8 + oz) * N + j];
            for (int oy = 0; oy < 4; ++oy) {
                const int y = by - 1 + oy;
                const R wy = wg[(4 + oy) * N + j];
                for (int ox = 0; ox < 4; ++ox) {
                    const int x = bx - 1 + ox;
                    const R w = wg[ox * N + j] * wy * wz;
                    R u0, u1, u2;
                    if (staged) {
                        const int c = ((z - bz0) * ey + (y - by0)) * ex + (x - bx0);
                        u0 = su[c];
                        u1 = su[MAXR + c];
                        u2 = su[2 * MAXR + c];
                    } else {
                        const int64_t g = gidx(x, y, z);
                        u0 = ub[g];
                        u1 = ub[g + TILE_CELLS];
                        u2 = ub[g + 2 * TILE_CELLS];
                    }
                    U0 += u0 * w;
                    U1 += u1 * w;
                    U2 += u2 * w;
                }
            }
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
    if (mode == 0 && blk == 0 && lane == 0) *P.ctr = *P.ctr + 1;
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
__device__ __forceinline__ double block_min256(double v, double *sh) {
    return -block_max256(-v, sh);
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
    const typename S::T *src = (const typename S::T *)B.f[parity];
    double m = 0.0, umax = 0.0;
    for (int r = r0; r < r1; ++r) {
        const int z = r / B.ny, y = r - z * B.ny;
        for (int x = threadIdx.x; x < B.nx; x += 256) {
            R g[Q];
            pull<ST>(src, B.plane, B.nx, B.ny, B.nz, B.sx, B.zbc == 1, x, y, z, inv, g);
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

// Per droplet (one workgroup): z range, FP64 area, volume and area-weighted
// centroid, then the edge crossings of z = z_min + xi.
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
    zmin = block_min256(zmin, sh);
    zmax = block_max256(zmax, sh);
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
    }
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
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_tri_sums(const DevPtrs &P, bool f64, hipStream_t s) {
    if (P.n_chunks == 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(k_tri_sums<double>, dim3(P.n_chunks), dim3(256), 0, s, P);
    else hipLaunchKernelGGL(k_tri_sums<float>, dim3(P.n_chunks), dim3(256), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_set_v0(const DevPtrs &P, bool, hipStream_t s) {
    if (P.n_drops == 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_v0, dim3(P.n_drops), dim3(64), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_node(const DevPtrs &P, bool f64, int mode, hipStream_t s) {
    if (P.nblk == 0) return hipSuccess;
    const dim3 grid((P.nblk + 3) / 4);
    if (f64) hipLaunchKernelGGL(k_node<double>, grid, dim3(256), 0, s, P, mode);
    else hipLaunchKernelGGL(k_node<float>, grid, dim3(256), 0, s, P, mode);
    return hipGetLastError();
}

hipError_t launch_spread(const DevPtrs &P, bool f64, hipStream_t s) {
    if (P.nblk == 0 || P.total_tiles == 0) return hipSuccess;
    const int chunks = P.total_tiles / TILE_CELLS;
    const int grid = min((chunks + 3) / 4, 2048);
    if (f64) hipLaunchKernelGGL(k_spread<double>, dim3(grid), dim3(256), 0, s, P);
    else hipLaunchKernelGGL(k_spread<float>, dim3(grid), dim3(256), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_stream_collide(const DevPtrs &P, int storage, int parity, int full_u,
                                 float scale, const Launch &L, hipStream_t s) {
    const dim3 block(L.bx, L.by), grid(L.grid);
    const float inv = 1.0f / scale;
    switch (storage) {
    case 0: hipLaunchKernelGGL(k_stream_collide<0>, grid, block, 0, s, P, parity, full_u, scale, inv); break;
    case 1: hipLaunchKernelGGL(k_stream_collide<1>, grid, block, 0, s, P, parity, full_u, scale, inv); break;
    case 2: hipLaunchKernelGGL(k_stream_collide<2>, grid, block, 0, s, P, parity, full_u, scale, inv); break;
    default: hipLaunchKernelGGL(k_stream_collide<3>, grid, block, 0, s, P, parity, full_u, scale, inv); break;
    }
    return hipGetLastError();
}

hipError_t launch_interp(const DevPtrs &P, bool f64, int mode, double *Uout, hipStream_t s) {
    if (P.nblk == 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(k_interp<double>, dim3(P.nblk), dim3(64), 0, s, P, mode, Uout);
    else hipLaunchKernelGGL(k_interp<float>, dim3(P.nblk), dim3(64), 0, s, P, mode, Uout);
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

hipError_t launch_drop_obs(const DevPtrs &P, bool f64, hipStream_t s) {
    if (P.n_drops == 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(k_drop_obs<double>, dim3(P.n_drops), dim3(256), 0, s, P);
    else hipLaunchKernelGGL(k_drop_obs<float>, dim3(P.n_drops), dim3(256), 0, s, P);
    return hipGetLastError();
}

}  // namespace iblb
