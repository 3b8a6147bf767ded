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

// Address spaces: tables that stay constant during a launch are read through
// the constant space (scalar loads); population and band pointers taken from
// those tables are global memory.
#define IBLB_CONST __attribute__((address_space(4)))
#define IBLB_GLOBAL __attribute__((address_space(1)))

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
// Addressing of one x-row for the pull: byte offsets (32-bit, a plane is
// < 4 GiB) of the 9 source rows (y - c_y, z - c_z) and the wall flags.  The
// loads then take a uniform 64-bit plane base plus a 32-bit per-lane offset.
struct RowAddr {
    uint32_t ro[3][3];  // [c_y + 1][c_z + 1] -> byte offset of row (y - c_y, z - c_z)
    bool wlo, whi;      // z = 0 / z = nz-1 next to a wall
};

__device__ __forceinline__ RowAddr row_addr(int y, int z, int ny, int nz, int sx, bool zper,
                                            uint32_t eb) {
    RowAddr a;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    int zm = z - 1, zp = z + 1;
    if (zper) {
        zm = z == 0 ? nz - 1 : zm;
        zp = z == nz - 1 ? 0 : zp;
    } else {
        zm = max(zm, 0);       // wall rows are never read through these
        zp = min(zp, nz - 1);
    }
    const int ys[3] = {yp, y, ym};  // c_y = -1, 0, +1  ->  source y - c_y
    const int zs[3] = {zp, z, zm};
    const uint32_t rs = (uint32_t)sx * eb;
#pragma unroll
    for (int a1 = 0; a1 < 3; ++a1)
#pragma unroll
        for (int b1 = 0; b1 < 3; ++b1) a.ro[a1][b1] = (uint32_t)(zs[b1] * ny + ys[a1]) * rs;
    a.wlo = !zper && z == 0;
    a.whi = !zper && z == nz - 1;
    return a;
}

// Pre-collision deviations of cell x of the row: the value stored at x - c_i,
// or, where x - c_i lies in a wall, the opposite population stored at x
// itself (halfway bounce-back).
template <int ST>
__device__ __forceinline__ void pull(const IBLB_GLOBAL char *__restrict__ src, uint64_t pb,
                                     const RowAddr &ra, int x, int nx, float inv,
                                     typename Stor<ST>::R (&g)[Q]) {
    using S = Stor<ST>;
    using T = typename S::T;
    constexpr uint32_t EB = sizeof(T);
    const uint32_t xo = (uint32_t)x * EB;
    const uint32_t xmo = (uint32_t)(x == 0 ? nx - 1 : x - 1) * EB;
    const uint32_t xpo = (uint32_t)(x == nx - 1 ? 0 : x + 1) * EB;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
        const bool bb = (cz == 1 && ra.wlo) || (cz == -1 && ra.whi);
        uint32_t off;
        const IBLB_GLOBAL char *base;
        if (bb) {
            base = src + (uint64_t)opp_of(i) * pb;
            off = ra.ro[1][1] + xo;
        } else {
            base = src + (uint64_t)i * pb;
            off = ra.ro[cy + 1][cz + 1] + (cx == 1 ? xmo : (cx == -1 ? xpo : xo));
        }
        g[i] = S::ld((const T *)(const IBLB_GLOBAL T *)(base + off), inv);
    }
}

// ------------------------------------------------------- stream + collide
// One launch advances every cell of every box by one step.  A workgroup
// takes whole x-rows (a row group); threads stride along x, so the +-1
// shifted loads of a row stay inside one workgroup.  UROW: every wavefront
// lies in a single row (threads_x a multiple of 64), so the row addressing
// is wave-uniform and kept in scalar registers.
template <int ST, bool UROW>
__global__ void __launch_bounds__(K1_MAX_THREADS)
    k_stream_collide(DevPtrs P, int parity, int full_u, float scale, float inv) {
    using S = Stor<ST>;
    using T = typename S::T;
    using R = typename S::R;
    constexpr uint32_t EB = sizeof(T);
    const int tx = threadIdx.x, ty = threadIdx.y, BX = blockDim.x, BY = blockDim.y;
    const int ctr = *P.ctr;
    const IBLB_CONST RowGroup *rows = (const IBLB_CONST RowGroup *)P.rows;
    for (int gi = blockIdx.x; gi < P.n_rowgroups; gi += gridDim.x) {
        const IBLB_CONST RowGroup &rg = rows[gi];
        const IBLB_CONST BoxDev *B = (const IBLB_CONST BoxDev *)P.boxes + rg.box;
        const int nx = B->nx, ny = B->ny, nz = B->nz, sx = B->sx;
        const bool zper = B->zbc == 1;
        const uint64_t pb = (uint64_t)B->plane * EB;
        const IBLB_GLOBAL char *__restrict__ src = (const IBLB_GLOBAL char *)B->f[parity];
        IBLB_GLOBAL char *__restrict__ dst = (IBLB_GLOBAL char *)B->f[parity ^ 1];
        const R omega = (R)B->omega, guo = (R)B->guo, rho0 = (R)B->rho0;
        const R gx = (R)B->g[0], gy = (R)B->g[1], gz = (R)B->g[2];
        const IBLB_GLOBAL int32_t *__restrict__ stamp = (const IBLB_GLOBAL int32_t *)B->stamp;
        const IBLB_GLOBAL R *__restrict__ Fb = (const IBLB_GLOBAL R *)B->Fband;
        IBLB_GLOBAL R *__restrict__ ub = (IBLB_GLOBAL R *)B->uband;
        const int tnx = B->tnx, tny = B->tny;
        for (int r0 = rg.r0 + ty; r0 < rg.r1; r0 += BY) {
            const int r = UROW ? __builtin_amdgcn_readfirstlane(r0) : r0;
            const int z = r / ny, y = r - z * ny;
            const RowAddr ra = row_addr(y, z, ny, nz, sx, zper, EB);
            const int64_t trow = ((int64_t)(z >> 2) * tny + (y >> 2)) * tnx;
            const int lyz = ((z & 3) << 4) | ((y & 3) << 2);
            for (int x = tx; x < nx; x += BX) {
                R g[Q];
                pull<ST>(src, pb, ra, x, nx, inv, g);
                const int64_t tile = trow + (x >> 2);
                const int loc = lyz | (x & 3);
                const bool stamped = stamp[tile] == ctr;
                R Fx = gx, Fy = gy, Fz = gz;
                if (stamped) {
                    const IBLB_GLOBAL R *fp = Fb + tile * 3 * TILE_CELLS + loc;
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
                const uint32_t own = ra.ro[1][1] + (uint32_t)x * EB;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const R w = (R)w_of(i);
                    const R cu = (R)cx_of(i) * ux + (R)cy_of(i) * uy + (R)cz_of(i) * uz;
                    const R cF = (R)cx_of(i) * Fx + (R)cy_of(i) * Fy + (R)cz_of(i) * Fz;
                    // f_eq - w rho0 (Eq. 3) and the Guo source (Eq. 4), cs^2 = 1/3
                    const R geq = w * (drho + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq));
                    const R src_i = guo * w * (R(3) * (cF - uF) + R(9) * cu * cF);
                    S::st((T *)(IBLB_GLOBAL T *)(dst + (uint64_t)i * pb + own),
                          g[i] + omega * (geq - g[i]) + src_i, scale);
                }
                if (stamped || full_u) {
                    IBLB_GLOBAL R *up = ub + tile * 3 * TILE_CELLS + loc;
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

// ------------------------------------------------------- per-triangle pass
// One thread per triangle (a,b,c): N = (q_b - q_a) x (q_c - q_a), area
// A_t = |N|/2, unit normal n_t, the volume-gradient share N/6 and the three
// corner forces -sigma dA_t/dq = (sigma/2)(q_prev - q_next) x n_t, stored as
// a record [TREC][Ttot] for the node gather.  Also the FP64 volume
// sum_t (a-r).((b-r)x(c-r))/6 and area per chunk of 256 triangles
// (positions relative to the droplet's reference point r), fixed tree.

template <typename R>
__global__ void __launch_bounds__(256) k_tri(DevPtrs P) {
    __shared__ double sv[256], sa[256];
    const TriChunk ch = P.chunks[blockIdx.x];
    const DropDev &D = P.drops[ch.drop];
    const R *qh = (const R *)P.qh, *ql = (const R *)P.ql;
    const int t = ch.t0 + threadIdx.x;
    const int T = P.Ttot, N = P.Ntot;
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
        R *tr = (R *)P.trec;
        tr[0 * T + t] = R(0.5) * len;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            tr[(1 + k) * T + t] = nt[k];
            tr[(4 + k) * T + t] = Nt[k] / R(6);
            tr[(7 + k) * T + t] = hs * f0[k];
            tr[(10 + k) * T + t] = hs * f1[k];
            tr[(13 + k) * T + t] = hs * f2[k];
        }
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
// triangles (CSR, ascending triangle id) the corner surface-tension forces,
// the 1-ring area chi, the sum of unit face normals and the volume
// gradient; then the wetting force -chi Pi(d) n/3 with Pi from integer
// powers (Eq. 10) and the optional volume penalty.  Also: base cell
// floor(q - 1/2) (decided exactly from the hi/lo pair), the four Peskin
// weights per axis, the block's stencil bounding box, and (mode 0) the epoch
// stamps of every tile holding a stencil cell.
template <typename R>
__global__ void __launch_bounds__(256) k_node(DevPtrs P, int mode) {
    const int lane = threadIdx.x & 63;
    const int blk = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (blk >= P.nblk) return;
    const int d = P.blk_drop[blk];
    const DropDev &D = P.drops[d];
    const BoxDev &B = P.boxes[D.box];
    const int N = P.Ntot, T = P.Ttot;
    const R *qh = (const R *)P.qh, *ql = (const R *)P.ql;
    const R *tr = (const R *)P.trec;
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
        const int e0 = P.csr_off[j], e1 = P.csr_off[j + 1];
        for (int e = e0; e < e1; e += 8) {
            int code[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) code[k] = e + k < e1 ? P.csr_ent[e + k] : -1;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (code[k] < 0) continue;
                const int t = code[k] / 3, c = code[k] - 3 * t;
                chi += tr[t];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    ns[a] += tr[(1 + a) * T + t];
                    gv[a] += tr[(4 + a) * T + t];
                    st[a] += tr[(7 + 3 * c + a) * T + t];
                }
            }
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
            const int ctr = *P.ctr;
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
                        ((IBLB_GLOBAL int32_t *)B.stamp)[((int64_t)tl[2][iz] * B.tny + tl[1][iy]) *
                                                              B.tnx + tl[0][ix]] = ctr;
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

// ----------------------------------------------------- stamped-tile list
// One wavefront per chunk of 64 tiles appends the chunk's stamped tiles to
// the list of this epoch (one integer atomic per chunk; the order of the
// list does not affect any result).  Also clears the other epoch's count.
__global__ void __launch_bounds__(256) k_compact(DevPtrs P) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int ctr = *P.ctr;
    const int slot = ctr & 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) P.tile_count[slot ^ 1] = 0;
    if (c >= P.total_tiles / TILE_CELLS) return;
    const BoxDev &B = P.boxes[P.tchunk_box[c]];
    const int lt = c * TILE_CELLS + lane - B.tile_base;
    const bool st = lt < B.n_tiles && ((const IBLB_GLOBAL int32_t *)B.stamp)[lt] == ctr;
    const uint64_t m = __ballot(st);
    if (m == 0) return;
    int base = 0;
    if (lane == 0) base = atomicAdd(P.tile_count + slot, __popcll(m));
    base = __shfl(base, 0, 64);
    if (st) P.tile_list[base + __popcll(m & ((1ull << lane) - 1ull))] = c * TILE_CELLS + lane;
}

template <typename R> __device__ __forceinline__ R bcast(R v, int l);
template <> __device__ __forceinline__ float bcast<float>(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <> __device__ __forceinline__ double bcast<double>(double v, int l) {
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    return __hiloint2double(hi, lo);
}

// ----------------------------------------------------------------- spread
// Eq. 8 as a gather: one wavefront per stamped tile, one lane per cell.
// Candidate node blocks (those whose stencil box meets the tile) are taken
// in ascending block order and, inside a block, nodes whose own stencil
// meets the tile in ascending node order, so every cell sums its
// contributions in one fixed order.  A block's node data are loaded once
// (one node per lane) and broadcast node by node.  Writes all 64 cells.
template <typename R>
__global__ void __launch_bounds__(256) k_spread(DevPtrs P) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int nwaves = gridDim.x * 4;
    const int ctr = *P.ctr;
    const int count = P.tile_count[ctr & 1];
    const int N = P.Ntot, nb = P.nblk;
    const R *phi = (const R *)P.phi, *wg = (const R *)P.wgt;
    for (int i = wave; i < count; i += nwaves) {
        const int gt = P.tile_list[i];
        const BoxDev &B = P.boxes[P.tchunk_box[gt / TILE_CELLS]];
        const int lt = gt - B.tile_base;
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
            if (mb < B.blk_end)
                hit = meets(P.bbox[0 * nb + mb], P.bbox[1 * nb + mb], x0, x1, B.nx, true) &&
                      meets(P.bbox[2 * nb + mb], P.bbox[3 * nb + mb], y0, y1, B.ny, true) &&
                      meets(P.bbox[4 * nb + mb], P.bbox[5 * nb + mb], z0, z1, B.nz, zper);
            uint64_t bmask = __ballot(hit);
            while (bmask) {
                const int blk = kb + __builtin_ctzll(bmask);
                bmask &= bmask - 1;
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
                if (!nmask) continue;
                int s0x = 0, s0y = 0, s0z = 0;
                R w[12], f[3];
#pragma unroll
                for (int k = 0; k < 12; ++k) w[k] = 0;
                f[0] = f[1] = f[2] = 0;
                if (nh) {
                    s0x = P.s0[j];
                    s0y = P.s0[N + j];
                    s0z = P.s0[2 * N + j];
#pragma unroll
                    for (int k = 0; k < 12; ++k) w[k] = wg[k * N + j];
#pragma unroll
                    for (int k = 0; k < 3; ++k) f[k] = phi[k * N + j];
                }
                while (nmask) {
                    const int nl = __builtin_ctzll(nmask);
                    nmask &= nmask - 1;
                    int ox = cxl - __builtin_amdgcn_readlane(s0x, nl);
                    int oy = cyl - __builtin_amdgcn_readlane(s0y, nl);
                    int oz = czl - __builtin_amdgcn_readlane(s0z, nl);
                    if (ox < 0) ox += B.nx;
                    if (oy < 0) oy += B.ny;
                    if (zper && oz < 0) oz += B.nz;
                    R wx[4], wy[4], wz[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        wx[k] = bcast(w[k], nl);
                        wy[k] = bcast(w[4 + k], nl);
                        wz[k] = bcast(w[8 + k], nl);
                    }
                    const R fx = bcast(f[0], nl), fy = bcast(f[1], nl), fz = bcast(f[2], nl);
                    const R ax = ox == 0 ? wx[0] : ox == 1 ? wx[1] : ox == 2 ? wx[2] : ox == 3 ? wx[3] : R(0);
                    const R ay = oy == 0 ? wy[0] : oy == 1 ? wy[1] : oy == 2 ? wy[2] : oy == 3 ? wy[3] : R(0);
                    const R az = oz == 0 ? wz[0] : oz == 1 ? wz[1] : oz == 2 ? wz[2] : oz == 3 ? wz[3] : R(0);
                    const R wv = ax * ay * az;
                    acc0 += fx * wv;
                    acc1 += fy * wv;
                    acc2 += fz * wv;
                }
            }
        }
        IBLB_GLOBAL R *Fb = (IBLB_GLOBAL R *)B.Fband + (int64_t)lt * 3 * TILE_CELLS;
        Fb[lane] = acc0;
        Fb[TILE_CELLS + lane] = acc1;
        Fb[2 * TILE_CELLS + lane] = acc2;
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
    const int blk = blockIdx.x;
    const DropDev &D = P.drops[P.blk_drop[blk]];
    const BoxDev &B = P.boxes[D.box];
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
    auto gidx = [&](int x, int y, int z) -> int64_t {
        const int64_t tile = ((int64_t)(z >> 2) * B.tny + (y >> 2)) * B.tnx + (x >> 2);
        return tile * 3 * TILE_CELLS + (((z & 3) << 4) | ((y & 3) << 2) | (x & 3));
    };
    if (staged) {
        const int x0w = wrapn(bx0, B.nx);
        for (int r = tid >> 4; r < ey * ez; r += 16) {
            const int iz = r / ey, iy = r - iz * ey;
            const int y = wrapn(by0 + iy, B.ny);
            const int z = zper ? wrapn(bz0 + iz, B.nz) : bz0 + iz;
            for (int ix = tid & 15; ix < ex; ix += 16) {
                int x = x0w + ix;
                while (x >= B.nx) x -= B.nx;
                const int64_t g = gidx(x, y, z);
                const int c = r * ex + ix;
                su[c] = ub[g];
                su[MAXR + c] = ub[g + TILE_CELLS];
                su[2 * MAXR + c] = ub[g + 2 * TILE_CELLS];
            }
        }
    }
    __syncthreads();
    const int j = blk * NB + lane;
    const bool valid = j - D.node_off < D.n_nodes;
    R U0 = 0, U1 = 0, U2 = 0;
    if (valid) {
        const R *wg = (const R *)P.wgt;
        const int bx = P.base[j], by = P.base[N + j], bz = P.base[2 * N + j];
        const int z = bz - 1 + wave;
        if (zper || (z >= 0 && z < B.nz)) {
            const R wz = wg[(8 + wave) * N + j];
            R wx[4], wy[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                wx[o] = wg[o * N + j];
                wy[o] = wg[(4 + o) * N + j];
            }
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
    const IBLB_GLOBAL char *src = (const IBLB_GLOBAL char *)B.f[parity];
    const uint64_t pb = (uint64_t)B.plane * sizeof(typename S::T);
    double m = 0.0, umax = 0.0;
    for (int r = r0; r < r1; ++r) {
        const int z = r / B.ny, y = r - z * B.ny;
        const RowAddr ra = row_addr(y, z, B.ny, B.nz, B.sx, B.zbc == 1, sizeof(typename S::T));
        for (int x = threadIdx.x; x < B.nx; x += 256) {
            R g[Q];
            pull<ST>(src, pb, ra, x, B.nx, inv, g);
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
    hipLaunchKernelGGL(k_compact, dim3((chunks + 3) / 4), dim3(256), 0, s, P);
    const int grid = min((P.total_tiles + 3) / 4, 2048);
    if (f64) hipLaunchKernelGGL(k_spread<double>, dim3(grid), dim3(256), 0, s, P);
    else hipLaunchKernelGGL(k_spread<float>, dim3(grid), dim3(256), 0, s, P);
    return hipGetLastError();
}

template <int ST>
static hipError_t launch_sc(const DevPtrs &P, int parity, int full_u, float scale, const Launch &L,
                            hipStream_t s) {
    // never launch a shape the kernel was not compiled for
    if (L.bx < 1 || L.by < 1 || L.bx * L.by > K1_MAX_THREADS || L.grid < 1) return hipErrorInvalidValue;
    const dim3 block(L.bx, L.by), grid(L.grid);
    const float inv = 1.0f / scale;
    if (L.bx % 64 == 0)
        hipLaunchKernelGGL((k_stream_collide<ST, true>), grid, block, 0, s, P, parity, full_u, scale, inv);
    else
        hipLaunchKernelGGL((k_stream_collide<ST, false>), grid, block, 0, s, P, parity, full_u, scale, inv);
    return hipGetLastError();
}

hipError_t launch_stream_collide(const DevPtrs &P, int storage, int parity, int full_u,
                                 float scale, const Launch &L, hipStream_t s) {
    switch (storage) {
    case 0: return launch_sc<0>(P, parity, full_u, scale, L, s);
    case 1: return launch_sc<1>(P, parity, full_u, scale, L, s);
    case 2: return launch_sc<2>(P, parity, full_u, scale, L, s);
    default: return launch_sc<3>(P, parity, full_u, scale, L, s);
    }
}

hipError_t launch_interp(const DevPtrs &P, bool f64, int mode, double *Uout, hipStream_t s) {
    if (P.nblk == 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL(k_interp<double>, dim3(P.nblk), dim3(256), 0, s, P, mode, Uout);
    else hipLaunchKernelGGL(k_interp<float>, dim3(P.nblk), dim3(256), 0, s, P, mode, Uout);
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
