// Device-side helpers shared by the fluid and mesh kernels (gfx950).
#pragma once
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

__device__ __forceinline__ int wrapn(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
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

// Value of v in lane l (l wave-uniform), as a scalar.
template <typename R> __device__ __forceinline__ R bcast(R v, int l);
template <> __device__ __forceinline__ float bcast<float>(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
template <> __device__ __forceinline__ double bcast<double>(double v, int l) {
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int bcast_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

template <typename R> struct Vec4;
template <> struct Vec4<float> { using T = float4; };
template <> struct Vec4<double> { using T = double4; };

template <typename R> __device__ __forceinline__ R pick4(int o, R a0, R a1, R a2, R a3) {
    return o == 0 ? a0 : (o == 1 ? a1 : (o == 2 ? a2 : (o == 3 ? a3 : R(0))));
}

// Fixed-order FP64 sum of a droplet's per-chunk partials; every lane of the
// wave returns the same value, identical in every wave that calls it.
__device__ __forceinline__ double droplet_partial_sum(const double *part, int off, int n, int lane) {
    double s = 0.0;
    for (int k = lane; k < n; k += 64) s += part[off + k];
    return wave_sum(s);
}

// Node coordinate = hi + lo (lo keeps what the advection increments lose in
// hi; stays zero in practice for FP64).
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
template <typename R>
__device__ __forceinline__ void diff(const Node3<R> &b, const Node3<R> &a, R (&d)[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = (b.h[k] - a.h[k]) + (b.l[k] - a.l[k]);
}
template <typename R>
__device__ __forceinline__ void cross3(const R (&a)[3], const R (&b)[3], R (&c)[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Does the interval [lo, hi] (unwrapped) meet cells [t0, t1] of an axis of
// n cells?  Periodic axes wrap; others compare directly.
__device__ __forceinline__ bool meets(int lo, int hi, int t0, int t1, int n, bool per) {
    if (!per) return lo <= t1 && hi >= t0;
    if (hi - lo + 1 >= n) return true;
    const int l = wrapn(lo, n), h = l + (hi - lo);
    return (l <= t1 && h >= t0) || (l <= t1 + n && h >= t0 + n);
}

// ------------------------------------------------------- pulled populations
// Addressing of one x-row for the pull: byte offsets (32-bit, a plane is
// < 4 GiB) of the 9 source rows (y - c_y, z - c_z) and the wall flags.
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
        zm = max(zm, 0);  // wall rows are never read through these
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

// BGK collision with the Guo source (Eqs. 1-6) of one cell in deviation
// form, given its pulled deviations g and force density F: writes the 19
// post-collision deviations at byte offset `own` of each plane of dst and
// returns u (with the half-force correction) and rho.
template <int ST>
__device__ __forceinline__ void collide_store(typename Stor<ST>::R (&g)[Q], typename Stor<ST>::R Fx,
                                              typename Stor<ST>::R Fy, typename Stor<ST>::R Fz,
                                              typename Stor<ST>::R rho0, typename Stor<ST>::R omega,
                                              typename Stor<ST>::R guo, IBLB_GLOBAL char *dst,
                                              uint64_t pb, uint32_t own, float scale,
                                              typename Stor<ST>::R (&u)[3],
                                              typename Stor<ST>::R &rho_out) {
    using S = Stor<ST>;
    using T = typename S::T;
    using R = typename S::R;
    // moments (Eqs. 5-6): rho = rho0 + sum g, rho u = sum c g + F/2
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
    u[0] = ux;
    u[1] = uy;
    u[2] = uz;
    rho_out = rho;
}

}  // namespace iblb
