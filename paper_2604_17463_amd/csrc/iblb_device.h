// Device-side helpers shared by the fluid and mesh kernels (gfx950).
#pragma once
#include "iblb_internal.h"


#include <cfloat>
#include <climits>

namespace iblb {

// Address spaces: tables that stay constant during a launch are read through
// the constant space (scalar loads); population and band pointers taken from
// those tables are global memory.
#define IBLB_CONST __attribute__((address_space(4)))
#define IBLB_GLOBAL __attribute__((address_space(1)))

// ---------------------------------------------------------------- storage
// Population storage: T in memory, R in registers.  raw() returns the stored
// value (for FP16 still multiplied by the deviation scale s), put() rounds to
// nearest even, put_nt() is the same store marked as streaming (no reuse
// expected before it leaves the caches).
template <int ST> struct Stor;
template <> struct Stor<0> {  // FP64 deviations
    using T = double;
    using R = double;
    static constexpr bool SCALED = false;
    static __device__ __forceinline__ R raw(const IBLB_GLOBAL T *p) { return *p; }
    static __device__ __forceinline__ void put(IBLB_GLOBAL T *p, R v) { *p = v; }
    static __device__ __forceinline__ void put_nt(IBLB_GLOBAL T *p, R v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Stor<1> {  // FP32 deviations
    using T = float;
    using R = float;
    static constexpr bool SCALED = false;
    static __device__ __forceinline__ R raw(const IBLB_GLOBAL T *p) { return *p; }
    static __device__ __forceinline__ void put(IBLB_GLOBAL T *p, R v) { *p = v; }
    static __device__ __forceinline__ void put_nt(IBLB_GLOBAL T *p, R v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Stor<2> {  // binary16, deviations times s
    using T = _Float16;
    using R = float;
    static constexpr bool SCALED = true;
    static __device__ __forceinline__ R raw(const IBLB_GLOBAL T *p) { return (R)*p; }
    static __device__ __forceinline__ void put(IBLB_GLOBAL T *p, R v) { *p = (T)v; }
    static __device__ __forceinline__ void put_nt(IBLB_GLOBAL T *p, R v) { __builtin_nontemporal_store((T)v, p); }
};
template <> struct Stor<3> {  // bfloat16 deviations
    using T = __bf16;
    using R = float;
    static constexpr bool SCALED = false;
    static __device__ __forceinline__ R raw(const IBLB_GLOBAL T *p) { return (R)*p; }
    static __device__ __forceinline__ void put(IBLB_GLOBAL T *p, R v) { *p = (T)v; }
    static __device__ __forceinline__ void put_nt(IBLB_GLOBAL T *p, R v) { __builtin_nontemporal_store((T)v, p); }
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
// Minimum / maximum over the 64 lanes of a wave whose lanes are all active:
// rotate-and-combine inside each row of 16 lanes (DPP row_ror 8, 4, 2, 1:
// no LDS round trip), then combine the four row results as scalars.
template <bool MAX> __device__ __forceinline__ int wave_minmax(int v) {
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x124, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x122, 0xf, 0xf, false));
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x121, 0xf, 0xf, false));
    const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return op(op(r0, r1), op(r2, r3));
}
__device__ __forceinline__ int wave_min(int v) { return wave_minmax<false>(v); }
__device__ __forceinline__ int wave_max(int v) { return wave_minmax<true>(v); }

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

// Halfway bounce-back on a moving wall: a population reflected at the wall
// z = 0 (c_z = +1 in the first layer) or at z = nz (c_z = -1 in the last)
// also carries the momentum the wall imparts, 2 w_i rho0 (c_i . u_w) / c_s^2.
// k = 6 rho0 s (u_x, u_y) of the lower wall, then of the upper wall, with s
// the storage scale (g is in stored units).
template <typename R>
__device__ __forceinline__ void wall_shift(R (&g)[Q], bool wlo, bool whi, const R (&k)[4]) {
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const int cz = cz_of(i);
        if (cz == 0) continue;
        const R kx = cz == 1 ? k[0] : k[2], ky = cz == 1 ? k[1] : k[3];
        const R d = (R)w_of(i) * ((R)cx_of(i) * kx + (R)cy_of(i) * ky);
        if (cz == 1 ? wlo : whi) g[i] += d;
    }
}

// Byte offsets of cell x and of its periodic x-neighbours x - 1, x + 1
// within a row.
struct XOff {
    uint32_t c, m, p;
};
template <uint32_t EB> __device__ __forceinline__ XOff x_off(int x, int nx) {
    return {(uint32_t)x * EB, (uint32_t)(x == 0 ? nx - 1 : x - 1) * EB,
            (uint32_t)(x == nx - 1 ? 0 : x + 1) * EB};
}

// Stored pre-collision deviations of cell x of the row: the value stored at
// x - c_i, or, where x - c_i lies in a wall, the opposite population stored
// at x itself (halfway bounce-back).  The row part of every address (plane,
// source row) depends on `ra` only; when `ra` is the same in all lanes it
// stays in scalar registers and each load adds only the lane's x offset.
template <int ST>
__device__ __forceinline__ void pull_raw(const IBLB_GLOBAL char *__restrict__ src, uint64_t pb,
                                         const RowAddr &ra, const XOff &xo, typename Stor<ST>::R (&g)[Q]) {
    using S = Stor<ST>;
    using T = typename S::T;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
        const bool bb = (cz == 1 && ra.wlo) || (cz == -1 && ra.whi);
        const IBLB_GLOBAL char *row = bb ? src + (uint64_t)opp_of(i) * pb + ra.ro[1][1]
                                         : src + (uint64_t)i * pb + ra.ro[cy + 1][cz + 1];
        const uint32_t lo = bb ? xo.c : (cx == 1 ? xo.m : (cx == -1 ? xo.p : xo.c));
        g[i] = S::raw((const IBLB_GLOBAL T *)(row + lo));
    }
}

// The same in true (unscaled) deviations.
template <int ST>
__device__ __forceinline__ void pull(const IBLB_GLOBAL char *__restrict__ src, uint64_t pb, const RowAddr &ra,
                                     int x, int nx, float inv, typename Stor<ST>::R (&g)[Q]) {
    using S = Stor<ST>;
    pull_raw<ST>(src, pb, ra, x_off<sizeof(typename S::T)>(x, nx), g);
    if constexpr (S::SCALED) {
#pragma unroll
        for (int i = 0; i < Q; ++i) g[i] *= inv;
    }
}

// BGK collision with the Guo source (Eqs. 1-6) of one cell in deviation
// form.  g holds the pulled deviations in stored units (times s for scaled
// storage), F the force density; out receives the 19 post-collision
// deviations in stored units, u (with the half-force correction) and rho
// are returned.
//
// Arithmetic: with c_s^2 = 1/3 the post-collision value is
//   g*_i = (1 - omega) g_i + omega f^eq_i' + S_i,   f^eq_i' = f^eq_i - w_i rho0.
// Population i and its opposite share c.u and c.F up to sign, so the
// parts even in c (E_i) and odd in c (O_i) are formed once per pair:
//   E_i = w_i [omega (drho + rho (4.5 (c.u)^2 - 1.5 u.u)) + guo (9 (c.u)(c.F) - 3 u.F)]
//   O_i = w_i [3 omega rho (c.u) + 3 guo (c.F)]
//   g*_i = (1 - omega) g_i + E_i + O_i,  g*_opp = (1 - omega) g_opp + E_i - O_i.
// Scaled storage multiplies E and O by s (folded into the weights) and
// divides only the four moments by s.
template <int ST>
__device__ __forceinline__ void collide(const typename Stor<ST>::R (&g)[Q], typename Stor<ST>::R Fx,
                                        typename Stor<ST>::R Fy, typename Stor<ST>::R Fz,
                                        typename Stor<ST>::R rho0, typename Stor<ST>::R omega,
                                        typename Stor<ST>::R guo, float scale, float inv,
                                        typename Stor<ST>::R (&out)[Q], typename Stor<ST>::R (&u)[3],
                                        typename Stor<ST>::R &rho_out) {
    using S = Stor<ST>;
    using R = typename S::R;
    // moments (Eqs. 5-6) from pair sums and differences
    R sp[9], dp[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        sp[k] = g[k + 1] + g[k + 10];
        dp[k] = g[k + 1] - g[k + 10];
    }
    R drho = g[0], jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        drho += sp[k];
        if (cx_of(k + 1) == 1) jx += dp[k];
        if (cx_of(k + 1) == -1) jx -= dp[k];
        if (cy_of(k + 1) == 1) jy += dp[k];
        if (cy_of(k + 1) == -1) jy -= dp[k];
        if (cz_of(k + 1) == 1) jz += dp[k];
        if (cz_of(k + 1) == -1) jz -= dp[k];
    }
    if constexpr (S::SCALED) {
        const R iv = (R)inv;
        drho *= iv;
        jx *= iv;
        jy *= iv;
        jz *= iv;
    }
    const R rho = rho0 + drho;
    const R irho = R(1) / rho;
    const R ux = (jx + R(0.5) * Fx) * irho;
    const R uy = (jy + R(0.5) * Fy) * irho;
    const R uz = (jz + R(0.5) * Fz) * irho;
    const R usq = ux * ux + uy * uy + uz * uz;
    const R uF = ux * Fx + uy * Fy + uz * Fz;
    const R base = omega * (drho - R(1.5) * rho * usq) - R(3) * guo * uF;
    const R ea = R(4.5) * omega * rho, eb = R(9) * guo;
    const R oa = R(3) * omega * rho, ob = R(3) * guo;
    const R omc = R(1) - omega;
    R w0 = R(1) / R(3), w1 = R(1) / R(18), w2 = R(1) / R(36);
    if constexpr (S::SCALED) {
        w0 *= (R)scale;
        w1 *= (R)scale;
        w2 *= (R)scale;
    }
    out[0] = omc * g[0] + w0 * base;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int i = k + 1;
        const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
        R cu = 0, cF = 0;
        if (cx == 1) { cu += ux; cF += Fx; }
        if (cx == -1) { cu -= ux; cF -= Fx; }
        if (cy == 1) { cu += uy; cF += Fy; }
        if (cy == -1) { cu -= uy; cF -= Fy; }
        if (cz == 1) { cu += uz; cF += Fz; }
        if (cz == -1) { cu -= uz; cF -= Fz; }
        const R w = (cx * cx + cy * cy + cz * cz) == 1 ? w1 : w2;
        const R E = w * (cu * (ea * cu + eb * cF) + base);
        const R O = w * (oa * cu + ob * cF);
        out[i] = omc * g[i] + (E + O);
        out[i + 9] = omc * g[i + 9] + (E - O);
    }
    u[0] = ux;
    u[1] = uy;
    u[2] = uz;
    rho_out = rho;
}


// Store the 19 post-collision values at byte offset `own` of each plane.
template <int ST, bool NT>
__device__ __forceinline__ void store_ptr(IBLB_GLOBAL char *__restrict__ dst, uint64_t pb, uint32_t own,
                                          const typename Stor<ST>::R (&out)[Q]) {
    using S = Stor<ST>;
    using T = typename S::T;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        IBLB_GLOBAL T *p = (IBLB_GLOBAL T *)(dst + (uint64_t)i * pb + own);
        if constexpr (NT)
            S::put_nt(p, out[i]);
        else
            S::put(p, out[i]);
    }
}

// ------------------------------------------------------- buffer addressing
// Populations of one buffer through two buffer resources: planes 0..9 from
// the buffer start and planes 10..18 from plane 10, so that each offset
// (plane part + row + x, all 32-bit) stays below 4 GiB as long as ten planes
// do.  In a wave that lies in one row the plane and row parts are scalar
// (soffset) and only the x part is per lane (voffset).
constexpr int32_t BUF_WORD3 = 0x00020000;  // gfx9 raw buffer: 32-bit data format

struct PopRes {
    __amdgpu_buffer_rsrc_t lo, hi;
};
__device__ __forceinline__ PopRes pop_res(const void *base, uint64_t pb) {
    const char *b = (const char *)base;
    const uint64_t nlo = 10 * pb, nhi = 9 * pb;
    return {__builtin_amdgcn_make_buffer_rsrc((void *)b, (short)0,
                                              (int)(uint32_t)(nlo < BUF_MAX_PLANE_GROUP ? nlo : BUF_MAX_PLANE_GROUP),
                                              BUF_WORD3),
            __builtin_amdgcn_make_buffer_rsrc((void *)(b + 10 * pb), (short)0, (int)(uint32_t)nhi, BUF_WORD3)};
}

typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
template <typename T> __device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s);
template <> __device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
}
template <> __device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
}
template <> __device__ __forceinline__ _Float16 bload<_Float16>(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
}
template <> __device__ __forceinline__ __bf16 bload<__bf16>(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
}
// aux bit 1 marks the store non-temporal
template <int AUX> __device__ __forceinline__ void bstore(double x, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, x), r, v, s, AUX);
}
template <int AUX> __device__ __forceinline__ void bstore(float x, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, v, s, AUX);
}
template <int AUX> __device__ __forceinline__ void bstore(_Float16 x, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, AUX);
}
template <int AUX> __device__ __forceinline__ void bstore(__bf16 x, __amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, AUX);
}

// pull_raw through buffer resources.  ROWV = false: the lanes of the wave
// share `ra`, so the row goes into the scalar offset with the plane; true:
// each lane has its own row, added to its per-lane offset (32-bit, so a
// lane holds no 64-bit addresses).
template <int ST, bool ROWV = false>
__device__ __forceinline__ void pull_buf(const PopRes &rs, uint32_t pb, const RowAddr &ra, const XOff &xo,
                                         typename Stor<ST>::R (&g)[Q]) {
    using T = typename Stor<ST>::T;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_of(i), cy = cy_of(i), cz = cz_of(i);
        const int o = opp_of(i);
        const uint32_t xv = cx == 1 ? xo.m : (cx == -1 ? xo.p : xo.c);
        if constexpr (ROWV) {
            // a wall population reads the opposite one at the cell itself;
            // the planes i and opp(i) lie in different halves, so both loads
            // are issued and the lane keeps the one it needs
            if (cz == 0) {
                g[i] = (typename Stor<ST>::R)bload<T>(i < 10 ? rs.lo : rs.hi, ra.ro[cy + 1][1] + xv,
                                                      (uint32_t)(i % 10) * pb);
            } else {
                const bool bb = (cz == 1 && ra.wlo) || (cz == -1 && ra.whi);
                const T a = bload<T>(i < 10 ? rs.lo : rs.hi, ra.ro[cy + 1][cz + 1] + xv, (uint32_t)(i % 10) * pb);
                const T b = bload<T>(o < 10 ? rs.lo : rs.hi, ra.ro[1][1] + xo.c, (uint32_t)(o % 10) * pb);
                g[i] = (typename Stor<ST>::R)(bb ? b : a);
            }
        } else {
            const bool bb = (cz == 1 && ra.wlo) || (cz == -1 && ra.whi);
            const __amdgpu_buffer_rsrc_t r = bb ? (o < 10 ? rs.lo : rs.hi) : (i < 10 ? rs.lo : rs.hi);
            const uint32_t so = bb ? (uint32_t)(o % 10) * pb + ra.ro[1][1]
                                   : (uint32_t)(i % 10) * pb + ra.ro[cy + 1][cz + 1];
            const uint32_t vo = bb ? xo.c : xv;
            g[i] = (typename Stor<ST>::R)bload<T>(r, vo, so);
        }
    }
}

// store_ptr through buffer resources; `own_row` is the row offset, scalar
// (ROWV = false) or per lane (ROWV = true).
template <int ST, bool NT, bool ROWV = false>
__device__ __forceinline__ void store_buf(const PopRes &rd, uint32_t pb, uint32_t own_row, uint32_t xoc,
                                          const typename Stor<ST>::R (&out)[Q]) {
    using T = typename Stor<ST>::T;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if constexpr (ROWV)
            bstore<NT ? 2 : 0>((T)out[i], i < 10 ? rd.lo : rd.hi, own_row + xoc, (uint32_t)(i % 10) * pb);
        else
            bstore<NT ? 2 : 0>((T)out[i], i < 10 ? rd.lo : rd.hi, xoc, (uint32_t)(i % 10) * pb + own_row);
    }
}

}  // namespace iblb
