/*
 * FP64 CPU oracle for the immersed boundary - lattice Boltzmann (IBLB)
 * wetting step of Bellantoni et al., "On the hydrodynamic behaviour of the
 * immersed boundary - lattice Boltzmann method for wetting problems".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow definition the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the library never does, and it
 * shares no code, header or table with the library.
 *
 * Every routine is written as the paper states it, in double precision, with
 * loops in the obvious order and no blocking or fusion:
 *   lattice      : D3Q19, c_s^2 = 1/3, dx = dt = 1                 (Sec. 2)
 *   equilibrium  : second-order f_eq                               (Eq. 3)
 *   Guo source   : S_i with the (1 - dt/2tau) prefactor            (Eq. 4)
 *   moments      : rho = sum f, u = (sum c f + F dt/2)/rho         (Eqs. 5-6)
 *   BGK step     : f(x+c,t+1) = f - (f - f_eq)/tau + S             (Eqs. 1-2)
 *   IB coupling  : interpolation / spreading with a discrete delta (Eqs. 7-8)
 *   forces       : surface tension (area gradient) and wetting
 *                  phi_Pi = -chi Pi(d) n / 3                       (Eqs. 9-11)
 *
 * Where the paper leaves a choice open, the reading taken is noted at the
 * routine (wall treatment, delta kernel, normal averaging, ...).
 *
 * Parity status: every routine below is pinned by the CPU tests (closed
 * forms, invariants, finite differences, brute force); the full multi-step
 * spreading dynamics has no printed data to compare with and is pinned only
 * through those pieces.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* D3Q19 velocity set in the oracle's own order: rest, 6 faces, 12 edges. */
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
};

/* Standard D3Q19 weights by speed class: 1/3 rest, 1/18 faces, 1/36 edges
 * (the paper names the weights w_i without listing them). */
static const double WV[Q] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
};
static inline double weight_of(int i) { return WV[i]; }

static int opposite_of(int i) {
    for (int k = 0; k < Q; ++k)
        if (CV[k][0] == -CV[i][0] && CV[k][1] == -CV[i][1] && CV[k][2] == -CV[i][2])
            return k;
    return -1;
}

/* c_s^2 = dx^2/(3 dt^2) = 1/3 with dx = dt = 1 */
static const double ICS2 = 3.0;      /* 1/c_s^2 */
static const double ICS4 = 9.0;      /* 1/c_s^4 */

/* Threads of the OpenMP loops from now on (n >= 1). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_lattice(int32_t *c, double *w, int32_t *opp) {
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = CV[i][a];
        w[i] = weight_of(i);
        opp[i] = opposite_of(i);
    }
}

/* Eq. 3: f_eq = w rho [1 + u.c/cs^2 + (u.c)^2/(2 cs^4) - u.u/(2 cs^2)]. */
static inline void feq_cell(double rho, const double *u, double *feq) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        feq[i] = weight_of(i) * rho *
                 (1.0 + cu * ICS2 + 0.5 * cu * cu * ICS4 - 0.5 * uu * ICS2);
    }
}

/* Eq. 4 (Guo): S_i = (1 - dt/(2 tau)) w_i [ (c_i - u)/cs^2 + (u.c_i) c_i / cs^4 ] . F */
static inline void guo_cell(double tau, const double *u, const double *F, double *S) {
    double pre = 1.0 - 1.0 / (2.0 * tau);
    for (int i = 0; i < Q; ++i) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        double s = 0.0;
        for (int a = 0; a < 3; ++a)
            s += ((CV[i][a] - u[a]) * ICS2 + cu * CV[i][a] * ICS4) * F[a];
        S[i] = pre * weight_of(i) * s;
    }
}

/* Eqs. 5-6: density and velocity with the half-force correction. */
static inline void moments_cell(const double *fcell, const double *F, double *rho, double *u) {
    double r = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        r += fcell[i];
        for (int a = 0; a < 3; ++a) m[a] += CV[i][a] * fcell[i];
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = (m[a] + 0.5 * F[a]) / r;
}

void orc_feq(double rho, const double *u, double *feq) { feq_cell(rho, u, feq); }
void orc_guo(double tau, const double *u, const double *F, double *S) { guo_cell(tau, u, F, S); }
void orc_moments(const double *fcell, const double *F, double *rho, double *u) {
    moments_cell(fcell, F, rho, u);
}

static inline int wrap(int i, int n) { return ((i % n) + n) % n; }
/* wrap for indices at most one period outside [0, n) */
static inline int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
static inline size_t cidx(int i, int j, int k, int nx, int ny) {
    return ((size_t)k * ny + j) * nx + i;
}

/*
 * One lattice Boltzmann step (Eqs. 1-6) for a whole box.
 *   f      : [19][nz][ny][nx] populations at time t (pre-collision)
 *   F      : [3][nz][ny][nx] spread IB force density, or NULL for none
 *   g      : uniform body force added to F everywhere
 *   fs     : scratch, same size as f (post-collision values)
 *   fnew   : [19][nz][ny][nx] populations at t+1
 *   rho,u  : moments at time t (u includes F/2), may be NULL
 * Streaming pulls f*_i(x - c_i) with periodic x and y.  In z the box is
 * periodic (zbc = 1) or closed by resting walls halfway between the first or
 * last cell layer and the ghost layer (zbc = 0): a population whose source
 * lies in the wall is the one that left x toward the wall, reflected
 * (f_i(x,t+1) = f*_opp(i)(x,t)).  The paper calls the wall a flat no-slip
 * solid and does not name the lattice scheme; halfway bounce-back is the
 * reading taken here.
 *   uwall  : NULL for resting walls, else the in-plane velocities of the
 *            walls, {x, y} of the wall at z = 0 then of the wall at z = nz.
 *            A wall moving with u_w adds to the reflected population the
 *            momentum it imparts, 2 w_i rho_w (c_i . u_w) / c_s^2 with
 *            rho_w = rho_wall (the free droplet in shear of Sec. 4 is
 *            driven by two such walls).
 */
void orc_lb_step(int nx, int ny, int nz, int zbc, double tau, const double *f,
                 const double *F, const double *g, const uint8_t *inside, double tau_in,
                 const double *uwall, double rho_wall,
                 double *fs, double *fnew, double *rho_out, double *u_out) {
    const size_t cells = (size_t)nx * ny * nz;
    int opp[Q];
    for (int i = 0; i < Q; ++i) opp[i] = opposite_of(i);

#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t x = cidx(i, j, k, nx, ny);
                double fc[Q], feq[Q], S[Q], Fx[3], rho, u[3];
                for (int q = 0; q < Q; ++q) fc[q] = f[q * cells + x];
                for (int a = 0; a < 3; ++a) Fx[a] = g[a] + (F ? F[a * cells + x] : 0.0);
                /* relaxation time of the cell: tau_in inside a droplet (Sec. 2,
                   below Eq. 13), tau elsewhere */
                const double tc = (inside && inside[x]) ? tau_in : tau;
                moments_cell(fc, Fx, &rho, u);
                feq_cell(rho, u, feq);
                guo_cell(tc, u, Fx, S);
                for (int q = 0; q < Q; ++q)
                    fs[q * cells + x] = fc[q] - (fc[q] - feq[q]) / tc + S[q];
                if (rho_out) rho_out[x] = rho;
                if (u_out)
                    for (int a = 0; a < 3; ++a) u_out[a * cells + x] = u[a];
            }

#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t x = cidx(i, j, k, nx, ny);
                for (int q = 0; q < Q; ++q) {
                    int ks = k - CV[q][2];
                    if (zbc == 0 && (ks < 0 || ks >= nz)) {
                        double v = fs[opp[q] * cells + x];
                        if (uwall) {
                            const double *uw = ks < 0 ? uwall : uwall + 2;
                            const double cu = CV[q][0] * uw[0] + CV[q][1] * uw[1];
                            v += 2.0 * WV[q] * rho_wall * cu * ICS2;
                        }
                        fnew[q * cells + x] = v;
                    } else {
                        size_t s = cidx(wrap1(i - CV[q][0], nx), wrap1(j - CV[q][1], ny),
                                        wrap1(ks, nz), nx, ny);
                        fnew[q * cells + x] = fs[q * cells + s];
                    }
                }
            }
}

/*
 * Inside / outside of closed droplet meshes (Sec. 2, below Eq. 13: fluid
 * nodes inside the droplet relax with tau_in, found by ray tracing).
 *
 * A cell (i, j, k) is inside when the vertical ray from its centre
 * (i + 1/2, j + 1/2, k + 1/2) down to z = -inf crosses the mesh an odd
 * number of times.  The decisions are exact: every coordinate is first put
 * on the integer grid Q(v) = round(v * 2^18) (half away from zero), so the
 * cell centre is (i * 2^18 + 2^17, ...), and all predicates are evaluated
 * in 128-bit integers.
 *   - The vertical line through p crosses triangle (a, b, c) when p lies in
 *     its xy projection.  Edge function e_uv(p) = (v_x - u_x)(p_y - u_y) -
 *     (v_y - u_y)(p_x - u_x); p is in the triangle when the three signs
 *     agree.  A zero is resolved as if p were moved by (eps, eps^2): its sign
 *     is that of -(v_y - u_y), or of (v_x - u_x) when v_y = u_y (simulation
 *     of simplicity), so that a point on an edge or vertex is counted by the
 *     same number of triangles, modulo 2, as a point next to it.  A triangle
 *     whose projection has no area is never crossed.
 *   - The crossing lies below the centre when z* <= z_c, with z* = N / D,
 *     D = e_ab + e_bc + e_ca, N = e_bc a_z + e_ca b_z + e_ab c_z
 *     (barycentric interpolation at p), decided as sign(D) (z_c D - N) >= 0.
 * x and y are periodic: the column is taken at the image of the cell centre
 * nearest to the triangle (droplets are smaller than half the box).
 * The parity runs over all triangles given, so several disjoint closed
 * meshes in one box may be passed together.
 */
typedef __int128 i128;
#define QSCALE 262144.0 /* 2^18 */

static inline int64_t qgrid(double v) { return (int64_t)llround(v * QSCALE); }

static inline int sos_sign(i128 e, int64_t dx, int64_t dy) {
    if (e > 0) return 1;
    if (e < 0) return -1;
    if (dy != 0) return dy > 0 ? -1 : 1; /* sign of -(v_y - u_y) */
    if (dx != 0) return dx > 0 ? 1 : -1;
    return 0;
}

static inline i128 edge_fn(int64_t ux, int64_t uy, int64_t vx, int64_t vy, int64_t px, int64_t py) {
    return (i128)(vx - ux) * (py - uy) - (i128)(vy - uy) * (px - ux);
}

void orc_inside(int nx, int ny, int nz, int n_tris, const int32_t *tris, const double *q,
                uint8_t *inside) {
    const size_t cells = (size_t)nx * ny * nz;
    memset(inside, 0, cells);
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            for (int t = 0; t < n_tris; ++t) {
                const double *A = q + 3 * (size_t)tris[3 * t], *B = q + 3 * (size_t)tris[3 * t + 1],
                             *C = q + 3 * (size_t)tris[3 * t + 2];
                /* image of the column nearest to the triangle */
                const double cx = (A[0] + B[0] + C[0]) / 3.0, cy = (A[1] + B[1] + C[1]) / 3.0;
                const double mx = floor((cx - (i + 0.5)) / nx + 0.5), my = floor((cy - (j + 0.5)) / ny + 0.5);
                const int64_t px = (int64_t)(i + (int64_t)mx * nx) * 262144 + 131072;
                const int64_t py = (int64_t)(j + (int64_t)my * ny) * 262144 + 131072;
                const int64_t ax = qgrid(A[0]), ay = qgrid(A[1]), az = qgrid(A[2]);
                const int64_t bx = qgrid(B[0]), by = qgrid(B[1]), bz = qgrid(B[2]);
                const int64_t kx = qgrid(C[0]), ky = qgrid(C[1]), kz = qgrid(C[2]);
                const i128 eab = edge_fn(ax, ay, bx, by, px, py);
                const i128 ebc = edge_fn(bx, by, kx, ky, px, py);
                const i128 eca = edge_fn(kx, ky, ax, ay, px, py);
                const int s1 = sos_sign(eab, bx - ax, by - ay);
                const int s2 = sos_sign(ebc, kx - bx, ky - by);
                const int s3 = sos_sign(eca, ax - kx, ay - ky);
                if (s1 == 0 || s1 != s2 || s2 != s3) continue;
                const i128 D = eab + ebc + eca;
                if (D == 0) continue;
                const i128 N = ebc * az + eca * bz + eab * kz;
                for (int k = 0; k < nz; ++k) {
                    const i128 zc = (i128)k * 262144 + 131072;
                    const i128 d = zc * D - N;
                    if ((D > 0 && d >= 0) || (D < 0 && d <= 0))
                        inside[cidx(i, j, k, nx, ny)] ^= 1;
                }
            }
}

/* Total mass sum_x sum_i f_i, pairwise over cells for a well-conditioned sum. */
static double pairwise(const double *v, size_t n) {
    if (n <= 64) {
        double s = 0.0;
        for (size_t i = 0; i < n; ++i) s += v[i];
        return s;
    }
    size_t h = n / 2;
    return pairwise(v, h) + pairwise(v + h, n - h);
}

double orc_mass(size_t cells, const double *f) {
    double *rho = (double *)malloc(cells * sizeof(double));
    for (size_t x = 0; x < cells; ++x) {
        double r = 0.0;
        for (int q = 0; q < Q; ++q) r += f[q * cells + x];
        rho[x] = r;
    }
    double m = pairwise(rho, cells);
    free(rho);
    return m;
}

/* Largest |sum_i c_i f_i| / rho over all cells (bare momentum velocity of the
 * state, without the force correction). */
double orc_max_u(size_t cells, const double *f) {
    double best = 0.0;
    for (size_t x = 0; x < cells; ++x) {
        double r = 0.0, m[3] = {0, 0, 0};
        for (int q = 0; q < Q; ++q) {
            r += f[q * cells + x];
            for (int a = 0; a < 3; ++a) m[a] += CV[q][a] * f[q * cells + x];
        }
        double v = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]) / r;
        if (v > best) best = v;
    }
    return best;
}

/*
 * Discrete delta (Eqs. 7-8).  The paper builds it "with interpolation
 * stencils" without naming one; the reading is Peskin's 4-point function
 *   phi(r) = (3 - 2r + sqrt(1 + 4r - 4r^2)) / 8      for |r| <= 1
 *          = (5 - 2r - sqrt(-7 + 12r - 4r^2)) / 8     for 1 <= |r| <= 2
 *          = 0                                        otherwise
 * and Delta(x) = phi(x) phi(y) phi(z) (dx = 1).
 */
double orc_peskin(double r) {
    r = fabs(r);
    if (r <= 1.0) return (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r)) / 8.0;
    if (r <= 2.0) return (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) / 8.0;
    return 0.0;
}

/*
 * Force spreading, Eq. 8: F(x) += phi_j Delta(q_j - x) for every node j in
 * ascending order.  Cell (i,j,k) is centred at (i+1/2, j+1/2, k+1/2).  The
 * candidate range per axis is deliberately wider than the support; cells
 * with |r| >= 2 get weight 0.  x and y indices wrap.  With walls, weight that
 * falls on a cell layer outside [0, nz) is not added to the fluid; it is
 * summed into to_wall[3] instead so that conservation can be checked.
 * F must be zeroed by the caller ([3][nz][ny][nx]).
 */
void orc_spread(int nx, int ny, int nz, int zbc, int n, const double *q,
                const double *phi, double *F, double *to_wall) {
    const size_t cells = (size_t)nx * ny * nz;
    for (int j = 0; j < n; ++j) {
        const double *p = q + 3 * j;
        int i0 = (int)floor(p[0]) - 3, j0 = (int)floor(p[1]) - 3, k0 = (int)floor(p[2]) - 3;
        for (int kk = k0; kk <= k0 + 6; ++kk) {
            double wz = orc_peskin(p[2] - (kk + 0.5));
            if (wz == 0.0) continue;
            for (int jj = j0; jj <= j0 + 6; ++jj) {
                double wy = orc_peskin(p[1] - (jj + 0.5));
                if (wy == 0.0) continue;
                for (int ii = i0; ii <= i0 + 6; ++ii) {
                    double wx = orc_peskin(p[0] - (ii + 0.5));
                    if (wx == 0.0) continue;
                    double w = wx * wy * wz;
                    int kz = kk;
                    if (zbc == 0 && (kz < 0 || kz >= nz)) {
                        if (to_wall)
                            for (int a = 0; a < 3; ++a) to_wall[a] += phi[3 * j + a] * w;
                        continue;
                    }
                    kz = wrap(kz, nz);
                    size_t x = cidx(wrap(ii, nx), wrap(jj, ny), kz, nx, ny);
                    for (int a = 0; a < 3; ++a) F[a * cells + x] += phi[3 * j + a] * w;
                }
            }
        }
    }
}

/*
 * Velocity interpolation, Eq. 7: U_j = sum_x u(x) Delta(q_j - x) (dx^3 = 1),
 * with the same kernel and cell centres as the spreading.  With walls, cells
 * outside [0, nz) are solid and carry u = 0.
 */
void orc_interp(int nx, int ny, int nz, int zbc, const double *u, int n,
                const double *q, double *U) {
    const size_t cells = (size_t)nx * ny * nz;
    for (int j = 0; j < n; ++j) {
        const double *p = q + 3 * j;
        double acc[3] = {0, 0, 0};
        int i0 = (int)floor(p[0]) - 3, j0 = (int)floor(p[1]) - 3, k0 = (int)floor(p[2]) - 3;
        for (int kk = k0; kk <= k0 + 6; ++kk) {
            double wz = orc_peskin(p[2] - (kk + 0.5));
            if (wz == 0.0) continue;
            if (zbc == 0 && (kk < 0 || kk >= nz)) continue;
            for (int jj = j0; jj <= j0 + 6; ++jj) {
                double wy = orc_peskin(p[1] - (jj + 0.5));
                if (wy == 0.0) continue;
                for (int ii = i0; ii <= i0 + 6; ++ii) {
                    double wx = orc_peskin(p[0] - (ii + 0.5));
                    if (wx == 0.0) continue;
                    size_t x = cidx(wrap(ii, nx), wrap(jj, ny), wrap(kk, nz), nx, ny);
                    double w = wx * wy * wz;
                    for (int a = 0; a < 3; ++a) acc[a] += u[a * cells + x] * w;
                }
            }
        }
        for (int a = 0; a < 3; ++a) U[3 * j + a] = acc[a];
    }
}

static void cross(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Triangle area A_t = |N|/2 and unit normal N/|N|, N = (q_b - q_a) x (q_c - q_a). */
void orc_triangle_geometry(int T, const int32_t *tri, const double *q, double *area,
                           double *normal) {
    for (int t = 0; t < T; ++t) {
        const double *a = q + 3 * tri[3 * t], *b = q + 3 * tri[3 * t + 1],
                     *c = q + 3 * tri[3 * t + 2];
        double e1[3], e2[3], N[3];
        for (int k = 0; k < 3; ++k) { e1[k] = b[k] - a[k]; e2[k] = c[k] - a[k]; }
        cross(e1, e2, N);
        double len = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        area[t] = 0.5 * len;
        for (int k = 0; k < 3; ++k) normal[3 * t + k] = N[k] / len;
    }
}

/* Enclosed volume of a closed outward mesh: sum_t q_a . (q_b x q_c) / 6. */
double orc_volume(int T, const int32_t *tri, const double *q) {
    double v = 0.0;
    for (int t = 0; t < T; ++t) {
        double bc[3];
        cross(q + 3 * tri[3 * t + 1], q + 3 * tri[3 * t + 2], bc);
        const double *a = q + 3 * tri[3 * t];
        v += (a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2]) / 6.0;
    }
    return v;
}

/*
 * Moments of the volume a closed mesh encloses, about the point ref:
 * out = {V, int x, int y, int z, int xx, int yy, int zz, int xy, int xz, int yz}.
 * The solid is the signed sum of the tetrahedra (ref, a, b, c) of its
 * triangles; over a tetrahedron with vertices p_0..p_3 (p_0 = ref = 0)
 *   int dV = v,  int x_i dV = v/4 sum_k p_ki,
 *   int x_i x_j dV = v/20 (sum_k p_ki p_kj + (sum_k p_ki)(sum_k p_kj)),
 * v = a . (b x c) / 6.  Used for the deformation index of Sec. 4 (semi-axes
 * of the ellipsoid with the same second moments).
 */
void orc_volume_moments(int T, const int32_t *tri, const double *q, const double *ref, double *out) {
    for (int k = 0; k < 10; ++k) out[k] = 0.0;
    static const int PI[6] = {0, 1, 2, 0, 0, 1}, PJ[6] = {0, 1, 2, 1, 2, 2};
    for (int t = 0; t < T; ++t) {
        double p[3][3];
        for (int c = 0; c < 3; ++c)
            for (int a = 0; a < 3; ++a) p[c][a] = q[3 * tri[3 * t + c] + a] - ref[a];
        double bc[3];
        cross(p[1], p[2], bc);
        const double v = (p[0][0] * bc[0] + p[0][1] * bc[1] + p[0][2] * bc[2]) / 6.0;
        double s[3];
        for (int a = 0; a < 3; ++a) s[a] = p[0][a] + p[1][a] + p[2][a];
        out[0] += v;
        for (int a = 0; a < 3; ++a) out[1 + a] += v * s[a] / 4.0;
        for (int m = 0; m < 6; ++m) {
            const int i = PI[m], j = PJ[m];
            double pp = 0.0;
            for (int c = 0; c < 3; ++c) pp += p[c][i] * p[c][j];
            out[4 + m] += v * (pp + s[i] * s[j]) / 20.0;
        }
    }
}

double orc_area(int T, const int32_t *tri, const double *q) {
    double s = 0.0;
    double *A = (double *)malloc(sizeof(double) * (size_t)T);
    double *n = (double *)malloc(sizeof(double) * 3 * (size_t)T);
    orc_triangle_geometry(T, tri, q, A, n);
    for (int t = 0; t < T; ++t) s += A[t];
    free(A);
    free(n);
    return s;
}

/* Eq. 11: A = sigma (m-1)(n-1) / ((n-m) xi) (1 + cos theta_eq). */
double orc_wetting_A(double sigma, double theta, double xi, int n, int m) {
    return sigma * (double)((m - 1) * (n - 1)) / ((double)(n - m) * xi) * (1.0 + cos(theta));
}

/* Eq. 10: Pi(d) = A [ (xi/d)^n - (xi/d)^m ]. */
double orc_pi(double d, double A, double xi, int n, int m) {
    return A * (pow(xi / d, n) - pow(xi / d, m));
}

/*
 * Nodal interface forces at positions q (Eqs. 9-11).
 *   phi_ST : surface tension.  The paper implements it as a finite-element
 *            strain energy of a clean interface of tension sigma; the energy
 *            taken is sigma * (total mesh area), so phi_ST,j = -sigma dA/dq_j.
 *            For triangle (a,b,c) with unit normal n the gradient of its area
 *            with respect to q_a is (1/2)(q_b - q_c) x n, cyclically.
 *   chi_j  : 1-ring area, sum of the areas of the triangles sharing node j.
 *   n_j    : average of the unit normals of those triangles, renormalised
 *            (plain average; the paper does not weight it).
 *   phi_Pi : -chi_j Pi(d_j) n_j / 3 with d_j = q_j,z, the height above the
 *            wall plane z = 0.
 *   phi_V  : optional volume penalty -k_V (V - V0)/V0 * dV/dq_j, used only
 *            when k_V > 0 (not part of the paper's model; off by default).
 * Outputs phi = phi_ST + phi_Pi + phi_V; the parts may be NULL.
 * Returns the number of nodes with d <= 0 (Pi undefined there).
 */
int orc_node_forces(int N, int T, const int32_t *tri, const double *q, double sigma,
                    double A, double xi, int n_exp, int m_exp, double k_vol, double V0,
                    double *phi, double *phi_st, double *phi_pi, double *phi_v,
                    double *chi_out, double *nhat_out) {
    double *area = (double *)malloc(sizeof(double) * (size_t)T);
    double *nt = (double *)malloc(sizeof(double) * 3 * (size_t)T);
    double *st = (double *)calloc(3 * (size_t)N, sizeof(double));
    double *gv = (double *)calloc(3 * (size_t)N, sizeof(double));
    double *chi = (double *)calloc((size_t)N, sizeof(double));
    double *ns = (double *)calloc(3 * (size_t)N, sizeof(double));
    orc_triangle_geometry(T, tri, q, area, nt);

    for (int t = 0; t < T; ++t) {
        for (int corner = 0; corner < 3; ++corner) {
            int j = tri[3 * t + corner];
            int nxt = tri[3 * t + (corner + 1) % 3];
            int prv = tri[3 * t + (corner + 2) % 3];
            double edge[3], f[3];
            for (int k = 0; k < 3; ++k) edge[k] = q[3 * prv + k] - q[3 * nxt + k];
            cross(edge, nt + 3 * t, f);
            for (int k = 0; k < 3; ++k) st[3 * j + k] += 0.5 * sigma * f[k];
            chi[j] += area[t];
            for (int k = 0; k < 3; ++k) ns[3 * j + k] += nt[3 * t + k];
            /* dV/dq_j of the triangle's cone: (q_next x q_prev)/6 */
            double g6[3];
            cross(q + 3 * nxt, q + 3 * prv, g6);
            for (int k = 0; k < 3; ++k) gv[3 * j + k] += g6[k] / 6.0;
        }
    }

    double V = k_vol > 0.0 ? orc_volume(T, tri, q) : V0;
    int bad = 0;
    for (int j = 0; j < N; ++j) {
        double len = sqrt(ns[3 * j] * ns[3 * j] + ns[3 * j + 1] * ns[3 * j + 1] +
                          ns[3 * j + 2] * ns[3 * j + 2]);
        double nh[3] = {ns[3 * j] / len, ns[3 * j + 1] / len, ns[3 * j + 2] / len};
        double d = q[3 * j + 2];
        if (d <= 0.0) ++bad;
        double Pi = orc_pi(d, A, xi, n_exp, m_exp);
        for (int k = 0; k < 3; ++k) {
            double fpi = -chi[j] * Pi * nh[k] / 3.0;
            double fv = k_vol > 0.0 ? -k_vol * (V - V0) / V0 * gv[3 * j + k] : 0.0;
            if (phi) phi[3 * j + k] = st[3 * j + k] + fpi + fv;
            if (phi_st) phi_st[3 * j + k] = st[3 * j + k];
            if (phi_pi) phi_pi[3 * j + k] = fpi;
            if (phi_v) phi_v[3 * j + k] = fv;
            if (nhat_out) nhat_out[3 * j + k] = nh[k];
        }
        if (chi_out) chi_out[j] = chi[j];
    }
    free(area); free(nt); free(st); free(gv); free(chi); free(ns);
    return bad;
}

/* Node -> incident triangles, each entry 3*t + corner, sorted by t. */
void orc_csr(int N, int T, const int32_t *tri, int32_t *offsets, int32_t *entries) {
    if (N <= 0) return;
    for (int j = 0; j <= N; ++j) offsets[j] = 0;
    for (int t = 0; t < T; ++t)
        for (int c = 0; c < 3; ++c) offsets[tri[3 * t + c] + 1] += 1;
    for (int j = 0; j < N; ++j) offsets[j + 1] += offsets[j];
    int32_t *fill = (int32_t *)calloc((size_t)N, sizeof(int32_t));
    for (int t = 0; t < T; ++t)
        for (int c = 0; c < 3; ++c) {
            int j = tri[3 * t + c];
            entries[offsets[j] + fill[j]++] = 3 * t + c;
        }
    free(fill);
}

/*
 * Integer binning of nodes.  The base cell along an axis is floor(q - 1/2):
 * the cell whose centre is the nearest one at or below q; the 4-point stencil
 * of the node is base-1 .. base+2.  Computed exactly as floor(q) when the
 * fractional part of q is at least 1/2 and floor(q) - 1 otherwise.  x and y
 * are wrapped into [0, n); z is kept as is.
 */
void orc_base_cells(int N, const double *q, int nx, int ny, int32_t *base) {
    for (int j = 0; j < N; ++j)
        for (int a = 0; a < 3; ++a) {
            double v = q[3 * j + a];
            double fl = floor(v);
            long b = (long)fl - ((v - fl) >= 0.5 ? 0 : 1);
            if (a == 0) b = wrap((int)b, nx);
            if (a == 1) b = wrap((int)b, ny);
            base[3 * j + a] = (int32_t)b;
        }
}

/*
 * Set flags[tile] = 1 for every tile (tile^3 cells, tile-major index
 * (tz*ty_n + ty)*tx_n + tx) that holds a stencil cell of any node; stencil
 * cells outside [0, nz) in z are skipped when the box has walls.
 */
void orc_touched_tiles(int N, const double *q, int nx, int ny, int nz, int zbc, int tx, int ty,
                       int tz, uint8_t *flags) {
    int tnx = (nx + tx - 1) / tx, tny = (ny + ty - 1) / ty;
    int32_t *b = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)N);
    orc_base_cells(N, q, nx, ny, b);
    for (int j = 0; j < N; ++j)
        for (int dz = -1; dz <= 2; ++dz) {
            int kz = b[3 * j + 2] + dz;
            if (zbc == 0 && (kz < 0 || kz >= nz)) continue;
            kz = wrap(kz, nz);
            for (int dy = -1; dy <= 2; ++dy)
                for (int dx = -1; dx <= 2; ++dx) {
                    int ix = wrap(b[3 * j] + dx, nx), iy = wrap(b[3 * j + 1] + dy, ny);
                    flags[((size_t)(kz / tz) * tny + iy / ty) * tnx + ix / tx] = 1;
                }
        }
    free(b);
}

/*
 * Mesh observables at positions q.
 * out[0] volume, out[1] area, out[2] z_min, out[3] z_max, out[4] height
 * h = z_max - z_min (the paper's height: highest minus lowest node),
 * out[5..7] area-weighted surface centroid, out[8] contact radius,
 * out[9] apparent angle 2 atan(h / r_c), out[10] number of edge crossings.
 * The contact radius is not defined in the paper; it is read here as the mean
 * horizontal distance from the centroid of the points where mesh edges cross
 * the plane z_c = z_min + xi (linear interpolation along each edge, every
 * undirected edge once, an edge crossing when exactly one end lies below z_c).
 */
void orc_mesh_observables(int N, int T, const int32_t *tri, const double *q, double xi,
                          double *out) {
    double *A = (double *)malloc(sizeof(double) * (size_t)T);
    double *nt = (double *)malloc(sizeof(double) * 3 * (size_t)T);
    orc_triangle_geometry(T, tri, q, A, nt);
    double area = 0.0, cen[3] = {0, 0, 0};
    for (int t = 0; t < T; ++t) {
        area += A[t];
        for (int k = 0; k < 3; ++k)
            cen[k] += A[t] * (q[3 * tri[3 * t] + k] + q[3 * tri[3 * t + 1] + k] +
                              q[3 * tri[3 * t + 2] + k]) / 3.0;
    }
    for (int k = 0; k < 3; ++k) cen[k] /= area;
    double zmin = q[2], zmax = q[2];
    for (int j = 1; j < N; ++j) {
        if (q[3 * j + 2] < zmin) zmin = q[3 * j + 2];
        if (q[3 * j + 2] > zmax) zmax = q[3 * j + 2];
    }
    double zc = zmin + xi, rsum = 0.0;
    int cnt = 0;
    for (int t = 0; t < T; ++t)
        for (int c = 0; c < 3; ++c) {
            int a = tri[3 * t + c], b = tri[3 * t + (c + 1) % 3];
            if (a > b) continue; /* each undirected edge once */
            const double *pa = q + 3 * a, *pb = q + 3 * b;
            int ba = pa[2] < zc, bb = pb[2] < zc;
            if (ba == bb) continue;
            double s = (zc - pa[2]) / (pb[2] - pa[2]);
            double px = pa[0] + s * (pb[0] - pa[0]) - cen[0];
            double py = pa[1] + s * (pb[1] - pa[1]) - cen[1];
            rsum += sqrt(px * px + py * py);
            ++cnt;
        }
    double rc = cnt ? rsum / cnt : 0.0;
    out[0] = orc_volume(T, tri, q);
    out[1] = area;
    out[2] = zmin;
    out[3] = zmax;
    out[4] = zmax - zmin;
    out[5] = cen[0]; out[6] = cen[1]; out[7] = cen[2];
    out[8] = rc;
    out[9] = rc > 0.0 ? 2.0 * atan((zmax - zmin) / rc) : 0.0;
    out[10] = cnt;
    free(A);
    free(nt);
}
