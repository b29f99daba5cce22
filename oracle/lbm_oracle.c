/*
 * lbm_oracle.c -- plain FP64 CPU oracle of the coupled lattice-Boltzmann /
 * immersed-boundary step of Wu, Xu, Kim & Alber, "Three-dimensional multiscale
 * model of deformable platelets adhesion to vessel wall in blood flow"
 * (arXiv:1312.2234).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the GPU
 * library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product path never does, and
 * it shares no source, header, table or helper with the GPU library.
 *
 * Every routine is the definition from the paper written out with loops, in
 * double precision, without blocking, fusion or reordering:
 *   - D3Q19 velocities, weights and numbering: Eq. (21) and the numbering implied
 *     by the on-site wall equations Eq. (23)-(30) (the velocity figure is absent),
 *   - density and momentum: Eq. (17)-(18); velocity shift v = u + F dt / 2 rho
 *     stated beneath Eq. (19),
 *   - equilibrium: Eq. (20); BGK collision Eq. (16); Guo forced update Eq. (19),
 *   - immersed-boundary spreading / interpolation: Eq. (33)-(36),
 *   - spring forces of the membrane network: Eq. (2)-(3),
 *   - per-step order: Fig. 1 (forces -> spread -> LBM -> interpolate -> move).
 *
 * Readings where the paper is silent, garbled or inconsistent (the design notes
 * list them with reasons):
 *   R1  Eq. (19) prints "+ c_s^2 I" in the second-order source term; the oracle
 *       uses "- c_s^2 I" (Guo et al. 2002), without which sum_i S_i != 0 and the
 *       scheme creates mass.
 *   R2  Both the equilibrium and the source use the shifted velocity v.
 *   R3  Eq. (36) prints the zero branch of phi as "|x| <= 2"; read as |x| >= 2.
 *   R4  Walls (walls = 1): halfway bounce-back with the moving-wall term
 *       6 w_i rho_w c_i.u_w (rho_w = 1) on planes y = -1/2 and y = ny - 1/2 (wall
 *       normal along y); x and z are periodic.
 *   R22 On-site walls (walls = 2): the velocity boundary of Eq. (23)-(30) on the
 *       rows y = 0 and y = ny - 1 themselves, turned from the paper's z-normal wall
 *       to a y-normal one.  With the Guo force the fluid velocity is
 *       (sum c f + F/2) / rho, so the momentum the rule imposes is rho v_w - F/2
 *       (the printed rule, which has no force, is the case F = 0); the wall node
 *       then moves exactly with the wall.
 *   R5  The interpolated velocity is v^{n+1} = (sum c f^{n+1} + (F_body + g^n)/2)
 *       / rho^{n+1}, the field after the LBM step (Fig. 1), taken at X^n; stencil
 *       rows inside a wall take that wall's velocity; spreading drops them.
 *   R6  Position update: explicit Euler, dt = 1.
 *   R7  Eq. (3) gives the force on node i as -k(|R|-L)R/|R| with R = X_j - X_i;
 *       as the negative gradient of Eq. (2) the force on i is +k(|R|-L)R/|R|
 *       (a stretched spring pulls its ends together).  The oracle follows the
 *       gradient of the energy.
 *   R8  Bending stand-in for the finite-element bending of Eq. (6)-(10): the
 *       dihedral energy E = k_b sum_hinges (1 - cos(theta - theta_0)).
 *   R23 Area and volume constraints, Eq. (4)-(5): Eq. (11) prints the force as
 *       +dH/dx; as for R7 the oracle takes F = -grad H.  Volumes by the divergence
 *       theorem over outward-oriented triangles; rest values from the rest shape.
 *
 * Units: lattice units, h = dt = rho_0 = 1.  Arrays are SoA, x fastest:
 * node index n = x + nx*(y + ny*z); populations f[i*N + n] in paper order
 * i = 1..19 stored at 0..18; vector fields v[d*N + n].
 *
 * Build: gcc -O2 -fopenmp -fPIC -shared -o liboracle.so lbm_oracle.c -lm
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* Eq. (21) weights and the D3Q19 set in the paper's numbering (1..19 -> 0..18).
 * The numbering is the one fixed by Eq. (23)-(30): c_z = 0 for 1,2,3,4,7,8,11,12,19;
 * c_z = -1 for 6,10,14,16,18; c_z = +1 for 5,9,13,15,17; opposite pairs from
 * Eq. (24)-(28); signs of c_x, c_y from Eq. (29)-(30). */
static const int CV[Q][3] = {
    {+1, 0, 0}, {-1, 0, 0}, {0, +1, 0}, {0, -1, 0}, {0, 0, +1}, {0, 0, -1},
    {+1, +1, 0}, {+1, -1, 0}, {+1, 0, +1}, {+1, 0, -1},
    {-1, +1, 0}, {-1, -1, 0}, {-1, 0, +1}, {-1, 0, -1},
    {0, +1, +1}, {0, +1, -1}, {0, -1, +1}, {0, -1, -1},
    {0, 0, 0}};
static const double WT[Q] = {
    2.0 / 36, 2.0 / 36, 2.0 / 36, 2.0 / 36, 2.0 / 36, 2.0 / 36,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
    12.0 / 36};
static const double CS2 = 1.0 / 3.0; /* c_s^2, text under Eq. (20) */

typedef struct {
    int32_t nx, ny, nz;
    int32_t walls;   /* 1: bounce-back walls normal to y; 2: on-site walls on rows 0 and
                        ny-1 (R22); 0: periodic in y too */
    double tau;
    double body[3];  /* constant body force, added to the IB force field */
    double uw_lo[3]; /* velocity of the lower wall (y = -1/2, or row 0 on-site) */
    double uw_hi[3]; /* velocity of the upper wall (y = ny - 1/2, or row ny-1 on-site) */
} orc_params;

/* threads an OpenMP region of the oracle uses (1 without OpenMP) */
int32_t orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* set the threads later OpenMP regions use (for timing only; results do not depend on it) */
void orc_set_threads(int32_t n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* accessors so that tests can check the tables against the paper */
void orc_tables(int32_t* c, double* w, int32_t* opp) {
    for (int i = 0; i < Q; ++i) {
        for (int d = 0; d < 3; ++d) c[3 * i + d] = CV[i][d];
        w[i] = WT[i];
        int o = -1;
        for (int j = 0; j < Q; ++j)
            if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] && CV[j][2] == -CV[i][2]) o = j;
        opp[i] = o;
    }
}

static int opposite(int i) {
    for (int j = 0; j < Q; ++j)
        if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] && CV[j][2] == -CV[i][2]) return j;
    return -1;
}

static int64_t wrap(int64_t a, int64_t n) { int64_t r = a % n; return r < 0 ? r + n : r; }

/* Eq. (20): f_i^eq(rho, v) = w_i rho [1 + c.v/cs2 + (c.v)^2/(2 cs2^2) - v.v/(2 cs2)] */
void orc_feq(double rho, const double* v, double* feq) {
    double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    for (int i = 0; i < Q; ++i) {
        double cv = CV[i][0] * v[0] + CV[i][1] * v[1] + CV[i][2] * v[2];
        feq[i] = WT[i] * rho * (1.0 + cv / CS2 + cv * cv / (2.0 * CS2 * CS2) - vv / (2.0 * CS2));
    }
}

/* Eq. (19) source term with dt = 1 and reading R1:
 * S_i = w_i (1 - 1/(2 tau)) [ (F.c_i)/cs2 + (v F^T + F v^T) : (c_i c_i^T - cs2 I) / (2 cs2^2) ] */
void orc_source(double tau, const double* v, const double* F, double* S) {
    for (int i = 0; i < Q; ++i) {
        double Fc = F[0] * CV[i][0] + F[1] * CV[i][1] + F[2] * CV[i][2];
        double contr = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double A = v[a] * F[b] + F[a] * v[b];
                double B = (double)CV[i][a] * CV[i][b] - (a == b ? CS2 : 0.0);
                contr += A * B;
            }
        S[i] = WT[i] * (1.0 - 1.0 / (2.0 * tau)) * (Fc / CS2 + contr / (2.0 * CS2 * CS2));
    }
}

/* Eq. (36) (reading R3) and the Peskin 4-point kernel (kernel = 1). */
double orc_phi(int32_t kernel, double r) {
    double a = fabs(r);
    if (kernel == 0) {
        if (a >= 2.0) return 0.0;
        return 0.25 * (1.0 + cos(M_PI * r / 2.0));
    }
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
}

/* f = f^eq(rho, u) at every node; rho == NULL means 1, u == NULL means 0. */
void orc_init(const orc_params* p, double* f, const double* rho, const double* u) {
    int64_t N = (int64_t)p->nx * p->ny * p->nz;
    for (int64_t n = 0; n < N; ++n) {
        double r = rho ? rho[n] : 1.0;
        double v[3] = {u ? u[n] : 0.0, u ? u[N + n] : 0.0, u ? u[2 * N + n] : 0.0};
        double feq[Q];
        orc_feq(r, v, feq);
        for (int i = 0; i < Q; ++i) f[i * N + n] = feq[i];
    }
}

/* The 19 populations of node n (row y) as the step sees them.  With on-site walls
 * (walls = 2, reading R22) the populations entering the fluid at a wall row have no
 * source node; Hecht and Harting's rule, Eq. (23)-(30), sets them from the others.
 * The paper writes it for the wall z = 0; here the wall normal is y, the inward
 * normal is n = +e_y on row 0 and -e_y on row ny-1, and x, z are the transverse
 * directions t.  With F the force at the node and J = rho v_w - F/2 (R22):
 *   Eq. (23)       rho (1 - n.v_w) = sum_{c.n=0} f + 2 sum_{c.n=-1} f - n.F/2
 *   Eq. (29)-(30)  N_t = 1/2 sum_{c.n=0} c_t f - J_t / 3
 *   Eq. (24)       f_i = f_opp(i) + n.J / 3                       (c_i = n)
 *   Eq. (25)-(28)  f_i = f_opp(i) + (n.J + c_it J_t) / 6 - c_it N_t  (c_i = n + c_it e_t)
 * Every other node, and every population with c.n <= 0, is returned as stored. */
static void node_populations(const orc_params* p, const double* f, const double* g, int64_t n, int64_t y,
                             double fn[Q]) {
    int64_t N = (int64_t)p->nx * p->ny * p->nz;
    for (int i = 0; i < Q; ++i) fn[i] = f[i * N + n];
    if (p->walls != 2 || (y != 0 && y != p->ny - 1)) return;
    int s = y == 0 ? 1 : -1; /* n = s e_y */
    const double* vw = y == 0 ? p->uw_lo : p->uw_hi;
    double F[3];
    for (int d = 0; d < 3; ++d) F[d] = p->body[d] + (g ? g[d * N + n] : 0.0);
    double par = 0.0, out = 0.0;
    for (int i = 0; i < Q; ++i) {
        int cn = s * CV[i][1];
        if (cn == 0) par += fn[i];
        if (cn == -1) out += fn[i];
    }
    double rho = (par + 2.0 * out - 0.5 * s * F[1]) / (1.0 - s * vw[1]); /* Eq. (23) */
    double J[3];
    for (int d = 0; d < 3; ++d) J[d] = rho * vw[d] - 0.5 * F[d];
    double Nt[3] = {0.0, 0.0, 0.0}; /* Eq. (29)-(30); Nt[1] unused */
    for (int t = 0; t < 3; t += 2) {
        double m = 0.0;
        for (int i = 0; i < Q; ++i)
            if (CV[i][1] == 0) m += CV[i][t] * fn[i];
        Nt[t] = 0.5 * m - J[t] / 3.0;
    }
    double nJ = s * J[1];
    for (int i = 0; i < Q; ++i) {
        if (s * CV[i][1] != 1) continue;
        int o = opposite(i);
        int t = CV[i][0] != 0 ? 0 : (CV[i][2] != 0 ? 2 : -1);
        if (t < 0)
            fn[i] = fn[o] + nJ / 3.0;                                            /* Eq. (24) */
        else
            fn[i] = fn[o] + (nJ + CV[i][t] * J[t]) / 6.0 - CV[i][t] * Nt[t];     /* Eq. (25)-(28) */
    }
}

/* The populations of every node as the next step sees them (node_populations):
 * a copy of f, with the on-site wall rule applied at the wall rows when walls = 2. */
void orc_complete(const orc_params* p, const double* f, const double* g, double* fc) {
    int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double fn[Q];
        node_populations(p, f, g, n, (n / nx) % ny, fn);
        for (int i = 0; i < Q; ++i) fc[i * N + n] = fn[i];
    }
}

/* Eq. (17)-(18) and the shift under Eq. (19):
 * rho = sum f, v = (sum c f + F/2) / rho with F = F_body + g(x). */
void orc_moments(const orc_params* p, const double* f, const double* g, double* rho, double* v) {
    int64_t N = (int64_t)p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double r = 0.0, j[3] = {0, 0, 0}, fn[Q];
        node_populations(p, f, g, n, (n / p->nx) % p->ny, fn);
        for (int i = 0; i < Q; ++i) {
            r += fn[i];
            for (int d = 0; d < 3; ++d) j[d] += CV[i][d] * fn[i];
        }
        rho[n] = r;
        for (int d = 0; d < 3; ++d) {
            double F = p->body[d] + (g ? g[d * N + n] : 0.0);
            v[d * N + n] = (j[d] + 0.5 * F) / r;
        }
    }
}

/* Collision of one LBM time step, Eq. (16), (19), (20):
 * f*_i(x) = f_i - (f_i - f_i^eq(rho, v))/tau + S_i(v, F) at every node. */
void orc_collide(const orc_params* p, const double* f, const double* g, double* fs) {
    int64_t N = (int64_t)p->nx * p->ny * p->nz;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double r = 0.0, j[3] = {0, 0, 0}, F[3], v[3], feq[Q], S[Q], fn[Q];
        node_populations(p, f, g, n, (n / p->nx) % p->ny, fn);
        for (int i = 0; i < Q; ++i) {
            r += fn[i];
            for (int d = 0; d < 3; ++d) j[d] += CV[i][d] * fn[i];
        }
        for (int d = 0; d < 3; ++d) {
            F[d] = p->body[d] + (g ? g[d * N + n] : 0.0);
            v[d] = (j[d] + 0.5 * F[d]) / r;
        }
        orc_feq(r, v, feq);
        orc_source(p->tau, v, F, S);
        for (int i = 0; i < Q; ++i)
            fs[i * N + n] = fn[i] - (fn[i] - feq[i]) / p->tau + S[i];
    }
}

/* Streaming of one LBM time step (reading R4 at walls):
 * f_i(x, t+1) = f*_i(x - c_i); across a wall f_i(x, t+1) = f*_{opp(i)}(x) + 6 w_i rho_w c_i.u_w.
 * On-site walls (R22): a population entering through the wall has no source and is
 * stored as 0; node_populations sets it when the state is read. */
void orc_stream(const orc_params* p, const double* fs, double* fout) {
    int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t n = x + nx * (y + ny * z);
                for (int i = 0; i < Q; ++i) {
                    int64_t ys = y - CV[i][1];
                    if (p->walls == 2 && (ys < 0 || ys >= ny)) {
                        fout[i * N + n] = 0.0;
                    } else if (p->walls && (ys < 0 || ys >= ny)) {
                        const double* uw = ys < 0 ? p->uw_lo : p->uw_hi;
                        double cu = CV[i][0] * uw[0] + CV[i][1] * uw[1] + CV[i][2] * uw[2];
                        fout[i * N + n] = fs[opposite(i) * N + n] + 6.0 * WT[i] * 1.0 * cu;
                    } else {
                        int64_t xs = wrap(x - CV[i][0], nx);
                        int64_t zs = wrap(z - CV[i][2], nz);
                        ys = wrap(ys, ny);
                        fout[i * N + n] = fs[i * N + xs + nx * (ys + ny * zs)];
                    }
                }
            }
}

/* Inverse of orc_stream: every post-collision value reaches exactly one pre-collision
 * slot of the next step (a permutation plus the constant wall term), so
 * f*_i(x - c_i) = f_i(x, t+1), and across a wall f*_{opp(i)}(x) = f_i(x, t+1) - 6 w_i c_i.u_w. */
void orc_unstream(const orc_params* p, const double* f, double* fs) {
    int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t n = x + nx * (y + ny * z);
                for (int i = 0; i < Q; ++i) {
                    int64_t ys = y - CV[i][1];
                    if (p->walls == 2 && (ys < 0 || ys >= ny)) {
                        fs[opposite(i) * N + n] = 0.0; /* leaves through the wall: not used */
                    } else if (p->walls && (ys < 0 || ys >= ny)) {
                        const double* uw = ys < 0 ? p->uw_lo : p->uw_hi;
                        double cu = CV[i][0] * uw[0] + CV[i][1] * uw[1] + CV[i][2] * uw[2];
                        fs[opposite(i) * N + n] = f[i * N + n] - 6.0 * WT[i] * 1.0 * cu;
                    } else {
                        int64_t xs = wrap(x - CV[i][0], nx);
                        int64_t zs = wrap(z - CV[i][2], nz);
                        ys = wrap(ys, ny);
                        fs[i * N + xs + nx * (ys + ny * zs)] = f[i * N + n];
                    }
                }
            }
}

/* One LBM time step, Eq. (16), (19), (20), (reading R4 at walls): collide, then stream. */
void orc_step(const orc_params* p, const double* f, const double* g, double* fout) {
    int64_t N = (int64_t)p->nx * p->ny * p->nz;
    double* fs = (double*)malloc(sizeof(double) * Q * N);
    orc_collide(p, f, g, fs);
    orc_stream(p, fs, fout);
    free(fs);
}

/* Eq. (34)-(35) with h = 1: g(x) = sum_m F_m phi(x-X_mx) phi(y-X_my) phi(z-X_mz)
 * over the 4x4x4 stencil floor(X)-1 .. floor(X)+2; x, z periodic; rows outside
 * [0, ny) are dropped when walls are present (reading R5), wrapped otherwise. */
void orc_spread(const orc_params* p, int32_t kernel, int64_t nn, const double* X, const double* Fm,
                double* g) {
    int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
    memset(g, 0, sizeof(double) * 3 * N);
    for (int64_t m = 0; m < nn; ++m) {
        double Xm[3] = {X[m], X[nn + m], X[2 * nn + m]};
        int64_t b[3];
        for (int d = 0; d < 3; ++d) b[d] = (int64_t)floor(Xm[d]) - 1;
        for (int c = 0; c < 4; ++c)
            for (int bb = 0; bb < 4; ++bb)
                for (int a = 0; a < 4; ++a) {
                    int64_t xi = b[0] + a, yi = b[1] + bb, zi = b[2] + c;
                    double w = orc_phi(kernel, (double)xi - Xm[0]) * orc_phi(kernel, (double)yi - Xm[1]) *
                               orc_phi(kernel, (double)zi - Xm[2]);
                    if (p->walls && (yi < 0 || yi >= ny)) continue;
                    int64_t n = wrap(xi, nx) + nx * (wrap(yi, ny) + ny * wrap(zi, nz));
                    for (int d = 0; d < 3; ++d) g[d * N + n] += Fm[d * nn + m] * w;
                }
    }
}

/* Eq. (33) with h = 1: U_m = sum_x v(x) phi phi phi over the same stencil;
 * stencil rows inside a wall contribute that wall's velocity (reading R5). */
void orc_interp(const orc_params* p, int32_t kernel, int64_t nn, const double* X, const double* v,
                double* U) {
    int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < nn; ++m) {
        double Xm[3] = {X[m], X[nn + m], X[2 * nn + m]};
        int64_t b[3];
        for (int d = 0; d < 3; ++d) b[d] = (int64_t)floor(Xm[d]) - 1;
        double acc[3] = {0, 0, 0};
        for (int c = 0; c < 4; ++c)
            for (int bb = 0; bb < 4; ++bb)
                for (int a = 0; a < 4; ++a) {
                    int64_t xi = b[0] + a, yi = b[1] + bb, zi = b[2] + c;
                    double w = orc_phi(kernel, (double)xi - Xm[0]) * orc_phi(kernel, (double)yi - Xm[1]) *
                               orc_phi(kernel, (double)zi - Xm[2]);
                    if (p->walls && (yi < 0 || yi >= ny)) {
                        const double* uw = yi < 0 ? p->uw_lo : p->uw_hi;
                        for (int d = 0; d < 3; ++d) acc[d] += uw[d] * w;
                    } else {
                        int64_t n = wrap(xi, nx) + nx * (wrap(yi, ny) + ny * wrap(zi, nz));
                        for (int d = 0; d < 3; ++d) acc[d] += v[d * N + n] * w;
                    }
                }
        for (int d = 0; d < 3; ++d) U[d * nn + m] = acc[d];
    }
}

/* Reading R6: X <- X + U (dt = 1). */
void orc_advance(int64_t nn, double* X, const double* U) {
    for (int64_t k = 0; k < 3 * nn; ++k) X[k] += U[k];
}

/* Viscous shear stress at the two wall-adjacent rows, y = 0 and y = ny-1:
 * sigma_ab = -(1 - 1/(2 tau)) sum_i c_ia c_ib (f_i - f_i^eq(rho, v))
 *            - (1 - 1/(2 tau)) (F_a v_b + F_b v_a) / 2,
 * the stress of the Guo-forced BGK scheme (the paper gives no formula).
 * Output per row: [2][nz][nx] = sigma_xy, sigma_zy. */
void orc_wall_stress(const orc_params* p, const double* f, const double* g, double* lo, double* hi) {
    int64_t nx = p->nx, ny = p->ny, nz = p->nz, N = nx * ny * nz;
    double k = 1.0 - 1.0 / (2.0 * p->tau);
    for (int side = 0; side < 2; ++side) {
        int64_t y = side == 0 ? 0 : ny - 1;
        double* out = side == 0 ? lo : hi;
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t n = x + nx * (y + ny * z);
                double r = 0.0, j[3] = {0, 0, 0}, F[3], v[3], feq[Q], fn[Q];
                node_populations(p, f, g, n, y, fn);
                for (int i = 0; i < Q; ++i) {
                    r += fn[i];
                    for (int d = 0; d < 3; ++d) j[d] += CV[i][d] * fn[i];
                }
                for (int d = 0; d < 3; ++d) {
                    F[d] = p->body[d] + (g ? g[d * N + n] : 0.0);
                    v[d] = (j[d] + 0.5 * F[d]) / r;
                }
                orc_feq(r, v, feq);
                const int comps[2] = {0, 2};
                for (int q = 0; q < 2; ++q) {
                    int a = comps[q], b = 1;
                    double s = 0.0;
                    for (int i = 0; i < Q; ++i) s += (double)CV[i][a] * CV[i][b] * (fn[i] - feq[i]);
                    out[q * nz * nx + z * nx + x] = -k * s - k * 0.5 * (F[a] * v[b] + F[b] * v[a]);
                }
            }
    }
}

/* ---------------------------------------------------------------- membrane forces
 * Inputs of the coupled step (Fig. 1, first box); X, anchors: [3][n].
 *  springs  Eq. (2)-(3) (reading R7): edges (i,j), rest length L = |X_j - X_i| of the
 *           rest shape, U = k/2 (|R| - L)^2, force on i = +k (|R| - L) R/|R|;
 *  tethers  U = k_t/2 |X - A|^2, force = -k_t (X - A);
 *  bending  (reading R8) hinges (x0, x1, x2, x3): shared edge x1-x2, triangles
 *           (x0,x1,x2) and (x3,x2,x1); E = k_b (1 - cos(theta - theta0)). */
static void sub3(const double* a, const double* b, double* o) { for (int d = 0; d < 3; ++d) o[d] = a[d] - b[d]; }
static void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void getp(const double* X, int64_t nn, int64_t i, double* o) { for (int d = 0; d < 3; ++d) o[d] = X[d * nn + i]; }

/* signed dihedral angle: atan2((nA^ x nB^).e^, nA^.nB^), nA = (x1-x0)x(x2-x0), nB = (x2-x3)x(x1-x3) */
static double hinge_angle(const double* x0, const double* x1, const double* x2, const double* x3) {
    double a[3], b[3], nA[3], nB[3], e[3], c[3];
    sub3(x1, x0, a); sub3(x2, x0, b); cross3(a, b, nA);
    sub3(x2, x3, a); sub3(x1, x3, b); cross3(a, b, nB);
    sub3(x2, x1, e);
    double la = sqrt(dot3(nA, nA)), lb = sqrt(dot3(nB, nB)), le = sqrt(dot3(e, e));
    cross3(nA, nB, c);
    return atan2(dot3(c, e) / (la * lb * le), dot3(nA, nB) / (la * lb));
}

void orc_hinge_angles(int64_t nn, const double* X, int64_t nh, const int32_t* hinges, double* theta) {
    for (int64_t h = 0; h < nh; ++h) {
        double x[4][3];
        for (int k = 0; k < 4; ++k) getp(X, nn, hinges[4 * h + k], x[k]);
        theta[h] = hinge_angle(x[0], x[1], x[2], x[3]);
    }
}

void orc_edge_lengths(int64_t nn, const double* X, int64_t ne, const int32_t* edges, double* len) {
    for (int64_t e = 0; e < ne; ++e) {
        double a[3], b[3], r[3];
        getp(X, nn, edges[2 * e], a); getp(X, nn, edges[2 * e + 1], b); sub3(b, a, r);
        len[e] = sqrt(dot3(r, r));
    }
}

/* Total membrane energy (for finite-difference checks of the forces). */
double orc_membrane_energy(int64_t nn, const double* X, int64_t ne, const int32_t* edges,
                           const double* rest_len, double k_spring, int64_t nh, const int32_t* hinges,
                           const double* rest_theta, double k_bend, const double* anchors, double k_tether) {
    double E = 0.0;
    for (int64_t e = 0; e < ne; ++e) {
        double a[3], b[3], r[3];
        getp(X, nn, edges[2 * e], a); getp(X, nn, edges[2 * e + 1], b); sub3(b, a, r);
        double s = sqrt(dot3(r, r)) - rest_len[e];
        E += 0.5 * k_spring * s * s;
    }
    for (int64_t h = 0; h < nh; ++h) {
        double x[4][3];
        for (int k = 0; k < 4; ++k) getp(X, nn, hinges[4 * h + k], x[k]);
        E += k_bend * (1.0 - cos(hinge_angle(x[0], x[1], x[2], x[3]) - rest_theta[h]));
    }
    if (anchors)
        for (int64_t i = 0; i < nn; ++i)
            for (int d = 0; d < 3; ++d) {
                double s = X[d * nn + i] - anchors[d * nn + i];
                E += 0.5 * k_tether * s * s;
            }
    return E;
}

/* F = -grad(E) of the energy above, written out term by term. */
void orc_membrane_forces(int64_t nn, const double* X, int64_t ne, const int32_t* edges,
                         const double* rest_len, double k_spring, int64_t nh, const int32_t* hinges,
                         const double* rest_theta, double k_bend, const double* anchors, double k_tether,
                         double* F) {
    memset(F, 0, sizeof(double) * 3 * nn);
    for (int64_t e = 0; e < ne; ++e) {
        int64_t i = edges[2 * e], j = edges[2 * e + 1];
        double a[3], b[3], r[3];
        getp(X, nn, i, a); getp(X, nn, j, b); sub3(b, a, r);
        double len = sqrt(dot3(r, r));
        double s = k_spring * (len - rest_len[e]) / len;
        for (int d = 0; d < 3; ++d) {
            F[d * nn + i] += s * r[d];
            F[d * nn + j] -= s * r[d];
        }
    }
    for (int64_t h = 0; h < nh; ++h) {
        int64_t id[4];
        double x[4][3];
        for (int k = 0; k < 4; ++k) { id[k] = hinges[4 * h + k]; getp(X, nn, id[k], x[k]); }
        double theta = hinge_angle(x[0], x[1], x[2], x[3]);
        double dEdth = k_bend * sin(theta - rest_theta[h]);
        /* gradient of theta with respect to the four vertices */
        double a[3], b[3], nA[3], nB[3], e[3];
        sub3(x[1], x[0], a); sub3(x[2], x[0], b); cross3(a, b, nA);
        sub3(x[2], x[3], a); sub3(x[1], x[3], b); cross3(a, b, nB);
        sub3(x[2], x[1], e);
        double L = sqrt(dot3(e, e)), AA = dot3(nA, nA), BB = dot3(nB, nB);
        double qA[3], qB[3];
        for (int d = 0; d < 3; ++d) { qA[d] = nA[d] / AA; qB[d] = nB[d] / BB; }
        double t02[3], t32[3], t01[3], t31[3];
        sub3(x[0], x[2], t02); sub3(x[3], x[2], t32); sub3(x[0], x[1], t01); sub3(x[3], x[1], t31);
        double c02 = dot3(t02, e) / L, c32 = dot3(t32, e) / L, c01 = dot3(t01, e) / L, c31 = dot3(t31, e) / L;
        for (int d = 0; d < 3; ++d) {
            double g0 = -L * qA[d];
            double g3 = -L * qB[d];
            double g1 = -c02 * qA[d] - c32 * qB[d];
            double g2 = c01 * qA[d] + c31 * qB[d];
            F[d * nn + id[0]] -= dEdth * g0;
            F[d * nn + id[1]] -= dEdth * g1;
            F[d * nn + id[2]] -= dEdth * g2;
            F[d * nn + id[3]] -= dEdth * g3;
        }
    }
    if (anchors)
        for (int64_t i = 0; i < nn; ++i)
            for (int d = 0; d < 3; ++d) F[d * nn + i] -= k_tether * (X[d * nn + i] - anchors[d * nn + i]);
}

/* ---------------------------------------------------------------- area and volume constraints
 * Eq. (4)-(5) (reading R23: the force is -grad H, as for the springs under R7).  Triangles
 * (a, b, c) with the outward normal n = (b - a) x (c - a) (right-hand rule); a body's
 * triangles are contiguous, body_tri[b] .. body_tri[b+1].
 *   triangle area   S_t = |n| / 2
 *   body area       S^total = sum over the body's triangles of S_t
 *   body volume     V = sum over the body's triangles of a.(b x c) / 6   (divergence theorem)
 *   H = sum_bodies [ k_s (S^total - S_0^total)^2 / (2 S_0^total) + k_v (V - V_0)^2 / (2 V_0) ]
 *       + sum_triangles k_t (S_t - S_0,t)^2 / (2 S_0,t)
 * with the rest values measured on the rest shape (orc_triangle_rest). */
static double tri_area(const double* a, const double* b, const double* c, double n[3]) {
    double u[3], v[3];
    sub3(b, a, u); sub3(c, a, v); cross3(u, v, n);
    return 0.5 * sqrt(dot3(n, n));
}

static double tri_volume6(const double* a, const double* b, const double* c) {
    double bc[3];
    cross3(b, c, bc);
    return dot3(a, bc);
}

/* body[2b] = S^total, body[2b+1] = V of each body for the shape X; area[t] = S_t (may be NULL) */
static void body_measures(int64_t nn, const double* X, const int32_t* tri, int64_t nb, const int32_t* body_tri,
                          double* area, double* body) {
    for (int64_t b = 0; b < nb; ++b) {
        double S = 0.0, V6 = 0.0;
        for (int64_t t = body_tri[b]; t < body_tri[b + 1]; ++t) {
            double p[3][3], n[3];
            for (int k = 0; k < 3; ++k) getp(X, nn, tri[3 * t + k], p[k]);
            double s = tri_area(p[0], p[1], p[2], n);
            if (area) area[t] = s;
            S += s;
            V6 += tri_volume6(p[0], p[1], p[2]);
        }
        body[2 * b] = S;
        body[2 * b + 1] = V6 / 6.0;
    }
}

/* Rest values of Eq. (4)-(5) on the rest shape: S_0 per triangle, (S_0^total, V_0) per body. */
void orc_triangle_rest(int64_t nn, const double* X_rest, const int32_t* tri, int64_t nb, const int32_t* body_tri,
                       double* area0, double* body0) {
    body_measures(nn, X_rest, tri, nb, body_tri, area0, body0);
}

double orc_constraint_energy(int64_t nn, const double* X, const int32_t* tri, int64_t nb, const int32_t* body_tri,
                             const double* area0, const double* body0, double k_s, double k_t, double k_v) {
    int64_t nt = body_tri[nb];
    double* area = (double*)malloc(sizeof(double) * (nt > 0 ? nt : 1));
    double* body = (double*)malloc(sizeof(double) * 2 * (nb > 0 ? nb : 1));
    body_measures(nn, X, tri, nb, body_tri, area, body);
    double H = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
        double dS = body[2 * b] - body0[2 * b], dV = body[2 * b + 1] - body0[2 * b + 1];
        H += k_s * dS * dS / (2.0 * body0[2 * b]) + k_v * dV * dV / (2.0 * body0[2 * b + 1]);
    }
    for (int64_t t = 0; t < nt; ++t) {
        double d = area[t] - area0[t];
        H += k_t * d * d / (2.0 * area0[t]);
    }
    free(area);
    free(body);
    return H;
}

/* F = -grad H of orc_constraint_energy, [3][nn] (overwritten).  Per triangle (a, b, c):
 *   dS_t/da = (1/2) n_hat x (c - b),  dS_t/db = (1/2) n_hat x (a - c),  dS_t/dc = (1/2) n_hat x (b - a)
 *   dV/da = (b x c)/6,  dV/db = (c x a)/6,  dV/dc = (a x b)/6
 * and dH/dx = [k_s (S^total - S_0^total)/S_0^total + k_t (S_t - S_0,t)/S_0,t] dS_t/dx
 *            + k_v (V - V_0)/V_0 dV/dx, summed over the triangles at the node. */
void orc_constraint_forces(int64_t nn, const double* X, const int32_t* tri, int64_t nb, const int32_t* body_tri,
                           const double* area0, const double* body0, double k_s, double k_t, double k_v, double* F) {
    memset(F, 0, sizeof(double) * 3 * nn);
    double* body = (double*)malloc(sizeof(double) * 2 * (nb > 0 ? nb : 1));
    body_measures(nn, X, tri, nb, body_tri, NULL, body);
    for (int64_t b = 0; b < nb; ++b) {
        double cs = k_s * (body[2 * b] - body0[2 * b]) / body0[2 * b];
        double cv = k_v * (body[2 * b + 1] - body0[2 * b + 1]) / body0[2 * b + 1];
        for (int64_t t = body_tri[b]; t < body_tri[b + 1]; ++t) {
            int64_t id[3];
            double p[3][3], n[3];
            for (int k = 0; k < 3; ++k) { id[k] = tri[3 * t + k]; getp(X, nn, id[k], p[k]); }
            double S = tri_area(p[0], p[1], p[2], n);
            double ct = k_t * (S - area0[t]) / area0[t];
            double nl = 2.0 * S; /* |n| */
            double nh[3] = {n[0] / nl, n[1] / nl, n[2] / nl};
            for (int k = 0; k < 3; ++k) {
                const double* pb = p[(k + 1) % 3];
                const double* pc = p[(k + 2) % 3];
                double e[3], dS[3], dV[3];
                sub3(pc, pb, e);
                cross3(nh, e, dS);
                cross3(pb, pc, dV);
                for (int d = 0; d < 3; ++d)
                    F[d * nn + id[k]] -= (cs + ct) * 0.5 * dS[d] + cv * dV[d] / 6.0;
            }
        }
    }
    free(body);
}
