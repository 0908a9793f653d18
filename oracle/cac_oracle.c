/*
 * cac_oracle.c -- plain FP64 CPU oracle for one coupled time step of the
 * conservative Allen-Cahn (CAC) lattice Boltzmann method with geometric
 * ghost-node wetting and global phase-field volume correction
 * (Bello, Mander, Lauricella, Guglielmo, La Rocca, Montessori,
 *  "Accurate wetting dynamics via a conservative Allen-Cahn based lattice
 *  Boltzmann approach for multiphase flows", Sec. II).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU path is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, table or header with the GPU library.
 *
 * Style: per-node loops in the paper's order and notation, full Hermite
 * tensors contracted index by index, double precision throughout.  No
 * blocking, fusion or reordering beyond what the equations state.
 *
 * Time step (the paper fixes wetting -> CAC advance -> volume correction,
 * Sec. II C; it is silent on where the LB update sits; the reading used
 * here is W -> H -> P -> V, all explicit at time level n):
 *   W  ghost update at boundary solid nodes (Sec. II B, Eqs. (36)-(47)),
 *      Jacobi: donor gradients read the previous ghosts;
 *   H  hydrodynamic collide + stream (Sec. II A, Eqs. (3)-(23)); the
 *      non-equilibrium moment A2 of Eq. (14) is either the local second
 *      moment of the node's populations (collision = 0) or the gradient form
 *      of Eq. (15) from the velocity field (collision = 1);
 *   P  CAC finite-difference update (Sec. II A 1, Eqs. (24)-(35));
 *   V  global volume correction (Sec. II C, Eqs. (48)-(55)).
 *
 * Lattice: D3Q27, canonical order below, c_s^2 = 1/3, dx = dt = 1.
 * Index n = x + nx*(y + ny*z); periodic index wrap in all directions;
 * solid walls are voxel layers given by the mask.
 *
 * Storage conventions of the oracle state:
 *   f[i*N+n]  post-streaming (pre-collision) populations f^n_i on fluid nodes
 *   phi[n]    phi^n on fluid nodes, previous ghost g^{n-1} on wall nodes
 *   u[d*N+n], pstar[n]  macroscopic fields of the last collision
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 27

typedef struct {
    double rho_l, rho_g, nu_l, nu_g; /* Eqs. (8)-(10) */
    double sigma, delta;             /* surface tension, interface width (text after Eq. (19)) */
    double D;                        /* CAC interface diffusivity, Eq. (24); kappa = 4D/delta, Eq. (26) */
    double g[3];                     /* body acceleration: F_ext = (rho - rho_g) g */
    double eps_phi;                  /* interface band threshold of Eq. (51) */
    double eps_n;                    /* normal guard: n = 0 when |grad phi| <= eps_n */
    double sin_tol, cot_max;         /* cot regularisation, text after Eq. (45) */
    int volume_correction;           /* 1: apply Eq. (53) every step */
    int wall_compression;            /* compressive flux a at wall nodes: 0 -> a = 0,
                                      * 1 -> a = g (1 - g) grad(phi)_c / |grad(phi)_c| */
    int collision;                   /* non-equilibrium moment A2 of Eq. (14): 0 -> local second
                                      * moment of the pre-collision populations; 1 -> gradient
                                      * form of Eq. (15) from the velocity field */
    int ghost_localization;          /* factor of the ghost extrapolation, Eq. (46): 1 -> lambda_s of
                                      * Eq. (47); 0 -> 1 (diagnostic reading of the angle study) */
} orc_params;

/* ------------------------------------------------------------------ */
/* D3Q27 lattice (Sec. II A: "D3Q27", lattice weights of the textbook set) */

static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

static const double CS2 = 1.0 / 3.0;

static int norm2(int i) { return CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2]; }

static double weight_of(int i)
{
    switch (norm2(i)) {
    case 0: return 8.0 / 27.0;
    case 1: return 2.0 / 27.0;
    case 2: return 1.0 / 54.0;
    default: return 1.0 / 216.0;
    }
}

static int opposite_of(int i)
{
    for (int k = 0; k < Q; ++k)
        if (CV[k][0] == -CV[i][0] && CV[k][1] == -CV[i][1] && CV[k][2] == -CV[i][2]) return k;
    return -1;
}

/* Tables filled once from the definitions above and below. */
static double W_TAB[Q];
static int OPP_TAB[Q];
static double H2_TAB[Q][3][3];
static double H3_TAB[Q][3][3][3];
static void tables_init(void);
static inline double weight(int i) { return W_TAB[i]; }
static inline int opposite(int i) { return OPP_TAB[i]; }

void orc_lattice(int *c, double *w, int *opp)
{
    for (int i = 0; i < Q; ++i) {
        for (int d = 0; d < 3; ++d) c[3 * i + d] = CV[i][d];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}

static inline int delta_ab(int a, int b) { return a == b; }

/* Second-order Hermite tensor, Eq. (12): H2 = c c - c_s^2 I. */
static double hermite2_def(int i, int a, int b) { return CV[i][a] * CV[i][b] - CS2 * delta_ab(a, b); }

/* Third-order Hermite tensor, Eq. (13): H3 = c c c - c_s^2 S(c I), with S the
 * unnormalised sum over the three distinct index permutations. */
static double hermite3_def(int i, int a, int b, int g)
{
    return CV[i][a] * CV[i][b] * CV[i][g] -
           CS2 * (CV[i][a] * delta_ab(b, g) + CV[i][b] * delta_ab(a, g) + CV[i][g] * delta_ab(a, b));
}

static void tables_init(void)
{
    static int done = 0;
    if (done) return;
    for (int i = 0; i < Q; ++i) {
        W_TAB[i] = weight_of(i);
        OPP_TAB[i] = opposite_of(i);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                H2_TAB[i][a][b] = hermite2_def(i, a, b);
                for (int g = 0; g < 3; ++g) H3_TAB[i][a][b][g] = hermite3_def(i, a, b, g);
            }
    }
    done = 1;
}

static inline double hermite2(int i, int a, int b) { return H2_TAB[i][a][b]; }
static inline double hermite3(int i, int a, int b, int g) { return H3_TAB[i][a][b][g]; }

/* Library constructor: the tables are ready before any entry point runs. */
__attribute__((constructor)) static void oracle_ctor(void) { tables_init(); }

/* ------------------------------------------------------------------ */
/* Node-level pieces of the collision                                  */

/* Third-order equilibrium, Eq. (11). */
void orc_feq(double pstar, const double u[3], double out[Q])
{
    for (int i = 0; i < Q; ++i) {
        double cu = 0.0, h2 = 0.0, h3 = 0.0;
        for (int a = 0; a < 3; ++a) cu += CV[i][a] * u[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) h2 += hermite2(i, a, b) * u[a] * u[b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int g = 0; g < 3; ++g) h3 += hermite3(i, a, b, g) * u[a] * u[b] * u[g];
        out[i] = weight(i) * (pstar + cu / CS2 + h2 / (2.0 * CS2 * CS2) + h3 / (6.0 * CS2 * CS2 * CS2));
    }
}

/* Guo forcing term, Eq. (17), with the forcing expressed as an acceleration a
 * (force per unit mass; identical to the printed form when rho = 1). */
void orc_guo(const double u[3], const double a[3], double out[Q])
{
    for (int i = 0; i < Q; ++i) {
        double cu = 0.0;
        for (int d = 0; d < 3; ++d) cu += CV[i][d] * u[d];
        double s = 0.0;
        for (int d = 0; d < 3; ++d) s += ((CV[i][d] - u[d]) / CS2 + cu * CV[i][d] / (CS2 * CS2)) * a[d];
        out[i] = weight(i) * s;
    }
}

/* Regularised non-equilibrium populations, Eq. (14), with A3 built by the
 * recursion of Eq. (16): A3_abg = u_a A2_bg + u_b A2_ag + u_g A2_ab.
 * A2 is a full 3x3 row-major symmetric tensor. */
void orc_fneq_reg(const double u[3], const double A2[9], double out[Q])
{
    double A3[3][3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int g = 0; g < 3; ++g)
                A3[a][b][g] = u[a] * A2[3 * b + g] + u[b] * A2[3 * a + g] + u[g] * A2[3 * a + b];
    for (int i = 0; i < Q; ++i) {
        double h2 = 0.0, h3 = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) h2 += hermite2(i, a, b) * A2[3 * a + b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int g = 0; g < 3; ++g) h3 += hermite3(i, a, b, g) * A3[a][b][g];
        out[i] = weight(i) * (h2 / (2.0 * CS2 * CS2) + h3 / (6.0 * CS2 * CS2 * CS2));
    }
}

/* Macroscopic part of the collision at one fluid node (Sec. II A).  Inputs:
 * pre-collision populations f, local phase field phi with its isotropic
 * gradient G and Laplacian L.  Outputs: p* (Eq. (6)), velocity u (Eq. (7)),
 * acceleration a = F/rho of the total force (Eq. (18)) and omega (Eq. (10)).
 *
 * Readings where the paper is silent:
 *  - forces enter S_i and u as accelerations a = F/rho;
 *  - F_nu (Eq. (21)) uses the equilibrium at u' = j + a'/2 built without F_nu;
 *  - F_ext = (rho(phi) - rho_g) g. */
void orc_macro_node(const orc_params *p, double phi, const double G[3], double L, const double f[Q],
                    double *pstar_out, double u_out[3], double a_out[3], double *omega_out)
{
    /* chemical potential and capillary force, Eq. (19) and the definition after it:
     * mu_phi = 4 beta (phi - phi_l)(phi - phi_g)(phi - phi_0) - kappa_phi lap(phi),
     * phi_l = 1, phi_g = 0, phi_0 = 1/2, beta = 12 sigma/delta, kappa_phi = 3 sigma delta/2 */
    const double beta = 12.0 * p->sigma / p->delta;
    const double kappa_phi = 1.5 * p->sigma * p->delta;
    const double mu_phi = 4.0 * beta * (phi - 1.0) * (phi - 0.0) * (phi - 0.5) - kappa_phi * L;
    double Fs[3];
    for (int d = 0; d < 3; ++d) Fs[d] = mu_phi * G[d];

    /* mixture laws, Eqs. (8)-(10) */
    const double rho = p->rho_g + (p->rho_l - p->rho_g) * phi;
    const double mu = p->rho_g * p->nu_g + (p->rho_l * p->nu_l - p->rho_g * p->nu_g) * phi;
    const double nu = mu / rho;
    const double omega = 1.0 / (0.5 + nu / CS2);
    double grad_rho[3];
    for (int d = 0; d < 3; ++d) grad_rho[d] = (p->rho_l - p->rho_g) * G[d];

    /* kinetic moments, Eq. (6) and the first sum of Eq. (7) */
    double ps = 0.0, j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        ps += f[i];
        for (int d = 0; d < 3; ++d) j[d] += f[i] * CV[i][d];
    }

    /* pressure correction Eq. (20) and external force */
    double Fp[3], Fext[3], a1[3], u1[3];
    for (int d = 0; d < 3; ++d) {
        Fp[d] = -ps * CS2 * grad_rho[d];
        Fext[d] = (rho - p->rho_g) * p->g[d];
        a1[d] = (Fs[d] + Fp[d] + Fext[d]) / rho;
        u1[d] = j[d] + 0.5 * a1[d];
    }

    /* viscous correction Eq. (21) with Pi = sum_i (f_i - f_i^eq) c_i c_i */
    double feq1[Q], Pi[3][3] = {{0}};
    orc_feq(ps, u1, feq1);
    for (int i = 0; i < Q; ++i)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Pi[a][b] += (f[i] - feq1[i]) * CV[i][a] * CV[i][b];
    for (int d = 0; d < 3; ++d) {
        double Fnu = 0.0;
        for (int b = 0; b < 3; ++b) Fnu += Pi[d][b] * grad_rho[b];
        Fnu *= -nu * omega / CS2;
        a_out[d] = a1[d] + Fnu / rho;
        u_out[d] = j[d] + 0.5 * a_out[d]; /* Eq. (7) */
    }
    *pstar_out = ps;
    *omega_out = omega;
}

/* Local non-equilibrium moment (reading of Eq. (14)): the second moment of
 * f - (f^eq - S/2), f minus the shifted equilibrium of the trapezoidal
 * forcing (text after Eq. (17)).  A2 is a full 3x3 row-major tensor. */
void orc_a2_local(double pstar, const double u[3], const double a[3], const double f[Q], double A2[9])
{
    double feq[Q], S[Q];
    orc_feq(pstar, u, feq);
    orc_guo(u, a, S);
    for (int k = 0; k < 9; ++k) A2[k] = 0.0;
    for (int i = 0; i < Q; ++i)
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be)
                A2[3 * al + be] += (f[i] - feq[i] + 0.5 * S[i]) * CV[i][al] * CV[i][be];
}

/* Post-collision populations from the macroscopic fields and a
 * non-equilibrium moment A2: Eq. (3) with f^eq <- f^eq - S/2 (text after
 * Eq. (17)) and the regularised f^neq of Eqs. (14), (16):
 *   f_post = f^eq - S/2 + S + (1 - omega) f^neq_reg */
void orc_post_node(double pstar, const double u[3], const double a[3], double omega, const double A2[9],
                   double fpost[Q])
{
    double feq[Q], S[Q], fneq[Q];
    orc_feq(pstar, u, feq);
    orc_guo(u, a, S);
    orc_fneq_reg(u, A2, fneq);
    for (int i = 0; i < Q; ++i) fpost[i] = feq[i] + 0.5 * S[i] + (1.0 - omega) * fneq[i];
}

/* Collision at one fluid node with the local non-equilibrium moment
 * (collision = 0).  Outputs: post-collision populations, u and p*. */
void orc_collide_node(const orc_params *p, double phi, const double G[3], double L, const double f[Q],
                      double fpost[Q], double u_out[3], double *pstar_out)
{
    double a[3], omega, A2[9];
    orc_macro_node(p, phi, G, L, f, pstar_out, u_out, a, &omega);
    orc_a2_local(*pstar_out, u_out, a, f, A2);
    orc_post_node(*pstar_out, u_out, a, omega, A2, fpost);
}

/* ------------------------------------------------------------------ */
/* Grid helpers                                                        */

typedef struct { int nx, ny, nz; long N; } dims_t;

static inline int wrap(int v, int n) { return ((v % n) + n) % n; }

static inline long nidx(const dims_t *g, int x, int y, int z)
{
    return (long)wrap(x, g->nx) + (long)g->nx * ((long)wrap(y, g->ny) + (long)g->ny * wrap(z, g->nz));
}

static inline void ncoord(const dims_t *g, long n, int *x, int *y, int *z)
{
    *x = (int)(n % g->nx);
    *y = (int)((n / g->nx) % g->ny);
    *z = (int)(n / ((long)g->nx * g->ny));
}

static inline long neighbour(const dims_t *g, long n, int i)
{
    int x, y, z;
    ncoord(g, n, &x, &y, &z);
    x += CV[i][0];
    y += CV[i][1];
    z += CV[i][2];
    x = x < 0 ? x + g->nx : (x >= g->nx ? x - g->nx : x);
    y = y < 0 ? y + g->ny : (y >= g->ny ? y - g->ny : y);
    z = z < 0 ? z + g->nz : (z >= g->nz ? z - g->nz : z);
    return (long)x + (long)g->nx * ((long)y + (long)g->ny * z);
}

/* Isotropic gradient, Eq. (22): grad psi = (1/c_s^2) sum_i w_i psi(x + c_i) c_i */
static void grad_iso_at(const dims_t *g, const double *psi, long n, double G[3])
{
    G[0] = G[1] = G[2] = 0.0;
    for (int i = 0; i < Q; ++i) {
        double v = psi[neighbour(g, n, i)];
        for (int d = 0; d < 3; ++d) G[d] += weight(i) * v * CV[i][d];
    }
    for (int d = 0; d < 3; ++d) G[d] /= CS2;
}

/* Isotropic Laplacian, Eq. (23): (2/c_s^2)(sum_{i!=0} w_i psi(x+c_i) - (1-w_0) psi(x)) */
static double lap_iso_at(const dims_t *g, const double *psi, long n)
{
    double s = 0.0;
    for (int i = 1; i < Q; ++i) s += weight(i) * psi[neighbour(g, n, i)];
    return (2.0 / CS2) * (s - (1.0 - weight(0)) * psi[n]);
}

void orc_grad_iso(int nx, int ny, int nz, const double *psi, double *out)
{
    dims_t g = {nx, ny, nz, (long)nx * ny * nz};
#pragma omp parallel for schedule(static)
    for (long n = 0; n < g.N; ++n) {
        double G[3];
        grad_iso_at(&g, psi, n, G);
        for (int d = 0; d < 3; ++d) out[d * g.N + n] = G[d];
    }
}

void orc_lap_iso(int nx, int ny, int nz, const double *psi, double *out)
{
    dims_t g = {nx, ny, nz, (long)nx * ny * nz};
#pragma omp parallel for schedule(static)
    for (long n = 0; n < g.N; ++n) out[n] = lap_iso_at(&g, psi, n);
}

/* ------------------------------------------------------------------ */
/* Geometry: wall nodes, wall normal and donor (Sec. II B)              */

/* Link weights of Eq. (37): 1, 1/2, 1/3 for |c|^2 = 1, 2, 3. */
static double wall_link_weight(int q) { return 1.0 / (double)norm2(q); }

/* For every solid node with at least one fluid neighbour (the set B), in
 * ascending linear index: its index, 6 * (unnormalised wall normal of
 * Eq. (36)) as integers, and the donor link q* of Eqs. (39)-(40), or -1
 * when the normal vanishes (the node is skipped).  Admissible donors are
 * all fluid links of the node; exact ties go to the lowest link index.
 * Returns |B| (and writes at most cap entries), or -1 on bad input. */
int orc_wall_nodes(int nx, int ny, int nz, const uint8_t *solid, int32_t *idx, int32_t *n6, int32_t *qstar,
                   int cap)
{
    if (nx < 1 || ny < 1 || nz < 1 || !solid) return -1;
    dims_t g = {nx, ny, nz, (long)nx * ny * nz};
    int nb = 0;
    for (long s = 0; s < g.N; ++s) {
        if (!solid[s]) continue;
        int nfluid = 0;
        double nt[3] = {0, 0, 0};
        for (int q = 1; q < Q; ++q) {
            if (solid[neighbour(&g, s, q)]) continue;
            ++nfluid;
            for (int d = 0; d < 3; ++d) nt[d] += wall_link_weight(q) * (-CV[q][d]);
        }
        if (nfluid == 0) continue; /* not adjacent to the fluid */
        if (nb < cap) {
            /* the weights are multiples of 1/6, so 6*nt is an exact integer */
            int m6[3];
            for (int d = 0; d < 3; ++d) m6[d] = (int)lround(6.0 * nt[d]);
            idx[nb] = (int32_t)s;
            for (int d = 0; d < 3; ++d) n6[3 * nb + d] = m6[d];
            int best = -1;
            if (m6[0] != 0 || m6[1] != 0 || m6[2] != 0) {
                double nn = sqrt((double)(m6[0] * m6[0] + m6[1] * m6[1] + m6[2] * m6[2]));
                double best_score = -HUGE_VAL;
                for (int q = 1; q < Q; ++q) {
                    if (solid[neighbour(&g, s, q)]) continue;
                    /* S_q = ((-c_q) . n_w) / |c_q|, Eq. (39); numerator evaluated on the
                     * integer normal so equal scores compare equal */
                    int dot = -(CV[q][0] * m6[0] + CV[q][1] * m6[1] + CV[q][2] * m6[2]);
                    double score = (double)dot / (nn * sqrt((double)norm2(q)));
                    if (score > best_score) {
                        best_score = score;
                        best = q;
                    }
                }
            }
            qstar[nb] = best;
        }
        ++nb;
    }
    return nb;
}

/* ------------------------------------------------------------------ */
/* Substep W: ghost-node wetting update (Sec. II B, Eqs. (36)-(47))      */

/* Ghost value of a wall node with donor link q (x_f = x_s + c_q), unit wall
 * normal n_w (Eq. (38), pointing into the solid), donor value phi_f and
 * isotropic donor gradient G (Eq. (22)).  With G_par = G - (G.n_w) n_w the
 * tangential gradient (Eq. (42)), theta_c = pi - theta (Eq. (43)), the
 * corrected gradient G_c = G_par + d_n n_w with d_n = -|G_par| cot(theta_c)
 * (Eqs. (44)-(45)) and r_fs = -c_q (Eq. (41)), the extrapolation of Eq. (46)
 * is, in closed form,
 *   phi_g = phi_f + lambda_s G_c . r_fs
 *         = phi_f - lambda_s [ c_q . G_par - |G_par| cot(theta_c) (c_q . n_w) ],
 * lambda_s from Eq. (47) (or 1 for the diagnostic reading).  Gc receives the
 * corrected gradient (it sets the compressive flux on the wall node). */
static double ghost_value(const orc_params *p, int q, const double nw[3], double phi_f, const double G[3],
                          double theta, double Gc[3])
{
    const double gn = G[0] * nw[0] + G[1] * nw[1] + G[2] * nw[2];
    double Gpar[3];
    for (int d = 0; d < 3; ++d) Gpar[d] = G[d] - gn * nw[d];
    const double t = sqrt(Gpar[0] * Gpar[0] + Gpar[1] * Gpar[1] + Gpar[2] * Gpar[2]);
    /* cot(theta_c), replaced by +-cot_max where |sin(theta_c)| < sin_tol (text after Eq. (45)) */
    const double sc = sin(M_PI - theta), cc = cos(M_PI - theta);
    const double cot_c = (fabs(sc) < p->sin_tol) ? copysign(p->cot_max, cc) : cc / sc;
    for (int d = 0; d < 3; ++d) Gc[d] = Gpar[d] - t * cot_c * nw[d];
    const double cq_par = CV[q][0] * Gpar[0] + CV[q][1] * Gpar[1] + CV[q][2] * Gpar[2];
    const double cq_n = CV[q][0] * nw[0] + CV[q][1] * nw[1] + CV[q][2] * nw[2];
    const double l2 = 4.0 * phi_f * (1.0 - phi_f);
    const double lambda_s = p->ghost_localization ? sqrt(l2 > 0.0 ? l2 : 0.0) : 1.0;
    return phi_f - lambda_s * (cq_par - t * cot_c * cq_n);
}

/* phi_in: phi^n on fluid nodes and the previous ghosts on wall nodes.
 * theta: prescribed contact angle (radians) per node, read at wall nodes.
 * phi_hat (output, all nodes): a copy of phi_in with every non-skipped wall
 * node replaced by its new ghost value.  Donor gradients read phi_in only
 * (Jacobi update), so the result does not depend on the visiting order.
 * a_wall (output, optional, 3N): compressive flux assigned to wall nodes,
 * zero elsewhere; with wall_compression = 1 it is g (1 - g) times the unit
 * corrected gradient of Eq. (45), so the ghost enters the compressive term
 * as it enters the diffusive one; otherwise zero. */
int orc_ghost(const orc_params *p, int nx, int ny, int nz, const uint8_t *solid, const double *theta,
              const double *phi_in, double *phi_hat, double *a_wall)
{
    dims_t g = {nx, ny, nz, (long)nx * ny * nz};
    int nb = orc_wall_nodes(nx, ny, nz, solid, NULL, NULL, NULL, 0);
    if (nb < 0) return -1;
    int32_t *idx = malloc(sizeof(int32_t) * (nb + 1));
    int32_t *n6 = malloc(sizeof(int32_t) * 3 * (nb + 1));
    int32_t *qs = malloc(sizeof(int32_t) * (nb + 1));
    orc_wall_nodes(nx, ny, nz, solid, idx, n6, qs, nb);
    memcpy(phi_hat, phi_in, sizeof(double) * g.N);
    if (a_wall) memset(a_wall, 0, sizeof(double) * 3 * g.N);

#pragma omp parallel for schedule(static)
    for (int k = 0; k < nb; ++k) {
        const int q = qs[k];
        if (q < 0) continue; /* |n_w| = 0: skipped, ghost unchanged */
        const long xs = idx[k];
        /* unit wall normal, Eq. (38) */
        double nn = sqrt((double)n6[3 * k] * n6[3 * k] + (double)n6[3 * k + 1] * n6[3 * k + 1] +
                         (double)n6[3 * k + 2] * n6[3 * k + 2]);
        double nw[3] = {n6[3 * k] / nn, n6[3 * k + 1] / nn, n6[3 * k + 2] / nn};
        /* donor node x_f = x_s + c_q (Eq. (41)), its value and isotropic gradient */
        const long xf = neighbour(&g, xs, q);
        const double phi_f = phi_in[xf];
        double Gf[3], Gc[3];
        grad_iso_at(&g, phi_in, xf, Gf);
        const double gv = ghost_value(p, q, nw, phi_f, Gf, theta[xs], Gc);
        phi_hat[xs] = gv;
        if (a_wall && p->wall_compression) {
            double gc2 = Gc[0] * Gc[0] + Gc[1] * Gc[1] + Gc[2] * Gc[2];
            if (gc2 > p->eps_n * p->eps_n)
                for (int d = 0; d < 3; ++d) a_wall[d * g.N + xs] = gv * (1.0 - gv) * Gc[d] / sqrt(gc2);
        }
    }
    free(idx);
    free(n6);
    free(qs);
    return nb;
}

/* ------------------------------------------------------------------ */
/* Substep H: hydrodynamics (Sec. II A)                                 */

/* Gradient form of the non-equilibrium moment, Eq. (15), at every fluid node:
 *   A2_ab = -(c_s^2/omega) (d_a u_b + d_b u_a),
 * with the velocity derivatives taken by the isotropic gradient of Eq. (22)
 * applied to each velocity component.  Reading: a solid neighbour x + c_i of
 * node x holds the mirror image -u(x), so that the velocity vanishes at the
 * half-link, where halfway bounce-back puts the resting wall.  u: 3 planes of
 * N; omega: N; A2: 9 planes of N (row-major a, b), zero on solid nodes. */
void orc_a2grad(int nx, int ny, int nz, const uint8_t *solid, const double *u, const double *omega, double *A2)
{
    dims_t g = {nx, ny, nz, (long)nx * ny * nz};
    const long N = g.N;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        for (int k = 0; k < 9; ++k) A2[k * N + n] = 0.0;
        if (solid[n]) continue;
        double D[3][3] = {{0}}; /* D[b][a] = d_b u_a */
        for (int i = 0; i < Q; ++i) {
            long y = neighbour(&g, n, i);
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) {
                    const double ua = solid[y] ? -u[a * N + n] : u[a * N + y];
                    D[b][a] += weight(i) * CV[i][b] * ua / CS2;
                }
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A2[(3 * a + b) * N + n] = -(CS2 / omega[n]) * (D[a][b] + D[b][a]);
    }
}

/* f_in: pre-collision populations on fluid nodes.  Writes the post-collision
 * populations (fpost, optional), the streamed populations f_out (pull with
 * halfway bounce-back: f_out_i(x) = fpost_i(x - c_i) if that node is fluid,
 * else fpost_opp(i)(x)), and u, p* on fluid nodes.
 *
 * collision = 0: A2 is the local moment of each node's own populations.
 * collision = 1: the macroscopic fields of every node come first; A2 is then
 * the gradient form of Eq. (15) built from the new velocity field, and the
 * post-collision populations are assembled from p*, u, a, omega and that A2
 * (the thread-safe formulation of Sec. II A: both parts of the populations
 * follow from macroscopic quantities). */
int orc_hydro(const orc_params *p, int nx, int ny, int nz, const uint8_t *solid, const double *phi_hat,
              const double *f_in, double *fpost_out, double *f_out, double *u, double *pstar)
{
    dims_t g = {nx, ny, nz, (long)nx * ny * nz};
    const long N = g.N;
    double *fpost = fpost_out ? fpost_out : malloc(sizeof(double) * Q * N);
    if (!fpost) return -1;
    if (p->collision == 1) {
        double *acc = malloc(sizeof(double) * 3 * N), *om = malloc(sizeof(double) * N);
        double *A2 = malloc(sizeof(double) * 9 * N), *uf = calloc(3 * N, sizeof(double));
        if (!acc || !om || !A2 || !uf) return -1;
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; ++n) {
            om[n] = 1.0;
            if (solid[n]) continue;
            double G[3], f[Q], uu[3], aa[3], ps;
            grad_iso_at(&g, phi_hat, n, G);
            double L = lap_iso_at(&g, phi_hat, n);
            for (int i = 0; i < Q; ++i) f[i] = f_in[i * N + n];
            orc_macro_node(p, phi_hat[n], G, L, f, &ps, uu, aa, &om[n]);
            for (int d = 0; d < 3; ++d) {
                uf[d * N + n] = uu[d];
                acc[d * N + n] = aa[d];
                u[d * N + n] = uu[d];
            }
            pstar[n] = ps;
        }
        orc_a2grad(nx, ny, nz, solid, uf, om, A2);
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; ++n) {
            if (solid[n]) continue;
            double uu[3], aa[3], A[9], fp[Q];
            for (int d = 0; d < 3; ++d) {
                uu[d] = uf[d * N + n];
                aa[d] = acc[d * N + n];
            }
            for (int k = 0; k < 9; ++k) A[k] = A2[k * N + n];
            orc_post_node(pstar[n], uu, aa, om[n], A, fp);
            for (int i = 0; i < Q; ++i) fpost[i * N + n] = fp[i];
        }
        free(acc);
        free(om);
        free(A2);
        free(uf);
    } else {
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; ++n) {
            if (solid[n]) continue;
            double G[3], f[Q], fp[Q], uu[3], ps;
            grad_iso_at(&g, phi_hat, n, G);
            double L = lap_iso_at(&g, phi_hat, n);
            for (int i = 0; i < Q; ++i) f[i] = f_in[i * N + n];
            orc_collide_node(p, phi_hat[n], G, L, f, fp, uu, &ps);
            for (int i = 0; i < Q; ++i) fpost[i * N + n] = fp[i];
            for (int d = 0; d < 3; ++d) u[d * N + n] = uu[d];
            pstar[n] = ps;
        }
    }
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        if (solid[n]) continue;
        for (int i = 0; i < Q; ++i) {
            long src = neighbour(&g, n, opposite(i)); /* x - c_i */
            f_out[i * N + n] = solid[src] ? fpost[opposite(i) * N + n] : fpost[i * N + src];
        }
    }
    if (!fpost_out) free(fpost);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Substep P: CAC update (Sec. II A 1)                                  */

static double minmod(double a, double b)
{
    /* Eq. (32) */
    if (a * b <= 0.0) return 0.0;
    return (a > 0 ? 1.0 : -1.0) * fmin(fabs(a), fabs(b));
}

/* Advective flux through the face between node x and its +e_d neighbour,
 * Eqs. (30)-(34).  Zero when either node is solid (no flux through the wall
 * faces); slopes read phi_hat, which holds ghosts at wall nodes. */
static double face_flux(const dims_t *g, const uint8_t *solid, const double *phi, const double *u, long x, int d)
{
    static const int AX[3] = {1, 3, 5}; /* +e_x, +e_y, +e_z links */
    const int ip = AX[d], im = AX[d] + 1;
    const long y = neighbour(g, x, ip);
    if (solid[x] || solid[y]) return 0.0;
    const long xm = neighbour(g, x, im);
    const long yp = neighbour(g, y, ip);
    const double uf = 0.5 * (u[d * g->N + x] + u[d * g->N + y]);
    const double s_x = minmod(phi[x] - phi[xm], phi[y] - phi[x]);  /* Eq. (31) at x */
    const double s_y = minmod(phi[y] - phi[x], phi[yp] - phi[y]);  /* Eq. (31) at x + e_d */
    const double phiL = phi[x] + 0.5 * s_x;                        /* Eq. (33) */
    const double phiR = phi[y] - 0.5 * s_y;
    const double phiup = (uf >= 0.0) ? phiL : phiR;                /* Eq. (34) */
    return uf * phiup;                                             /* Eq. (30) */
}

/* phi_hat: phi^n on fluid nodes with the new ghosts on wall nodes; u: velocity
 * of the hydrodynamic substep; a_wall: compressive flux on wall nodes from the
 * ghost update (NULL: zero).  phistar (all nodes) = phi_hat, with fluid nodes
 * replaced by the tentative update of Eq. (28):
 *   phi* = phi - div_h(F_a) + D lap_iso(phi) + S_comp,
 *   S_comp = -kappa div_iso(a),  a = phi(1-phi) n on fluid nodes, a_wall on solid,
 * with the divergence of Eq. (35) taken with the isotropic weights w_i/c_s^2. */
int orc_phase(const orc_params *p, int nx, int ny, int nz, const uint8_t *solid, const double *phi_hat,
              const double *u, const double *a_wall, double *phistar)
{
    dims_t g = {nx, ny, nz, (long)nx * ny * nz};
    const long N = g.N;
    const double kappa = 4.0 * p->D / p->delta; /* Eq. (26) */
    double *a = calloc(3 * N, sizeof(double));
    if (!a) return -1;
    /* compressive flux field a = phi (1 - phi) n with n = grad phi / |grad phi|, Eq. (25) */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        if (solid[n]) {
            if (a_wall)
                for (int d = 0; d < 3; ++d) a[d * N + n] = a_wall[d * N + n];
            continue;
        }
        double G[3];
        grad_iso_at(&g, phi_hat, n, G);
        double gg = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        if (gg <= p->eps_n * p->eps_n) continue; /* n = 0 where the gradient vanishes */
        double inv = 1.0 / sqrt(gg);
        double ph = phi_hat[n];
        for (int d = 0; d < 3; ++d) a[d * N + n] = ph * (1.0 - ph) * G[d] * inv;
    }
    memcpy(phistar, phi_hat, sizeof(double) * N);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        if (solid[n]) continue;
        /* conservative MUSCL advection, Eq. (29) */
        double div_a = 0.0;
        for (int d = 0; d < 3; ++d) {
            static const int AXM[3] = {2, 4, 6};
            div_a += face_flux(&g, solid, phi_hat, u, n, d) - face_flux(&g, solid, phi_hat, u, neighbour(&g, n, AXM[d]), d);
        }
        /* isotropic diffusion */
        double lap = lap_iso_at(&g, phi_hat, n);
        /* isotropic divergence of the compressive flux */
        double div_c = 0.0;
        for (int i = 1; i < Q; ++i) {
            long y = neighbour(&g, n, i);
            double ac = a[y] * CV[i][0] + a[N + y] * CV[i][1] + a[2 * N + y] * CV[i][2];
            div_c += weight(i) / CS2 * ac;
        }
        phistar[n] = phi_hat[n] - div_a + p->D * lap - kappa * div_c;
    }
    free(a);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Substep V: global volume correction (Sec. II C)                      */

/* phi_new = phistar on all nodes, with fluid nodes corrected by Eq. (53).
 * Sums run in FP64 over fluid nodes in ascending index order.  Returns the
 * multiplier lambda_M = dM/W of Eq. (55) through *lambda (0 when W = 0 or the
 * correction is off). */
int orc_volume(const orc_params *p, int nx, int ny, int nz, const uint8_t *solid, const double *phistar,
               double M_target, double *phi_new, double *lambda)
{
    const long N = (long)nx * ny * nz;
    double Mstar = 0.0, W = 0.0;
    for (long n = 0; n < N; ++n) {
        if (solid[n]) continue;
        double ph = phistar[n];
        Mstar += ph;                                                          /* Eq. (49) */
        if (ph > p->eps_phi && ph < 1.0 - p->eps_phi) W += ph * (1.0 - ph);  /* Eqs. (51)-(52) */
    }
    double lam = 0.0;
    if (p->volume_correction && W > 0.0) lam = (M_target - Mstar) / W; /* Eqs. (50), (55) */
    for (long n = 0; n < N; ++n) {
        double ph = phistar[n];
        if (solid[n]) {
            phi_new[n] = ph;
            continue;
        }
        double chi = (ph > p->eps_phi && ph < 1.0 - p->eps_phi) ? ph * (1.0 - ph) : 0.0;
        phi_new[n] = ph + lam * chi;
    }
    if (lambda) *lambda = lam;
    return 0;
}

/* Threads the OpenMP loops use. */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* Set the number of threads of the OpenMP loops (n >= 1). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

/* Phase-field mass, Eq. (48): sum of phi over fluid nodes. */
double orc_mass(int nx, int ny, int nz, const uint8_t *solid, const double *phi)
{
    const long N = (long)nx * ny * nz;
    double M = 0.0;
    for (long n = 0; n < N; ++n)
        if (!solid[n]) M += phi[n];
    return M;
}

/* ------------------------------------------------------------------ */
/* Initial state and the full step                                      */

/* f = f^eq(p*0, u0) on fluid nodes (p*0, u0 may be NULL: zero), phi = phi0 on
 * all nodes (the values on wall nodes are the initial ghosts), and the target
 * mass M_target = sum over fluid nodes of phi0. */
int orc_init(int nx, int ny, int nz, const uint8_t *solid, const double *phi0, const double *pstar0,
             const double *u0, double *f, double *phi, double *M_target)
{
    const long N = (long)nx * ny * nz;
    memset(f, 0, sizeof(double) * Q * N);
    for (long n = 0; n < N; ++n) {
        phi[n] = phi0[n];
        if (solid[n]) continue;
        double uu[3] = {0, 0, 0}, feq[Q];
        if (u0)
            for (int d = 0; d < 3; ++d) uu[d] = u0[d * N + n];
        orc_feq(pstar0 ? pstar0[n] : 0.0, uu, feq);
        for (int i = 0; i < Q; ++i) f[i * N + n] = feq[i];
    }
    *M_target = orc_mass(nx, ny, nz, solid, phi0);
    return 0;
}

static int all_finite(const double *v, long n)
{
    for (long k = 0; k < n; ++k)
        if (!isfinite(v[k])) return 0;
    return 1;
}

/* Advance nsteps full steps W -> H -> P -> V.  fpost_last (optional) receives
 * the post-collision populations of the last step.  Returns 0, or 4 if a
 * non-finite value appeared in phi or u (the state is then left as it is). */
int orc_step(const orc_params *p, int nx, int ny, int nz, const uint8_t *solid, const double *theta, double *f,
             double *phi, double *u, double *pstar, double M_target, int nsteps, double *fpost_last)
{
    const long N = (long)nx * ny * nz;
    double *phi_hat = malloc(sizeof(double) * N);
    double *phistar = malloc(sizeof(double) * N);
    double *f_new = calloc((size_t)Q * N, sizeof(double));
    double *a_wall = malloc(sizeof(double) * 3 * N);
    if (!phi_hat || !phistar || !f_new || !a_wall) return -1;
    int rc = 0;
    for (int s = 0; s < nsteps && rc == 0; ++s) {
        orc_ghost(p, nx, ny, nz, solid, theta, phi, phi_hat, a_wall);
        orc_hydro(p, nx, ny, nz, solid, phi_hat, f, (s == nsteps - 1) ? fpost_last : NULL, f_new, u, pstar);
        orc_phase(p, nx, ny, nz, solid, phi_hat, u, a_wall, phistar);
        orc_volume(p, nx, ny, nz, solid, phistar, M_target, phi, NULL);
        memcpy(f, f_new, sizeof(double) * Q * N);
        if (!all_finite(phi, N) || !all_finite(u, 3 * N)) rc = 4;
    }
    free(phi_hat);
    free(phistar);
    free(f_new);
    free(a_wall);
    return rc;
}
