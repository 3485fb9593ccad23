/*
 * fpd_oracle.c -- plain, slow, single-threaded FP64 reference for one time step of the
 * fluid-particle-dynamics (FPD) method for a bead-spring fiber, solved with a D2Q9
 * multiple-relaxation-time lattice Boltzmann scheme (arXiv:2212.14153, Sec. II).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the GPU path is checked against.
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * build, load or call it; the product library never does.  It shares no code, header,
 * table or constant with the HIP path: every table below is written out here.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, no fast-math).
 *
 * Conventions (lattice units): dx = dt = 1, c_s^2 = 1/3, reference density rho0 = 1.
 *   - the paper's z axis is y here;
 *   - node (i, j) sits at the centre (i+1/2, j+1/2) of lattice square (i, j)
 *     (Sec. II.C, last paragraph before the integration steps);
 *   - the wall below y = 0 moves with -U x, the wall above y = ny with +U x, x is
 *     periodic (Sec. IV.A, Fig. 1b); or, for the single-particle benchmark of
 *     Sec. III.B, no walls: x and y both periodic;
 *   - populations f are stored k-major: f[(k*ny + j)*nx + i], k = 0..8;
 *   - bead positions R[2*b + {0,1}], b = 0..N-1 (the paper's bead i is b = i-1).
 *
 * Readings of points the paper leaves open (each one is also listed in the design notes):
 *   - MRT basis, equilibria and rates: the paper defers them to its refs [41,44]; the
 *     Lallemand-Luo D2Q9 moment basis is used, with the shear rate s_nu from the local
 *     viscosity, s_e, s_eps as parameters and s_q either fixed or the per-site value that
 *     makes (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16.
 *   - "centered formulation for the forcing term": Guo's forcing, i.e. the velocity is
 *     (j + f/2)/rho and the source is (I - S/2) M F_guo.
 *   - viscosity to relaxation: nu = eta / rho0 with rho0 = 1, tau = 3 nu + 1/2.
 *   - bead velocity, Eq. (5): the velocity field v^{n+1} is Guo's macroscopic velocity
 *     (j^{n+1} + f^n/2)/rho^{n+1} after the step, with f^n the force density that drove
 *     it; it is weighted by phi^n and normalised by int phi^n.  (With the bare j/rho
 *     instead, the bond-stretch modes of a chain inside a viscous body grow without
 *     bound at r_eta = 50, which the paper's stable runs rule out.)
 *   - bending energy: the printed forces (11),(12) are the exact negative gradient of
 *     U_b = -k_b sum_j t_{j+1}.t_j (linear in the cosine); they are evaluated here as
 *     printed, with tangents outside 1..N-1 taken as zero.
 *   - moving walls: half-way bounce-back with wall density rho0.
 *   - the driven particle of Sec. III.B: a constant external force F0 on every bead,
 *     added to F_i and spread by Eq. (4); in a periodic box a uniform body force g on
 *     every node (the caller takes g = -N F0 / (nx ny)) removes the net momentum input,
 *     so that the fluid far from the particle stays at rest on average.
 *   - drag of Eq. (17): the printed normalisation by int phi does not give a force;
 *     the diffuse-interface form of the surface integral is used, n dA -> -grad phi dr:
 *     F = int (p grad phi - sigma . grad phi) dr with sigma = eta (grad v + grad v^T),
 *     p = rho / 3 taken relative to rho0 / 3, gradients by the isotropic D2Q9 stencil
 *     3 sum_k w_k e_k q(x + e_k).
 *     The viscous and pressure parts are returned separately.
 *   - Eq. (15): V0 is the phi-weighted mean velocity of the particle, i.e. Eq. (5)
 *     evaluated on the current state.
 *   - the sandwich benchmark of Sec. III.A: its solid slabs are a fixed profile
 *     phi_s(y) (Eq. (14)) that enters Eq. (1) next to the beads' sum_i phi_i.
 *   - several fibers (the outlook of Sec. V): Eqs. (10)-(12) act inside each fiber; the
 *     paper names no force between fibers, so by default they meet through the fluid
 *     alone, and an optional excluded volume (a soft pair repulsion between beads of
 *     different fibers closer than d, 2a by default) keeps them from passing through
 *     each other.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- parameters ---- */

typedef struct orc_params {
    int    nx, ny;        /* lattice squares along x (periodic) and y (walls)          */
    double u_wall;        /* U: bottom wall moves with -U, top wall with +U             */
    double nu_f;          /* fluid kinematic viscosity eta_f / rho0                     */
    double eta_ratio;     /* r_eta = eta_s / eta_f                                       */
    double xi;            /* interface thickness xi of Eq. (2)                           */
    int    n_beads;       /* N                                                           */
    double radius;        /* a                                                           */
    double l0;            /* spring rest length l_0                                      */
    double k_s, k_b;      /* stretching and bending constants of Eq. (9)                 */
    double s_e, s_eps;    /* MRT rates of the energy and energy-square moments           */
    double s_q_fixed;     /* > 0: fixed heat-flux rate; <= 0: per-site magic value       */
    int    clamp_phi;     /* 1: clamp sum_i phi_i to 1 in Eq. (1) (off by default)       */
    int    periodic_y;    /* 1: no walls, y periodic too (Sec. III.B benchmark box)      */
    double fx_ext, fy_ext;   /* external force F0 on every bead                          */
    double gx_body, gy_body; /* uniform body force density on every node                 */
    const double *phi_static; /* NULL or [ny]: a fixed interface profile phi_s(y) added to
                                 sum_i phi_i in Eq. (1) (the solid slabs of Eq. (14))      */
    int    n_chains;      /* fibers: beads c*L .. c*L+L-1 form fiber c, L = N / n_chains
                             (<= 1: one fiber)                                             */
    double ev_k;          /* excluded volume between fibers: pair energy k/2 (d - r)^2     */
    double ev_range;      /* d (<= 0: 2a); beads of one fiber do not repel                 */
} orc_params;

/* ---------------------------------------------------------- D2Q9 lattice ---------- */

static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* Moment matrix of the Lallemand-Luo basis, rows ordered
 * (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy). */
static const double MM[9][9] = {
    { 1,  1,  1,  1,  1,  1,  1,  1,  1},
    {-4, -1, -1, -1, -1,  2,  2,  2,  2},
    { 4, -2, -2, -2, -2,  1,  1,  1,  1},
    { 0,  1,  0, -1,  0,  1, -1, -1,  1},
    { 0, -2,  0,  2,  0,  1, -1, -1,  1},
    { 0,  0,  1,  0, -1,  1,  1, -1, -1},
    { 0,  0, -2,  0,  2,  1,  1, -1, -1},
    { 0,  1, -1,  1, -1,  0,  0,  0,  0},
    { 0,  0,  0,  0,  0,  1, -1,  1, -1},
};

/* In IEEE double, tanh(t) rounds to exactly -1 for t <= -20 (1 - |tanh| = 2e^{-40} is
 * below half an ulp of 1), so phi of Eq. (2) is exactly 0 there. */
#define TANH_SATURATION 20.0

static size_t idx(const orc_params *p, int k, int i, int j)
{
    return ((size_t)k * (size_t)p->ny + (size_t)j) * (size_t)p->nx + (size_t)i;
}

/* --------------------------------------------- Eqs. (9)-(12): bead-spring forces -- */

/* Tangent t_m = R_{m,m+1} / R_{m,m+1} and bond length R_{m,m+1}, m = 1..N-1 in the
 * paper's numbering; outside that range the tangent is the zero vector (Eq. (12) reading). */
static void tangent(const double *R, int N, int m, double t[2], double *len)
{
    t[0] = 0.0; t[1] = 0.0; *len = 0.0;
    if (m < 1 || m > N - 1) return;
    double dx = R[2 * m] - R[2 * (m - 1)];      /* R_{m+1} - R_m with 0-based storage */
    double dy = R[2 * m + 1] - R[2 * (m - 1) + 1];
    double L = sqrt(dx * dx + dy * dy);
    t[0] = dx / L; t[1] = dy / L; *len = L;
}

/* v . (I - t t) / L */
static void proj_over_len(const double v[2], const double t[2], double L, double out[2])
{
    double vt = v[0] * t[0] + v[1] * t[1];
    out[0] = (v[0] - vt * t[0]) / L;
    out[1] = (v[1] - vt * t[1]) / L;
}

/* F_i = F_i^s + F_i^b, Eq. (10): stretching force Eq. (11a,b) and bending force
 * Eq. (12a-e), each bead i = 1..N of one fiber evaluated from the printed per-bead
 * formulas. */
static void fiber_forces(const orc_params *p, const double *R, int N, double *F)
{
    const double ks = p->k_s / (p->l0 * p->l0);
    for (int i = 1; i <= N; ++i) {
        double Fs[2] = {0.0, 0.0}, Fb[2] = {0.0, 0.0};
        double tm2[2], tm1[2], ti[2], tp1[2];
        double Lm2, Lm1, Li, Lp1;
        tangent(R, N, i - 2, tm2, &Lm2);
        tangent(R, N, i - 1, tm1, &Lm1);
        tangent(R, N, i, ti, &Li);
        tangent(R, N, i + 1, tp1, &Lp1);
        /* Eq. (11a) for interior beads, (11b) for the two ends */
        if (i >= 2) {                    /* bond (i-1, i) exists */
            Fs[0] -= ks * (Lm1 - p->l0) * tm1[0];
            Fs[1] -= ks * (Lm1 - p->l0) * tm1[1];
        }
        if (i <= N - 1) {                /* bond (i, i+1) exists */
            Fs[0] += ks * (Li - p->l0) * ti[0];
            Fs[1] += ks * (Li - p->l0) * ti[1];
        }
        /* Eq. (12a): k_b [ (t_i + t_{i-2}).(I - t_{i-1}t_{i-1})/R_{i-1,i}
         *                - (t_{i+1} + t_{i-1}).(I - t_i t_i)/R_{i,i+1} ];
         * Eqs. (12b-e) are this expression with the missing tangents set to zero. */
        if (i >= 2) {
            double s[2] = {ti[0] + tm2[0], ti[1] + tm2[1]}, q[2];
            proj_over_len(s, tm1, Lm1, q);
            Fb[0] += p->k_b * q[0];
            Fb[1] += p->k_b * q[1];
        }
        if (i <= N - 1) {
            double s[2] = {tp1[0] + tm1[0], tp1[1] + tm1[1]}, q[2];
            proj_over_len(s, ti, Li, q);
            Fb[0] -= p->k_b * q[0];
            Fb[1] -= p->k_b * q[1];
        }
        F[2 * (i - 1)] = Fs[0] + Fb[0];
        F[2 * (i - 1) + 1] = Fs[1] + Fb[1];
    }
}

/* Excluded volume between fibers (the paper names none; off unless ev_k > 0): beads i, j
 * of different fibers whose centres are r < d apart repel with the force of the pair
 * energy (k/2)(d - r)^2, k (d - r) along R_i - R_j (minimum image along periodic
 * directions).  Added to F_i as a sum over j in increasing order. */
static void excluded_volume(const orc_params *p, const double *R, int L, double *F)
{
    const double d = p->ev_range > 0.0 ? p->ev_range : 2.0 * p->radius;
    for (int i = 0; i < p->n_beads; ++i) {
        for (int j = 0; j < p->n_beads; ++j) {
            if (j / L == i / L) continue;          /* same fiber */
            double dx = R[2 * i] - R[2 * j], dy = R[2 * i + 1] - R[2 * j + 1];
            dx -= (double)p->nx * floor(dx / (double)p->nx + 0.5);
            if (p->periodic_y) dy -= (double)p->ny * floor(dy / (double)p->ny + 0.5);
            const double r = sqrt(dx * dx + dy * dy);
            if (!(r < d) || r == 0.0) continue;
            const double s = p->ev_k * (d - r) / r;
            F[2 * i] += s * dx;
            F[2 * i + 1] += s * dy;
        }
    }
}

/* Forces on every bead: each fiber on its own, the excluded volume between fibers when
 * it is switched on, plus the external force F0 of the driven-particle benchmark
 * (Sec. III.B). */
void orc_bead_forces(const orc_params *p, const double *R, double *F)
{
    const int C = p->n_chains > 1 ? p->n_chains : 1;
    const int L = p->n_beads / C;
    for (int c = 0; c < C; ++c) fiber_forces(p, R + 2 * c * L, L, F + 2 * c * L);
    if (p->ev_k > 0.0 && C > 1) excluded_volume(p, R, L, F);
    for (int b = 0; b < p->n_beads; ++b) {
        F[2 * b] += p->fx_ext;
        F[2 * b + 1] += p->fy_ext;
    }
}

/* ---------------------------------------------- Eq. (2): interface profile -------- */

/* phi_i at node (i, j) for a bead centred at (Rx, Ry); distances along periodic
 * directions are minimum images. */
double orc_phi(const orc_params *p, double Rx, double Ry, int i, int j)
{
    double dx = ((double)i + 0.5) - Rx;
    double dy = ((double)j + 0.5) - Ry;
    dx -= (double)p->nx * floor(dx / (double)p->nx + 0.5);
    if (p->periodic_y) dy -= (double)p->ny * floor(dy / (double)p->ny + 0.5);
    double r = sqrt(dx * dx + dy * dy);
    double t = (p->radius - r) / p->xi;
    if (t <= -TANH_SATURATION) return 0.0;     /* tanh(t) is exactly -1 here */
    return 0.5 * (tanh(t) + 1.0);
}

/* Rows that can hold a non-zero phi of a bead at height Ry: phi vanishes exactly once
 * |r - R| >= a + 20 xi, so every other row contributes exact zeros to every sum below
 * and the loops skip them without changing any result. */
static void phi_rows(const orc_params *p, double Ry, int *jlo, int *jhi)
{
    if (p->periodic_y) {     /* the support may wrap: take every row */
        *jlo = 0;
        *jhi = p->ny - 1;
        return;
    }
    double reach = p->radius + TANH_SATURATION * p->xi + 1.0;
    int lo = (int)floor(Ry - reach), hi = (int)ceil(Ry + reach);
    *jlo = lo < 0 ? 0 : lo;
    *jhi = hi > p->ny - 1 ? p->ny - 1 : hi;
}

/* Step (1) of Sec. II.C at time n, evaluated from the bead positions R^n:
 *   phi_i^n at every node (Eq. (2)), stored for the rows where it can be non-zero;
 *   A_i = int phi_i^n, the lattice sum in the denominators of Eqs. (4) and (5);
 *   F_i^n (Eqs. (10)-(12)); the force density f^n (Eq. (4), plus the uniform body
 *   force g); eta^n (Eq. (1)). */
typedef struct stage1 {
    int     N;
    int    *jlo, *jhi;      /* phi_i rows: phi[i] holds rows jlo[i]..jhi[i], all columns */
    double **phi;
    double *A, *F;
    double *eta, *fx, *fy;  /* per node */
} stage1;

static double phi_at(const orc_params *p, const stage1 *s1, int b, int i, int j)
{
    if (j < s1->jlo[b] || j > s1->jhi[b]) return 0.0;
    return s1->phi[b][(size_t)(j - s1->jlo[b]) * (size_t)p->nx + (size_t)i];
}

static void stage1_compute(const orc_params *p, const double *R, stage1 *s1)
{
    const int N = p->n_beads, nx = p->nx, ny = p->ny;
    const size_t S = (size_t)nx * (size_t)ny;
    const double eta_f = p->nu_f;                  /* rho0 = 1 */
    const double eta_s = p->eta_ratio * eta_f;
    s1->N = N;
    s1->jlo = (int *)calloc(N > 0 ? N : 1, sizeof(int));
    s1->jhi = (int *)calloc(N > 0 ? N : 1, sizeof(int));
    s1->phi = (double **)calloc(N > 0 ? N : 1, sizeof(double *));
    s1->A = (double *)calloc(N > 0 ? N : 1, sizeof(double));
    s1->F = (double *)calloc(N > 0 ? 2 * N : 1, sizeof(double));
    s1->eta = (double *)malloc(S * sizeof(double));
    s1->fx = (double *)calloc(S, sizeof(double));
    s1->fy = (double *)calloc(S, sizeof(double));
    double *sphi = (double *)calloc(S, sizeof(double));

    if (N > 0) orc_bead_forces(p, R, s1->F);
    for (int b = 0; b < N; ++b) {
        phi_rows(p, R[2 * b + 1], &s1->jlo[b], &s1->jhi[b]);
        int rows = s1->jhi[b] - s1->jlo[b] + 1;
        if (rows < 0) rows = 0;
        s1->phi[b] = (double *)calloc((size_t)(rows > 0 ? rows : 1) * (size_t)nx, sizeof(double));
        double sum = 0.0;
        for (int j = s1->jlo[b]; j <= s1->jhi[b]; ++j)
            for (int i = 0; i < nx; ++i) {
                double ph = orc_phi(p, R[2 * b], R[2 * b + 1], i, j);
                s1->phi[b][(size_t)(j - s1->jlo[b]) * (size_t)nx + (size_t)i] = ph;
                sum += ph;
            }
        s1->A[b] = sum;
    }
    /* sum over beads in bead order at every node */
    for (int b = 0; b < N; ++b) {
        double cx = s1->F[2 * b] / s1->A[b], cy = s1->F[2 * b + 1] / s1->A[b];
        for (int j = s1->jlo[b]; j <= s1->jhi[b]; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t s = (size_t)j * (size_t)nx + (size_t)i;
                double ph = phi_at(p, s1, b, i, j);
                sphi[s] += ph;
                s1->fx[s] += ph * cx;                      /* Eq. (4) */
                s1->fy[s] += ph * cy;
            }
    }
    for (size_t s = 0; s < S; ++s) {
        double sp = sphi[s];
        if (p->phi_static) sp += p->phi_static[s / (size_t)nx];
        if (p->clamp_phi && sp > 1.0) sp = 1.0;
        s1->eta[s] = eta_f + (eta_s - eta_f) * sp;         /* Eq. (1) */
        s1->fx[s] += p->gx_body;                           /* uniform body force */
        s1->fy[s] += p->gy_body;
    }
    free(sphi);
}

static void stage1_free(stage1 *s1)
{
    for (int b = 0; b < s1->N; ++b) free(s1->phi[b]);
    free(s1->phi); free(s1->jlo); free(s1->jhi); free(s1->A); free(s1->F);
    free(s1->eta); free(s1->fx); free(s1->fy);
}

/* Step (1) for callers: A[N], F[N][2], eta, fx, fy (per node). */
void orc_fields(const orc_params *p, const double *R, double *A, double *F,
                double *eta, double *fx, double *fy)
{
    const size_t S = (size_t)p->nx * (size_t)p->ny;
    stage1 s1;
    stage1_compute(p, R, &s1);
    for (int b = 0; b < p->n_beads; ++b) {
        A[b] = s1.A[b]; F[2 * b] = s1.F[2 * b]; F[2 * b + 1] = s1.F[2 * b + 1];
    }
    memcpy(eta, s1.eta, S * sizeof(double));
    memcpy(fx, s1.fx, S * sizeof(double));
    memcpy(fy, s1.fy, S * sizeof(double));
    stage1_free(&s1);
}

/* ------------------------------------------------- MRT collision with forcing ---- */

/* Equilibrium moments of the Lallemand-Luo basis. */
void orc_meq(double rho, double ux, double uy, double meq[9])
{
    double u2 = ux * ux + uy * uy;
    meq[0] = rho;
    meq[1] = -2.0 * rho + 3.0 * rho * u2;
    meq[2] = rho - 3.0 * rho * u2;
    meq[3] = rho * ux;
    meq[4] = -rho * ux;
    meq[5] = rho * uy;
    meq[6] = -rho * uy;
    meq[7] = rho * (ux * ux - uy * uy);
    meq[8] = rho * ux * uy;
}

/* m = M f */
void orc_moments(const double f[9], double m[9])
{
    for (int r = 0; r < 9; ++r) {
        double s = 0.0;
        for (int k = 0; k < 9; ++k) s += MM[r][k] * f[k];
        m[r] = s;
    }
}

/* f = M^{-1} m, with M^{-1} = M^T diag(1 / |row_r|^2) (the rows of M are orthogonal).
 * The table is formed once, on first use. */
static double MINV[9][9];
static int minv_ready = 0;

void orc_inverse_moments(const double m[9], double f[9])
{
    if (!minv_ready) {
        for (int r = 0; r < 9; ++r) {
            double norm = 0.0;
            for (int k = 0; k < 9; ++k) norm += MM[r][k] * MM[r][k];
            for (int k = 0; k < 9; ++k) MINV[k][r] = MM[r][k] / norm;
        }
        minv_ready = 1;
    }
    for (int k = 0; k < 9; ++k) {
        double s = 0.0;
        for (int r = 0; r < 9; ++r) s += MINV[k][r] * m[r];
        f[k] = s;
    }
}

/* One MRT collision at a node with force density (Fx, Fy):
 *   rho = sum f, j = sum f e, u = (j + F/2)/rho,
 *   m* = m - S (m - m_eq) + (I - S/2) M G,  f* = M^{-1} m*,
 * with Guo's source G_k = w_k [ (e_k - u)/c_s^2 + (e_k.u) e_k / c_s^4 ] . F. */
void orc_collide(const double f[9], double s_nu, double s_e, double s_eps, double s_q,
                 double Fx, double Fy, double fout[9])
{
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int k = 0; k < 9; ++k) {
        rho += f[k];
        jx += f[k] * EX[k];
        jy += f[k] * EY[k];
    }
    double ux = (jx + 0.5 * Fx) / rho;
    double uy = (jy + 0.5 * Fy) / rho;
    double G[9];
    for (int k = 0; k < 9; ++k) {
        double eu = EX[k] * ux + EY[k] * uy;
        double gx = 3.0 * (EX[k] - ux) + 9.0 * eu * EX[k];
        double gy = 3.0 * (EY[k] - uy) + 9.0 * eu * EY[k];
        G[k] = W[k] * (gx * Fx + gy * Fy);
    }
    double m[9], meq[9], Gm[9], ms[9];
    orc_moments(f, m);
    orc_meq(rho, ux, uy, meq);
    orc_moments(G, Gm);
    const double S[9] = {0.0, s_e, s_eps, 0.0, s_q, 0.0, s_q, s_nu, s_nu};
    for (int r = 0; r < 9; ++r)
        ms[r] = m[r] - S[r] * (m[r] - meq[r]) + (1.0 - 0.5 * S[r]) * Gm[r];
    orc_inverse_moments(ms, fout);
}

/* Shear rate from the local viscosity (rho0 = 1): s_nu = 1 / (3 eta + 1/2). */
static double shear_rate(double eta) { return 1.0 / (3.0 * eta + 0.5); }

/* Heat-flux rate: fixed, or the value giving (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16. */
static double q_rate(const orc_params *p, double s_nu)
{
    if (p->s_q_fixed > 0.0) return p->s_q_fixed;
    return 8.0 * (2.0 - s_nu) / (8.0 - s_nu);
}

/* -------------------------------------------- streaming with moving walls --------- */

/* Push every post-collision population to its neighbour; x wraps (y too without
 * walls); a population that would leave through a wall is reflected half-way back into the opposite direction at
 * the same node and picks up 6 w rho0 (e . u_wall) (moving-wall bounce-back). */
void orc_stream(const orc_params *p, const double *fpost, double *fnew)
{
    const int nx = p->nx, ny = p->ny;
    for (int k = 0; k < 9; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double v = fpost[idx(p, k, i, j)];
                int jd = j + EY[k];
                if (p->periodic_y) jd = (jd + ny) % ny;
                if (jd >= 0 && jd < ny) {
                    int id = ((i + EX[k]) % nx + nx) % nx;
                    fnew[idx(p, k, id, jd)] = v;
                } else {
                    double uw = (jd < 0) ? -p->u_wall : p->u_wall;
                    int kb = OPP[k];
                    fnew[idx(p, kb, i, j)] = v + 6.0 * W[kb] * (EX[kb] * uw);
                }
            }
}

/* ------------------------------------------------------- the LBM stage ------------ */

/* Step (2) with the on-lattice fields given: collide every node with its own shear
 * rate s_nu(x) and force density f(x), then stream.  f is replaced by f^{n+1}. */
void orc_lbm_step_fields(const orc_params *p, double *f, const double *s_nu,
                         const double *fx, const double *fy)
{
    const int nx = p->nx, ny = p->ny;
    const size_t S = (size_t)nx * (size_t)ny;
    double *post = (double *)malloc(9 * S * sizeof(double));
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t s = (size_t)j * (size_t)nx + (size_t)i;
            double fl[9], fo[9];
            for (int k = 0; k < 9; ++k) fl[k] = f[idx(p, k, i, j)];
            orc_collide(fl, s_nu[s], p->s_e, p->s_eps, q_rate(p, s_nu[s]), fx[s], fy[s], fo);
            for (int k = 0; k < 9; ++k) post[idx(p, k, i, j)] = fo[k];
        }
    orc_stream(p, post, f);
    free(post);
}

/* Bare velocity j/rho and density of the populations at every node. */
void orc_bare_velocity(const orc_params *p, const double *f, double *rho, double *vx,
                       double *vy)
{
    const int nx = p->nx, ny = p->ny;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int k = 0; k < 9; ++k) {
                double v = f[idx(p, k, i, j)];
                r += v; jx += v * EX[k]; jy += v * EY[k];
            }
            size_t s = (size_t)j * (size_t)nx + (size_t)i;
            rho[s] = r; vx[s] = jx / r; vy[s] = jy / r;
        }
}

/* ------------------------------------------------------- one full time step ------- */

/* The three-stage step of Sec. II.C:
 *  (1) phi_i^n, F_i^n, f^n, eta^n from R^n;
 *  (2) MRT-LBM collide + stream: f^n -> f^{n+1};
 *  (3) V_i^{n+1} = int phi_i^n v^{n+1} / int phi_i^n  (Eq. (5)),
 *      R_i^{n+1} = R_i^n + dt V_i^{n+1}  (forward Euler, dt = 1).
 * f and R are updated in place; V and F (may be NULL) receive V^{n+1} and F^n. */
void orc_step(const orc_params *p, double *f, double *R, double *V, double *F)
{
    const int N = p->n_beads, nx = p->nx, ny = p->ny;
    const size_t S = (size_t)nx * (size_t)ny;
    double *snu = (double *)malloc(S * sizeof(double));
    double *rho = (double *)malloc(S * sizeof(double));
    double *vx = (double *)malloc(S * sizeof(double));
    double *vy = (double *)malloc(S * sizeof(double));
    stage1 s1;

    /* (1) */
    stage1_compute(p, R, &s1);
    for (size_t s = 0; s < S; ++s) snu[s] = shear_rate(s1.eta[s]);
    /* (2) */
    orc_lbm_step_fields(p, f, snu, s1.fx, s1.fy);
    /* (3) velocity field after the step: Guo's macroscopic velocity
     *     v^{n+1} = (sum_k f_k^{n+1} e_k + f^n / 2) / rho^{n+1},
     * with f^n the force density that drove the step. */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int k = 0; k < 9; ++k) {
                double v = f[idx(p, k, i, j)];
                r += v; jx += v * EX[k]; jy += v * EY[k];
            }
            size_t s = (size_t)j * (size_t)nx + (size_t)i;
            rho[s] = r;
            vx[s] = (jx + 0.5 * s1.fx[s]) / r;
            vy[s] = (jy + 0.5 * s1.fy[s]) / r;
        }
    for (int b = 0; b < N; ++b) {
        double sx = 0.0, sy = 0.0;
        for (int j = s1.jlo[b]; j <= s1.jhi[b]; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t s = (size_t)j * (size_t)nx + (size_t)i;
                double ph = phi_at(p, &s1, b, i, j);
                sx += ph * vx[s];
                sy += ph * vy[s];
            }
        double Vx = sx / s1.A[b], Vy = sy / s1.A[b];
        if (V) { V[2 * b] = Vx; V[2 * b + 1] = Vy; }
        if (F) { F[2 * b] = s1.F[2 * b]; F[2 * b + 1] = s1.F[2 * b + 1]; }
        R[2 * b] += Vx;
        R[2 * b + 1] += Vy;
    }
    stage1_free(&s1);
    free(snu); free(rho); free(vx); free(vy);
}

/* n_steps full steps; if traj is not NULL it receives R after every step,
 * traj[(s*N + b)*2 + c]. */
void orc_run(const orc_params *p, double *f, double *R, long n_steps, double *V, double *F,
             double *traj)
{
    const int N = p->n_beads;
    for (long s = 0; s < n_steps; ++s) {
        orc_step(p, f, R, V, F);
        if (traj)
            for (int b = 0; b < 2 * N; ++b) traj[(size_t)s * 2 * (size_t)N + (size_t)b] = R[b];
    }
}

/* ------------------------------------------------------ initial state ------------ */

/* Second-order Maxwell-Boltzmann equilibrium of D2Q9. */
static double feq(int k, double rho, double ux, double uy)
{
    double eu = EX[k] * ux + EY[k] * uy;
    return W[k] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * (ux * ux + uy * uy));
}

/* init_flow 0: fluid at rest; 1: linear Couette profile u_x = U (2y/H - 1) at the node
 * centres; populations at equilibrium with rho = rho0 = 1. */
void orc_init(const orc_params *p, int init_flow, double *f)
{
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            double ux = 0.0;
            if (init_flow == 1)
                ux = p->u_wall * (2.0 * ((double)j + 0.5) / (double)p->ny - 1.0);
            for (int k = 0; k < 9; ++k) f[idx(p, k, i, j)] = feq(k, 1.0, ux, 0.0);
        }
}

/* Macroscopic read-out at step n: density, velocity u = (j + f^n/2)/rho with the force
 * density of the current bead state, and viscosity eta^n. */
void orc_macro(const orc_params *p, const double *f, const double *R, double *rho,
               double *ux, double *uy, double *eta)
{
    const int nx = p->nx, ny = p->ny;
    const size_t S = (size_t)nx * (size_t)ny;
    stage1 s1;
    stage1_compute(p, R, &s1);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double r = 0.0, jx = 0.0, jy = 0.0;
            for (int k = 0; k < 9; ++k) {
                double v = f[idx(p, k, i, j)];
                r += v; jx += v * EX[k]; jy += v * EY[k];
            }
            size_t s = (size_t)j * (size_t)nx + (size_t)i;
            rho[s] = r;
            ux[s] = (jx + 0.5 * s1.fx[s]) / r;
            uy[s] = (jy + 0.5 * s1.fy[s]) / r;
        }
    memcpy(eta, s1.eta, S * sizeof(double));
    stage1_free(&s1);
}

/* ------------------------------------- single-particle diagnostics (Sec. III.B) -- */

/* Isotropic D2Q9 gradient of a node field q: grad q (x) = 3 sum_k w_k e_k q(x + e_k)
 * (the isotropic discretisation the paper uses for gradients of phase-field variables,
 * Sec. II.C).  Neighbours wrap along periodic directions; with walls, rows 0 and ny-1
 * have no complete stencil and get NaN. */
void orc_iso_gradient(const orc_params *p, const double *q, double *gx, double *gy)
{
    const int nx = p->nx, ny = p->ny;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t s = (size_t)j * (size_t)nx + (size_t)i;
            if (!p->periodic_y && (j == 0 || j == ny - 1)) {
                gx[s] = NAN;
                gy[s] = NAN;
                continue;
            }
            double ax = 0.0, ay = 0.0;
            for (int k = 1; k < 9; ++k) {
                int in = ((i + EX[k]) % nx + nx) % nx;
                int jn = ((j + EY[k]) % ny + ny) % ny;
                double v = q[(size_t)jn * (size_t)nx + (size_t)in];
                ax += W[k] * EX[k] * v;
                ay += W[k] * EY[k] * v;
            }
            gx[s] = 3.0 * ax;
            gy[s] = 3.0 * ay;
        }
}

/* Diagnostics of bead b on the current state (pre-collision f at step n, positions R^n):
 *   out[0]    A = sum_x phi_b
 *   out[1,2]  V0 = sum_x phi_b v / A, v = (j + f^n/2)/rho (Eq. (5) on this state)
 *   out[3]    eps_v = sum_x phi_b |v - V0|^2 / A (Eq. (15))
 *   out[4,5]  viscous force of the fluid on the particle, -sum_x sigma . grad phi_b,
 *             sigma = eta (grad v + grad v^T) with eta of Eq. (1)
 *   out[6,7]  pressure force, sum_x (p - p0) grad phi_b with p = rho/3, p0 = 1/3 (the
 *             constant p0 adds nothing: sum_x grad phi_b telescopes to zero, and leaving
 *             it out avoids summing O(1) terms that cancel)
 * (Eq. (17) in its diffuse-interface form: n dA -> -grad phi dr.)  With walls the forces
 * are NaN when phi_b reaches the two outer rows at a wall (incomplete stencil). */
void orc_particle_stats(const orc_params *p, const double *f, const double *R, int b,
                        double *out)
{
    const int nx = p->nx, ny = p->ny;
    const size_t S = (size_t)nx * (size_t)ny;
    double *rho = (double *)malloc(S * sizeof(double));
    double *vx = (double *)malloc(S * sizeof(double));
    double *vy = (double *)malloc(S * sizeof(double));
    double *eta = (double *)malloc(S * sizeof(double));
    double *ph = (double *)malloc(S * sizeof(double));
    double *g[6];
    for (int m = 0; m < 6; ++m) g[m] = (double *)malloc(S * sizeof(double));
    orc_macro(p, f, R, rho, vx, vy, eta);
    double A = 0.0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t s = (size_t)j * (size_t)nx + (size_t)i;
            ph[s] = orc_phi(p, R[2 * b], R[2 * b + 1], i, j);
            A += ph[s];
        }
    double mx = 0.0, my = 0.0;
    for (size_t s = 0; s < S; ++s) {
        mx += ph[s] * vx[s];
        my += ph[s] * vy[s];
    }
    const double V0x = mx / A, V0y = my / A;
    double e = 0.0;
    for (size_t s = 0; s < S; ++s) {
        double dx = vx[s] - V0x, dy = vy[s] - V0y;
        e += ph[s] * (dx * dx + dy * dy);
    }
    orc_iso_gradient(p, ph, g[0], g[1]);   /* d_x phi, d_y phi */
    orc_iso_gradient(p, vx, g[2], g[3]);   /* d_x vx, d_y vx   */
    orc_iso_gradient(p, vy, g[4], g[5]);   /* d_x vy, d_y vy   */
    /* with walls the stencil is incomplete on rows 0 and ny-1: they hold no interface
     * as long as phi_b vanishes on the two outer rows at each wall; otherwise the
     * forces are undefined (NaN) */
    int wall_touch = 0;
    if (!p->periodic_y)
        for (int i = 0; i < nx; ++i)
            for (int r = 0; r < 2 && r < ny; ++r)
                if (ph[(size_t)r * nx + i] != 0.0 || ph[(size_t)(ny - 1 - r) * nx + i] != 0.0)
                    wall_touch = 1;
    double fvx = 0.0, fvy = 0.0, fpx = 0.0, fpy = 0.0;
    for (size_t s = 0; s < S; ++s) {
        int j = (int)(s / (size_t)nx);
        if (!p->periodic_y && (j == 0 || j == ny - 1) && !wall_touch) continue;
        double dpx = g[0][s], dpy = g[1][s];
        if (dpx == 0.0 && dpy == 0.0) continue;   /* outside the interface */
        double sxx = eta[s] * 2.0 * g[2][s];
        double syy = eta[s] * 2.0 * g[5][s];
        double sxy = eta[s] * (g[3][s] + g[4][s]);
        fvx -= sxx * dpx + sxy * dpy;
        fvy -= sxy * dpx + syy * dpy;
        fpx += (rho[s] - 1.0) / 3.0 * dpx;
        fpy += (rho[s] - 1.0) / 3.0 * dpy;
    }
    out[0] = A;
    out[1] = V0x;
    out[2] = V0y;
    out[3] = e / A;
    out[4] = fvx;
    out[5] = fvy;
    out[6] = fpx;
    out[7] = fpy;
    for (int m = 0; m < 6; ++m) free(g[m]);
    free(rho); free(vx); free(vy); free(eta); free(ph);
}
