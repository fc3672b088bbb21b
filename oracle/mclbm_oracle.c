/*
 * Plain FP64 CPU oracle of the moment-chain lattice Boltzmann method for
 * hyperelastic solids (Mueller, Faust, Schlueter, Mueller, arXiv 2502.00920).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU leg of
 * the benchmark can check the HIP library against an independent, slow and
 * obviously correct implementation.  It shares no code, header, table or
 * constant with the HIP path.
 *
 * What it computes: Algorithm 1 ("The proposed LB algorithm for non-linear
 * solid mechanics", Sect. 3.2) on a D2Q9 lattice (Tab. 1), one time step as
 * four whole-lattice passes in the printed order:
 *   A  moments -> equilibrium -> forcing -> BGK collision -> streaming
 *   B  boundary nodes: Dirichlet modified bounce-back (Eq. bbcon) and
 *      Neumann modified anti-bounce-back (Eq. abbcon), Sect. 3.3
 *   C  stresses: H = grad u by finite differences (Eq. defgrad, Sect. 3.2),
 *      P(H) (St. Venant-Kirchhoff / neo-Hooke, Sect. 4), Pi(H)
 *   D  source S = rho0 b + Div(P + Pi(H)) (Eq. source), moments, trapezoidal
 *      displacement update (Sect. 3.2)
 * Everything is in the paper's physical units: c_s = sqrt(mu/rho0),
 * c = sqrt(3) c_s, dt = dX / c (Sect. 2, Sect. 3.2).
 *
 * Readings of passages the paper leaves open (all listed in the design notes):
 *   - dt is derived from dX, mu, rho0; tau is dimensionless, so the collision
 *     factor dt/tau is 1/tau and the forcing factor is (1 - 1/(2 tau)).
 *   - Plane strain: lambda = 2 mu nu / (1 - 2 nu); this is the only reading
 *     under which the CFL bounds nu <= 1/4 and nu <= 5/11 of Sect. 3.2 hold.
 *   - Pi(H) = -mu (H + H^T + tr(H) I): the stress carried by the bare moment
 *     chain with the third moment Q of Eq. Qlin and j = rho0 du/dt.
 *   - The trapezoidal update carries the factor dt: u += dt/(2 rho0)(j'+j).
 *   - Time levels: the stresses T_n = P(H) + Pi(H) and the source S_n are
 *     evaluated from the current displacement u_n before the collision, so the
 *     collision at t_n, the moment j(t_{n+1}) and the boundary rules of step n
 *     all use level n (Sect. 3.1 states that S is taken at time t in both the
 *     collision and the moment computation).  The order printed in
 *     Algorithm 1, where the stress pass follows streaming and the collision
 *     therefore sees S_{n-1}, is kept as an option (time_levels = 1).
 *   - Nodes are cell centred, walls lie half way to the next (absent) node.
 *   - Finite differences: central in the interior, first-order one-sided
 *     (using the inward neighbour) at the outermost node.  Second-order
 *     one-sided differences there are an option (boundary order 2).
 *   - Neumann momentum flux at the wall (Sect. 3.3): with outward normal
 *     N = s e_a and tangential axis b, Pi_aa = -s T*_a + ext(T_aa),
 *     Pi_ab = Pi_ba = -s T*_b + ext(T_ba), Pi_bb = ext(Pi_bb of the
 *     populations); r_bd = r(X).  ext carries the node value to the half-way
 *     wall unchanged (zeroth order; default) or extrapolates linearly,
 *     (3 v(X) - v(X_in)) / 2 (option).
 *   - Corners: a link that crosses a Dirichlet wall is bounced back with that
 *     wall's j* (the mean j* when it crosses two Dirichlet walls); a link that
 *     crosses one Neumann wall uses that wall's Pi_bd; the diagonal link that
 *     crosses two Neumann walls uses a combined Pi_bd (normal entries from
 *     each wall, shear entry the mean of both, or as an option one wall's).
 *   - Initial state: f = f_eq(r0 = -rho0 tr H(u0), j0, Pi(H(u0))).
 *   - Collision: BGK (the paper's); two relaxation times as an option.
 * Periodic sides are an addition for tests (momentum balance, plane waves).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared -o liboracle.so
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- constants of the D2Q9 scheme, Tab. 1 --------------------------------- */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

enum { SIDE_LEFT = 0, SIDE_RIGHT = 1, SIDE_BOTTOM = 2, SIDE_TOP = 3 };
enum { BC_DIRICHLET = 0, BC_NEUMANN = 1, BC_PERIODIC = 2 };
enum { MAT_SVK = 0, MAT_NH = 1, MAT_LINEAR = 2 };
enum { LOAD_ZERO = 0, LOAD_CONST = 1, LOAD_DISP_RAMP = 2, LOAD_LINEAR_RAMP = 3,
       LOAD_SIN2_RAMP = 4, LOAD_SIN_PULSE = 5, LOAD_GAUSS = 6, LOAD_RICKER = 7, LOAD_TABLE = 8 };
enum { FIELD_U = 0, FIELD_J = 1, FIELD_R = 2, FIELD_PI = 3, FIELD_H = 4,
       FIELD_P = 5, FIELD_S = 6 };

typedef struct {
    int bc, kind;
    double amp[2], t0, t1, width;
    double *table;     /* LOAD_TABLE: the scalar program per step (owned copy) */
    int64_t table_len;
} side_t;

typedef struct {
    int nx, ny, material, extrap_linear, listing_order, boundary_order, corner, threads;
    double dx, rho0, mu, nu, tau, body[2];
    /* derived, Sect. 3.2 */
    double lam, cs2, c, dt, omega;
    double omega_plus; /* two-relaxation-time option: rate of the even part, 0 = BGK */
    double cq[9][2]; /* physical lattice velocities c_q = c * e_q */
    side_t side[4];
    /* state at the start of step n */
    int64_t n;
    double *f;     /* pre-collision populations f(t_n), [9][ny][nx] */
    double *u;     /* u_n, [2][ny][nx] */
    double *Sp;    /* listing order only: S_{n-1}, [2][ny][nx] */
    double *Tp;    /* listing order only: T_{n-1}, [4][ny][nx] */
    /* scratch of one step */
    double *fc, *fn, *r, *Pi, *un, *jA, *S, *T;
} orc_t;

#define IDX(h, x, y) ((size_t)(y) * (size_t)(h)->nx + (size_t)(x))

static size_t nn(const orc_t *h) { return (size_t)h->nx * (size_t)h->ny; }

/* ---- building blocks, exported so that tests can pin each one ------------ */

/* Equilibrium of the solid moment chain, Sect. 3.2 (f_eq in terms of r, j, Pi). */
void orc_feq(double cs2, const double cq[9][2], double r, const double j[2],
             const double Pi[3], double out[9])
{
    /* Pi = (xx, xy, yy) */
    for (int q = 0; q < 9; q++) {
        double cx = cq[q][0], cy = cq[q][1];
        double cj = cx * j[0] + cy * j[1];
        /* (Pi - r cs2 I) : (c c - cs2 I) */
        double Axx = Pi[0] - r * cs2, Axy = Pi[1], Ayy = Pi[2] - r * cs2;
        double contr = Axx * (cx * cx - cs2) + 2.0 * Axy * (cx * cy) + Ayy * (cy * cy - cs2);
        out[q] = W[q] * (r + cj / cs2 + contr / (2.0 * cs2 * cs2));
    }
}

/* Forcing term psi_q = w_q c_q . S / c_s^2, Eq. forcing. */
void orc_psi(double cs2, const double cq[9][2], const double S[2], double out[9])
{
    for (int q = 0; q < 9; q++)
        out[q] = W[q] * (cq[q][0] * S[0] + cq[q][1] * S[1]) / cs2;
}

/* BGK collision with forcing at one node (Algorithm 1, collide): the moments
 * r, j = sum c f + dt/2 S, Pi, then f - (dt/tau)(f - f_eq) + (1 - dt/(2 tau)) psi dt
 * with dt/tau = omega.  Writes r, j, Pi (xx, xy, yy) when the pointers are set. */
void orc_collide(double cs2, const double cq[9][2], double omega, double dt,
                 const double f[9], const double S[2], double out[9],
                 double *r_out, double j_out[2], double Pi_out[3])
{
    double r = 0, mx = 0, my = 0, pxx = 0, pxy = 0, pyy = 0;
    for (int q = 0; q < 9; q++) {
        r += f[q];
        mx += cq[q][0] * f[q];
        my += cq[q][1] * f[q];
        pxx += cq[q][0] * cq[q][0] * f[q];
        pxy += cq[q][0] * cq[q][1] * f[q];
        pyy += cq[q][1] * cq[q][1] * f[q];
    }
    double jj[2] = {mx + 0.5 * dt * S[0], my + 0.5 * dt * S[1]};
    double Pi3[3] = {pxx, pxy, pyy};
    double feq[9], psi[9];
    orc_feq(cs2, cq, r, jj, Pi3, feq);
    orc_psi(cs2, cq, S, psi);
    for (int q = 0; q < 9; q++)
        out[q] = f[q] - omega * (f[q] - feq[q]) + (1.0 - 0.5 * omega) * psi[q] * dt;
    if (r_out) *r_out = r;
    if (j_out) { j_out[0] = jj[0]; j_out[1] = jj[1]; }
    if (Pi_out) { Pi_out[0] = pxx; Pi_out[1] = pxy; Pi_out[2] = pyy; }
}

/* The same collision with two relaxation times (an option; the paper names
 * collision operators beyond BGK as a way to stability, Sect. 6): the
 * non-equilibrium part n = f - f_eq splits into its even part (n_q + n_qbar)/2,
 * relaxed at omega_plus, and its odd part (n_q - n_qbar)/2, relaxed at omega as
 * in BGK; the forcing, odd, keeps the factor (1 - omega/2).  With
 * omega_plus = omega this is the BGK collision above. */
void orc_collide_trt(double cs2, const double cq[9][2], double omega, double omega_plus, double dt,
                     const double f[9], const double S[2], double out[9],
                     double *r_out, double j_out[2], double Pi_out[3])
{
    double r = 0, mx = 0, my = 0, pxx = 0, pxy = 0, pyy = 0;
    for (int q = 0; q < 9; q++) {
        r += f[q];
        mx += cq[q][0] * f[q];
        my += cq[q][1] * f[q];
        pxx += cq[q][0] * cq[q][0] * f[q];
        pxy += cq[q][0] * cq[q][1] * f[q];
        pyy += cq[q][1] * cq[q][1] * f[q];
    }
    double jj[2] = {mx + 0.5 * dt * S[0], my + 0.5 * dt * S[1]};
    double Pi3[3] = {pxx, pxy, pyy};
    double feq[9], psi[9];
    orc_feq(cs2, cq, r, jj, Pi3, feq);
    orc_psi(cs2, cq, S, psi);
    for (int q = 0; q < 9; q++) {
        double nq = f[q] - feq[q], nb = f[OPP[q]] - feq[OPP[q]];
        double even = 0.5 * (nq + nb), odd = 0.5 * (nq - nb);
        out[q] = f[q] - omega_plus * even - omega * odd + (1.0 - 0.5 * omega) * psi[q] * dt;
    }
    if (r_out) *r_out = r;
    if (j_out) { j_out[0] = jj[0]; j_out[1] = jj[1]; }
    if (Pi_out) { Pi_out[0] = pxx; Pi_out[1] = pxy; Pi_out[2] = pyy; }
}

/* Plane-strain Lame parameter lambda from mu and nu. */
double orc_lambda(double mu, double nu) { return 2.0 * mu * nu / (1.0 - 2.0 * nu); }

/* First Piola-Kirchhoff stress, Sect. 4: P = (I + H) S with the second
 * Piola-Kirchhoff stress S of St. Venant-Kirchhoff or neo-Hooke.  H and P are
 * stored row-major (xx, xy, yx, yy), H_ab = d u_a / d X_b.  LINEAR is Hooke's
 * law of the linear-elastic scheme the paper compares with. */
void orc_stress_P(int material, double lam, double mu, const double H[4], double P[4])
{
    double F[2][2] = {{1.0 + H[0], H[1]}, {H[2], 1.0 + H[3]}};
    double Hm[2][2] = {{H[0], H[1]}, {H[2], H[3]}};
    double S2[2][2];
    if (material == MAT_LINEAR) {
        double tr = Hm[0][0] + Hm[1][1];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                P[2 * a + b] = (a == b ? lam * tr : 0.0) + mu * (Hm[a][b] + Hm[b][a]);
        return;
    }
    if (material == MAT_SVK) {
        double E[2][2];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                double HtH = Hm[0][a] * Hm[0][b] + Hm[1][a] * Hm[1][b];
                E[a][b] = 0.5 * (Hm[b][a] + Hm[a][b] + HtH);
            }
        double trE = E[0][0] + E[1][1];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                S2[a][b] = (a == b ? lam * trE : 0.0) + 2.0 * mu * E[a][b];
    } else {
        /* neo-Hooke: S = lam/2 (J^2 - 1) C^-1 + mu (I - C^-1)
         *              = [lam/2 (J^2 - 1) I + mu (C - I)] C^-1,
         * with C - I = H + H^T + H^T H and J^2 - 1 = (J - 1)(J + 1),
         * J - 1 = tr H + det H, formed from H so that small strains keep
         * their relative precision. */
        double CmI[2][2], C[2][2];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                double HtH = Hm[0][a] * Hm[0][b] + Hm[1][a] * Hm[1][b];
                CmI[a][b] = Hm[a][b] + Hm[b][a] + HtH;
                C[a][b] = (a == b ? 1.0 : 0.0) + CmI[a][b];
            }
        double Jm1 = (Hm[0][0] + Hm[1][1]) + (Hm[0][0] * Hm[1][1] - Hm[0][1] * Hm[1][0]);
        double J2m1 = Jm1 * (Jm1 + 2.0);
        double detC = C[0][0] * C[1][1] - C[0][1] * C[1][0];
        double Ci[2][2] = {{C[1][1] / detC, -C[0][1] / detC},
                           {-C[1][0] / detC, C[0][0] / detC}};
        double A[2][2];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                A[a][b] = (a == b ? 0.5 * lam * J2m1 : 0.0) + mu * CmI[a][b];
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++)
                S2[a][b] = A[a][0] * Ci[0][b] + A[a][1] * Ci[1][b];
    }
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            P[2 * a + b] = F[a][0] * S2[0][b] + F[a][1] * S2[1][b];
}

/* Stress of the bare moment chain as a function of H (Sect. 3.1):
 * Pi(H) = -mu (H + H^T + tr H I), row-major (xx, xy, yx, yy). */
void orc_lattice_Pi(double mu, const double H[4], double Pi[4])
{
    double tr = H[0] + H[3];
    Pi[0] = -(mu * (H[0] + H[0]) + mu * tr);
    Pi[1] = -(mu * (H[1] + H[2]));
    Pi[2] = -(mu * (H[2] + H[1]));
    Pi[3] = -(mu * (H[3] + H[3]) + mu * tr);
}

/* Time function of a boundary load at step n (step index as time). */
static double load_g(const side_t *s, double n)
{
    switch (s->kind) {
    case LOAD_ZERO: return 0.0;
    case LOAD_CONST: return 1.0;
    case LOAD_LINEAR_RAMP: return n < s->t1 ? n / s->t1 : 1.0;
    case LOAD_SIN2_RAMP: {
        if (n >= s->t1) return 1.0;
        double v = sin(M_PI * n / (2.0 * s->t1));
        return v * v;
    }
    case LOAD_SIN_PULSE: return n < s->t1 ? sin(M_PI * n / s->t1) : 0.0;
    case LOAD_GAUSS: {
        if (n > s->t1) return 0.0;
        double d = n - s->t0;
        return exp(-d * d / (2.0 * s->width * s->width));
    }
    case LOAD_RICKER: {
        if (n >= s->t1) return 0.0;
        double d2 = (n - s->t0) * (n - s->t0);
        double a = 2.0 / sqrt(3.0 * s->width * sqrt(M_PI));
        return a * (1.0 - d2 / s->width) * exp(-0.5 * d2 / s->width);
    }
    case LOAD_TABLE: {
        /* the sampled program, held at its last entry */
        if (!s->table || s->table_len < 1) return 0.0;
        int64_t k = (int64_t)n;
        return s->table[k < s->table_len ? k : s->table_len - 1];
    }
    default: return 0.0;
    }
}

/* Prescribed wall value at step n: j* for Dirichlet sides, T* for Neumann. */
static void side_value(const orc_t *h, int side, int64_t n, double out[2])
{
    const side_t *s = &h->side[side];
    if (s->kind == LOAD_DISP_RAMP) {
        /* a wall displacement amp reached at constant speed over t1 steps:
         * j* = rho0 times the wall speed for n < t1, then zero, since the method
         * prescribes the momentum j*, not the displacement */
        double k = (double)n < s->t1 ? h->rho0 / (s->t1 * h->dt) : 0.0;
        out[0] = s->amp[0] * k;
        out[1] = s->amp[1] * k;
        return;
    }
    double g = load_g(s, (double)n);
    out[0] = s->amp[0] * g;
    out[1] = s->amp[1] * g;
}

/* ---- lifetime ------------------------------------------------------------- */

static void *xcalloc(size_t n) { return calloc(n ? n : 1, sizeof(double)); }

void *orc_create(int nx, int ny, double dx, double rho0, double mu, double nu,
                 double tau, int material, double bx, double by)
{
    if (nx < 3 || ny < 3 || !(tau > 0.5) || !(mu > 0) || !(rho0 > 0) || !(dx > 0) ||
        !(nu > -1.0 && nu < 0.5) || material < 0 || material > 2)
        return NULL;
    orc_t *h = (orc_t *)calloc(1, sizeof(orc_t));
    h->nx = nx; h->ny = ny; h->dx = dx; h->rho0 = rho0; h->mu = mu; h->nu = nu;
    h->tau = tau; h->material = material; h->body[0] = bx; h->body[1] = by;
    h->threads = 1;
    h->boundary_order = 1;
    h->lam = orc_lambda(mu, nu);
    h->cs2 = mu / rho0;                        /* c_s = sqrt(mu/rho0), Sect. 3.1 */
    h->c = sqrt(3.0) * sqrt(h->cs2);           /* c = sqrt(3) c_s, Sect. 3.2 */
    h->dt = dx / h->c;                         /* c = dX/dt, Sect. 2 */
    h->omega = 1.0 / tau;                      /* dt/tau with tau in units of dt */
    for (int q = 0; q < 9; q++) {
        h->cq[q][0] = h->c * EX[q];
        h->cq[q][1] = h->c * EY[q];
    }
    for (int s = 0; s < 4; s++) {
        h->side[s].bc = BC_NEUMANN;
        h->side[s].kind = LOAD_ZERO;
    }
    size_t N = nn(h);
    h->f = xcalloc(9 * N); h->fc = xcalloc(9 * N); h->fn = xcalloc(9 * N);
    h->u = xcalloc(2 * N); h->un = xcalloc(2 * N); h->jA = xcalloc(2 * N);
    h->S = xcalloc(2 * N); h->T = xcalloc(4 * N);
    h->Sp = xcalloc(2 * N); h->Tp = xcalloc(4 * N);
    h->r = xcalloc(N); h->Pi = xcalloc(3 * N);
    return h;
}

void orc_destroy(void *hv)
{
    orc_t *h = (orc_t *)hv;
    if (!h) return;
    for (int k = 0; k < 4; k++) free(h->side[k].table);
    free(h->f); free(h->fc); free(h->fn); free(h->u); free(h->un); free(h->jA);
    free(h->S); free(h->T); free(h->Sp); free(h->Tp); free(h->r); free(h->Pi);
    free(h);
}

double orc_dt(void *hv) { return ((orc_t *)hv)->dt; }
int64_t orc_stepno(void *hv) { return ((orc_t *)hv)->n; }
void orc_set_threads(void *hv, int t) { ((orc_t *)hv)->threads = t > 0 ? t : 1; }
/* 0: zeroth-order wall values (default); 1: linear extrapolation. */
void orc_set_extrap_linear(void *hv, int on) { ((orc_t *)hv)->extrap_linear = on ? 1 : 0; }
/* 0: stresses at level n (default); 1: the printed order of Algorithm 1. */
void orc_set_listing_order(void *hv, int on) { ((orc_t *)hv)->listing_order = on ? 1 : 0; }

/* 1: first-order one-sided differences at the outermost nodes (Sect. 3.2, the
 * scheme's own); 2: second-order one-sided ones, the boundary stencils for which
 * the CFL discussion of Sect. 3.2 would admit nu <= 5/11 (an option). */
void orc_set_boundary_order(void *hv, int order) { ((orc_t *)hv)->boundary_order = order == 2 ? 2 : 1; }

/* The shear entry of the Pi_bd of a link that crosses two Neumann walls: 0 the
 * mean of the two walls' entries (default), 1 the x wall's, 2 the y wall's. */
void orc_set_corner(void *hv, int mode) { ((orc_t *)hv)->corner = (mode == 1 || mode == 2) ? mode : 0; }

/* tau_plus > 0.5: collide with two relaxation times (orc_collide_trt), the even
 * part at 1 / tau_plus; otherwise BGK. */
void orc_set_tau_plus(void *hv, double tau_plus) { ((orc_t *)hv)->omega_plus = tau_plus > 0.5 ? 1.0 / tau_plus : 0.0; }

int orc_set_side(void *hv, int side, int bc, int kind, double ax, double ay,
                 double t0, double t1, double width)
{
    orc_t *h = (orc_t *)hv;
    if (side < 0 || side > 3 || bc < 0 || bc > 2 || kind < 0 || kind > 8) return -1;
    if (kind == LOAD_DISP_RAMP && bc != BC_DIRICHLET) return -1;
    side_t *s = &h->side[side];
    s->bc = bc; s->kind = kind; s->amp[0] = ax; s->amp[1] = ay;
    s->t0 = t0; s->t1 = t1; s->width = width;
    return 0;
}

/* The sampled program of a TABLE side (copied; len >= 1). */
int orc_set_side_table(void *hv, int side, const double *table, int64_t len)
{
    orc_t *h = (orc_t *)hv;
    if (side < 0 || side > 3 || !table || len < 1) return -1;
    side_t *s = &h->side[side];
    free(s->table);
    s->table = (double *)malloc((size_t)len * sizeof(double));
    memcpy(s->table, table, (size_t)len * sizeof(double));
    s->table_len = len;
    return 0;
}

static int periodic_x(const orc_t *h) { return h->side[SIDE_LEFT].bc == BC_PERIODIC; }
static int periodic_y(const orc_t *h) { return h->side[SIDE_BOTTOM].bc == BC_PERIODIC; }

/* ---- finite differences, Sect. 3.2 ---------------------------------------- */

/* d v / d X_axis at node (x, y) of a scalar field v[ny][nx]. */
static double fd(const orc_t *h, const double *v, int x, int y, int axis)
{
    int L = axis == 0 ? h->nx : h->ny;
    int m = axis == 0 ? x : y;
    int per = axis == 0 ? periodic_x(h) : periodic_y(h);
    int mp, mm;
    double div;
    if (per) {
        mp = (m + 1) % L; mm = (m - 1 + L) % L; div = 2.0 * h->dx;
    } else if (m == 0 || m == L - 1) {
        /* one-sided: first order with the inward neighbour, or second order,
         * (-3 v_0 + 4 v_1 - v_2) / (2 dX) mirrored at the far side */
        int s = m == 0 ? 1 : -1;
#define AT(k) (axis == 0 ? v[IDX(h, m + s * (k), y)] : v[IDX(h, x, m + s * (k))])
        if (h->boundary_order == 2)
            return s * (-3.0 * AT(0) + 4.0 * AT(1) - AT(2)) / (2.0 * h->dx);
        return s * (AT(1) - AT(0)) / h->dx;
#undef AT
    } else {
        mp = m + 1; mm = m - 1; div = 2.0 * h->dx;
    }
    double vp = axis == 0 ? v[IDX(h, mp, y)] : v[IDX(h, x, mp)];
    double vm = axis == 0 ? v[IDX(h, mm, y)] : v[IDX(h, x, mm)];
    return (vp - vm) / div;
}

/* Stress pass (pass C of the algorithm): T = P(H) + Pi(H), H = grad u. */
static void stress_pass(orc_t *h, const double *u, double *T)
{
    size_t N = nn(h);
    int nx = h->nx, ny = h->ny;
#pragma omp parallel for num_threads(h->threads) schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            double H[4], P[4], Pl[4];
            H[0] = fd(h, u, x, y, 0);       /* d ux / dX */
            H[1] = fd(h, u, x, y, 1);       /* d ux / dY */
            H[2] = fd(h, u + N, x, y, 0);   /* d uy / dX */
            H[3] = fd(h, u + N, x, y, 1);   /* d uy / dY */
            orc_stress_P(h->material, h->lam, h->mu, H, P);
            orc_lattice_Pi(h->mu, H, Pl);
            for (int k = 0; k < 4; k++) T[k * N + IDX(h, x, y)] = P[k] + Pl[k];
        }
}

/* Source S_a = rho0 b_a + d_b T_ab, Eq. source. */
static void source_pass(orc_t *h, const double *T, double *S)
{
    size_t N = nn(h);
    int nx = h->nx, ny = h->ny;
#pragma omp parallel for num_threads(h->threads) schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t i = IDX(h, x, y);
            S[i] = h->rho0 * h->body[0] + (fd(h, T + 0 * N, x, y, 0) + fd(h, T + 1 * N, x, y, 1));
            S[N + i] = h->rho0 * h->body[1] + (fd(h, T + 2 * N, x, y, 0) + fd(h, T + 3 * N, x, y, 1));
        }
}

/* ---- initialisation --------------------------------------------------------- */

/* u0, j0: [2][ny][nx] host arrays (NULL means zero). */
void orc_init(void *hv, const double *u0, const double *j0)
{
    orc_t *h = (orc_t *)hv;
    size_t N = nn(h);
    for (size_t i = 0; i < 2 * N; i++) h->u[i] = u0 ? u0[i] : 0.0;
    for (int y = 0; y < h->ny; y++)
        for (int x = 0; x < h->nx; x++) {
            size_t i = IDX(h, x, y);
            double H[4], Pl[4], feq[9];
            H[0] = fd(h, h->u, x, y, 0); H[1] = fd(h, h->u, x, y, 1);
            H[2] = fd(h, h->u + N, x, y, 0); H[3] = fd(h, h->u + N, x, y, 1);
            orc_lattice_Pi(h->mu, H, Pl);
            double r0 = -h->rho0 * (H[0] + H[3]);
            double jj[2] = {j0 ? j0[i] : 0.0, j0 ? j0[N + i] : 0.0};
            double Pi3[3] = {Pl[0], Pl[1], Pl[3]};
            orc_feq(h->cs2, h->cq, r0, jj, Pi3, feq);
            for (int q = 0; q < 9; q++) h->f[q * N + i] = feq[q];
        }
    /* the printed order carries S and T of the previous level into the step */
    stress_pass(h, h->u, h->Tp);
    source_pass(h, h->Tp, h->Sp);
    h->n = 0;
}

/* ---- boundary momentum flux Pi_bd of one Neumann wall at node (x, y) ------ */

static void wall_Pi_bd(const orc_t *h, const double *T, int side, int x, int y, int64_t n,
                       double out[3])
{
    size_t N = nn(h);
    int a = (side == SIDE_LEFT || side == SIDE_RIGHT) ? 0 : 1;   /* normal axis */
    int b = 1 - a;                                                  /* tangential */
    double s = (side == SIDE_LEFT || side == SIDE_BOTTOM) ? -1.0 : 1.0;
    int xi = x - (a == 0 ? (int)s : 0), yi = y - (a == 1 ? (int)s : 0); /* inward */
    size_t i = IDX(h, x, y), ii = IDX(h, xi, yi);
    double Ts[2];
    side_value(h, side, n, Ts);
#define EXT(arr) (h->extrap_linear ? 0.5 * (3.0 * (arr)[i] - (arr)[ii]) : (arr)[i])
    /* T components: T_ab at offset (2a + b) * N */
    const double *T_aa = T + (size_t)(2 * a + a) * N;
    const double *T_ba = T + (size_t)(2 * b + a) * N;
    /* population Pi stored (xx, xy, yy): Pi_bb is xx for b = 0, yy for b = 1 */
    const double *Pi_bb = h->Pi + (size_t)(b == 0 ? 0 : 2) * N;
    double Paa = -s * Ts[a] + EXT(T_aa);
    double Pab = -s * Ts[b] + EXT(T_ba);
    double Pbb = EXT(Pi_bb);
#undef EXT
    double Pm[2][2];
    Pm[a][a] = Paa; Pm[a][b] = Pab; Pm[b][a] = Pab; Pm[b][b] = Pbb;
    out[0] = Pm[0][0]; out[1] = Pm[0][1]; out[2] = Pm[1][1];
}

/* ---- one time step ---------------------------------------------------------- */

static void step_once(orc_t *h)
{
    size_t N = nn(h);
    int nx = h->nx, ny = h->ny;
    int px = periodic_x(h), py = periodic_y(h);
    const double cs2 = h->cs2, dt = h->dt, om = h->omega;
    const int64_t n = h->n;
    /* S and T of the level the collision and the boundary rules use */
    const double *S, *T;
    if (h->listing_order) {
        S = h->Sp; T = h->Tp;
    } else {
        stress_pass(h, h->u, h->T);   /* stresses from u_n */
        source_pass(h, h->T, h->S);   /* S_n */
        S = h->S; T = h->T;
    }

    /* moments, equilibrium, forcing, BGK collision, streaming */
#pragma omp parallel for num_threads(h->threads) schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t i = IDX(h, x, y);
            double fl[9], fcl[9], r, jj[2], Pi3[3];
            for (int q = 0; q < 9; q++) fl[q] = h->f[q * N + i];
            double Sl[2] = {S[i], S[N + i]};
            if (h->omega_plus > 0)
                orc_collide_trt(cs2, h->cq, om, h->omega_plus, dt, fl, Sl, fcl, &r, jj, Pi3);
            else
                orc_collide(cs2, h->cq, om, dt, fl, Sl, fcl, &r, jj, Pi3);
            h->jA[i] = jj[0]; h->jA[N + i] = jj[1];
            h->r[i] = r;
            h->Pi[i] = Pi3[0]; h->Pi[N + i] = Pi3[1]; h->Pi[2 * N + i] = Pi3[2];
            for (int q = 0; q < 9; q++) h->fc[q * N + i] = fcl[q];
        }
#pragma omp parallel for num_threads(h->threads) schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++)
            for (int q = 0; q < 9; q++) {
                int xt = x + EX[q], yt = y + EY[q];
                if (px) xt = (xt + nx) % nx;
                if (py) yt = (yt + ny) % ny;
                if (xt < 0 || xt >= nx || yt < 0 || yt >= ny) continue; /* boundary rule */
                h->fn[q * N + IDX(h, xt, yt)] = h->fc[q * N + IDX(h, x, y)];
            }

    /* boundary nodes: Eq. bbcon (Dirichlet) and Eq. abbcon (Neumann) */
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            int wx = -1, wy = -1; /* walls the node lies on (non-periodic) */
            if (!px && x == 0) wx = SIDE_LEFT;
            if (!px && x == nx - 1) wx = SIDE_RIGHT;
            if (!py && y == 0) wy = SIDE_BOTTOM;
            if (!py && y == ny - 1) wy = SIDE_TOP;
            if (wx < 0 && wy < 0) continue;
            size_t i = IDX(h, x, y);
            double r = h->r[i];
            double PiX[3] = {0, 0, 0}, PiY[3] = {0, 0, 0}, PiC[3];
            if (wx >= 0 && h->side[wx].bc == BC_NEUMANN) wall_Pi_bd(h, T, wx, x, y, n, PiX);
            if (wy >= 0 && h->side[wy].bc == BC_NEUMANN) wall_Pi_bd(h, T, wy, x, y, n, PiY);
            PiC[0] = PiX[0]; PiC[2] = PiY[2];
            PiC[1] = h->corner == 1 ? PiX[1] : (h->corner == 2 ? PiY[1] : 0.5 * (PiX[1] + PiY[1]));
            for (int q = 1; q < 9; q++) {
                int xt = x + EX[q], yt = y + EY[q];
                int cx = !px && (xt < 0 || xt >= nx); /* crosses the x wall */
                int cy = !py && (yt < 0 || yt >= ny); /* crosses the y wall */
                if (!cx && !cy) continue;
                double fcq = h->fc[q * N + i];
                double cqx = h->cq[q][0], cqy = h->cq[q][1];
                int nd = 0;
                double js[2] = {0, 0};
                if (cx && h->side[wx].bc == BC_DIRICHLET) {
                    double v[2]; side_value(h, wx, n, v);
                    js[0] += v[0]; js[1] += v[1]; nd++;
                }
                if (cy && h->side[wy].bc == BC_DIRICHLET) {
                    double v[2]; side_value(h, wy, n, v);
                    js[0] += v[0]; js[1] += v[1]; nd++;
                }
                double val;
                if (nd > 0) {
                    js[0] /= nd; js[1] /= nd;
                    /* modified bounce-back, Eq. bbcon */
                    val = fcq - 2.0 / cs2 * W[q] * (cqx * js[0] + cqy * js[1]);
                } else {
                    /* modified anti-bounce-back, Eq. abbcon */
                    const double *Pb = (cx && cy) ? PiC : (cx ? PiX : PiY);
                    double Axx = Pb[0] - r * cs2, Axy = Pb[1], Ayy = Pb[2] - r * cs2;
                    double contr = Axx * (cqx * cqx - cs2) + 2.0 * Axy * (cqx * cqy) +
                                   Ayy * (cqy * cqy - cs2);
                    val = -fcq + 2.0 * W[q] * (r + contr / (2.0 * cs2 * cs2));
                }
                h->fn[OPP[q] * N + i] = val;
            }
        }

    if (h->listing_order) {
        /* the printed order: stresses from u_n after streaming; S_n feeds the
         * moment j(t_{n+1}) below and the next collision */
        stress_pass(h, h->u, h->Tp);
        source_pass(h, h->Tp, h->Sp);
        S = h->Sp;
    }
    /* moments of f(t_{n+1}) and the trapezoidal displacement update */
#pragma omp parallel for num_threads(h->threads) schedule(static)
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            size_t i = IDX(h, x, y);
            double mx = 0, my = 0;
            for (int q = 0; q < 9; q++) {
                mx += h->cq[q][0] * h->fn[q * N + i];
                my += h->cq[q][1] * h->fn[q * N + i];
            }
            double jx = mx + 0.5 * dt * S[i], jy = my + 0.5 * dt * S[N + i];
            h->un[i] = h->u[i] + dt / (2.0 * h->rho0) * (jx + h->jA[i]);
            h->un[N + i] = h->u[N + i] + dt / (2.0 * h->rho0) * (jy + h->jA[N + i]);
        }
    double *t;
    t = h->f; h->f = h->fn; h->fn = t;
    t = h->u; h->u = h->un; h->un = t;
    h->n = n + 1;
}

void orc_step(void *hv, int64_t nsteps)
{
    for (int64_t k = 0; k < nsteps; k++) step_once((orc_t *)hv);
}

/* ---- read-out ----------------------------------------------------------- */

/* S of the level the next collision uses, [2][ny][nx]. */
static void current_S(orc_t *h, double *out)
{
    size_t N = nn(h);
    if (h->listing_order) {
        memcpy(out, h->Sp, 2 * N * sizeof(double));
        return;
    }
    double *T = (double *)malloc(4 * N * sizeof(double));
    stress_pass(h, h->u, T);
    source_pass(h, T, out);
    free(T);
}

/* Fields at t_n, [comp][ny][nx]:
 *   U (2) = u_n; J (2) = sum c f(t_n) + dt/2 S, with the S the collision at t_n
 *   uses; R (1) = sum f; PI (3: xx, xy, yy) = sum c c f; H (4) and P (4) from
 *   u_n; S (2) = rho0 b + Div(P + Pi(H)) from u_n. */
int orc_read(void *hv, int field, double *out)
{
    orc_t *h = (orc_t *)hv;
    size_t N = nn(h);
    switch (field) {
    case FIELD_U: memcpy(out, h->u, 2 * N * sizeof(double)); return 0;
    case FIELD_J: {
        double *S = (double *)malloc(2 * N * sizeof(double));
        current_S(h, S);
        for (size_t i = 0; i < N; i++) {
            double mx = 0, my = 0;
            for (int q = 0; q < 9; q++) {
                mx += h->cq[q][0] * h->f[q * N + i];
                my += h->cq[q][1] * h->f[q * N + i];
            }
            out[i] = mx + 0.5 * h->dt * S[i];
            out[N + i] = my + 0.5 * h->dt * S[N + i];
        }
        free(S);
        return 0;
    }
    case FIELD_R:
    case FIELD_PI:
        for (size_t i = 0; i < N; i++) {
            double r = 0, pxx = 0, pxy = 0, pyy = 0;
            for (int q = 0; q < 9; q++) {
                double fq = h->f[q * N + i];
                r += fq;
                pxx += h->cq[q][0] * h->cq[q][0] * fq;
                pxy += h->cq[q][0] * h->cq[q][1] * fq;
                pyy += h->cq[q][1] * h->cq[q][1] * fq;
            }
            if (field == FIELD_R) out[i] = r;
            else { out[i] = pxx; out[N + i] = pxy; out[2 * N + i] = pyy; }
        }
        return 0;
    case FIELD_H:
    case FIELD_P:
        for (int y = 0; y < h->ny; y++)
            for (int x = 0; x < h->nx; x++) {
                size_t i = IDX(h, x, y);
                double H[4], P[4];
                H[0] = fd(h, h->u, x, y, 0); H[1] = fd(h, h->u, x, y, 1);
                H[2] = fd(h, h->u + N, x, y, 0); H[3] = fd(h, h->u + N, x, y, 1);
                if (field == FIELD_P) orc_stress_P(h->material, h->lam, h->mu, H, P);
                for (int k = 0; k < 4; k++) out[k * N + i] = field == FIELD_H ? H[k] : P[k];
            }
        return 0;
    case FIELD_S: {
        double *T = (double *)malloc(4 * N * sizeof(double));
        stress_pass(h, h->u, T);
        source_pass(h, T, out);
        free(T);
        return 0;
    }
    default: return -1;
    }
}

/* Pre-collision populations f(t_n), [9][ny][nx]. */
void orc_read_f(void *hv, double *out)
{
    orc_t *h = (orc_t *)hv;
    memcpy(out, h->f, 9 * nn(h) * sizeof(double));
}

/* Set the state at the start of the current step directly: the pre-collision
 * populations f(t_n) [9][ny][nx] and u_n [2][ny][nx] (either may be NULL to keep
 * it).  For the linear analysis of the step (its matrix, column by column). */
void orc_set_state(void *hv, const double *f, const double *u)
{
    orc_t *h = (orc_t *)hv;
    size_t N = nn(h);
    if (f) memcpy(h->f, f, 9 * N * sizeof(double));
    if (u) memcpy(h->u, u, 2 * N * sizeof(double));
}

/* The printed order's extra state: S_{n-1} [2][ny][nx] and T_{n-1} [4][ny][nx]
 * (read or set; NULL skips). */
void orc_get_prev(void *hv, double *Sp, double *Tp)
{
    orc_t *h = (orc_t *)hv;
    size_t N = nn(h);
    if (Sp) memcpy(Sp, h->Sp, 2 * N * sizeof(double));
    if (Tp) memcpy(Tp, h->Tp, 4 * N * sizeof(double));
}

void orc_set_prev(void *hv, const double *Sp, const double *Tp)
{
    orc_t *h = (orc_t *)hv;
    size_t N = nn(h);
    if (Sp) memcpy(h->Sp, Sp, 2 * N * sizeof(double));
    if (Tp) memcpy(h->Tp, Tp, 4 * N * sizeof(double));
}

/* Total population momentum sum_X sum_q c_q f_q(t_n). */
void orc_momentum(void *hv, double out[2])
{
    orc_t *h = (orc_t *)hv;
    size_t N = nn(h);
    double mx = 0, my = 0;
    for (size_t i = 0; i < N; i++)
        for (int q = 0; q < 9; q++) {
            mx += h->cq[q][0] * h->f[q * N + i];
            my += h->cq[q][1] * h->f[q * N + i];
        }
    out[0] = mx; out[1] = my;
}

/* Wall value (j* or T*) of a side at step n, as the boundary pass uses it. */
void orc_side_value(void *hv, int side, int64_t n, double out[2])
{
    side_value((orc_t *)hv, side, n, out);
}

/* Diagnostics at t_n: sum_X j, sum_X |j|^2/(2 rho0), max |u|, non-finite flag,
 * with j as orc_read returns it. */
void orc_diag(void *hv, double out[5])
{
    orc_t *h = (orc_t *)hv;
    size_t N = nn(h);
    double *j = (double *)malloc(2 * N * sizeof(double));
    orc_read(hv, FIELD_J, j);
    double sx = 0, sy = 0, ek = 0, mu2 = 0, bad = 0;
    for (size_t i = 0; i < N; i++) {
        double jx = j[i], jy = j[N + i], ux = h->u[i], uy = h->u[N + i];
        sx += jx; sy += jy;
        ek += (jx * jx + jy * jy) / (2.0 * h->rho0);
        double m = ux * ux + uy * uy;
        if (m > mu2) mu2 = m;
        if (!isfinite(jx) || !isfinite(jy) || !isfinite(ux) || !isfinite(uy)) bad = 1;
    }
    free(j);
    out[0] = sx; out[1] = sy; out[2] = ek; out[3] = sqrt(mu2); out[4] = bad;
}
