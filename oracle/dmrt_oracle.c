/*
 * dmrt_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU implementation of the double-MRT thermal
 * lattice Boltzmann step of Li, Yang & Zhang, "Double MRT Thermal Lattice
 * Boltzmann Method for Simulating Natural Convection of Low Prandtl Number
 * Fluids" (arXiv:1601.04633).  It exists to check the GPU library against.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never does.  It shares no code,
 * header, table or generator with the GPU library.
 *
 * Deliberately naive structure, so that it can be read against the paper:
 *   - array-of-structures state, pre-collision f(t), g(t);
 *   - the collision is a dense 9x9 (5x5) matrix-vector product with M (N)
 *     typed from Eq. 30 (Eq. 37), the inverse obtained numerically by
 *     Gauss-Jordan elimination;
 *   - the body force is added in distribution space, Eq. 26;
 *   - streaming pushes every post-collision population into a fresh array,
 *     then a separate pass handles the links that left the domain
 *     (halfway bounce-back, Eqs. 44-45).
 *
 * Readings taken where the paper is garbled or silent (each one is tested):
 *   R1  Eq. 34: the energy moment equilibrium is -2 drho + 3 rho0 |u|^2
 *       (the printed formula lacks the factor 3).
 *   R2  Eq. 37: the fifth row of N is (0, 1, -1, 1, -1); the printed last
 *       entry +1 makes the rows non-orthogonal and removes x-diffusion.
 *   R3  Eq. 26: the divisor is rho0 c_s^2 = 1/3 and f^eq is the rho0-based
 *       second-order equilibrium, so F_i = 3 G.(e_i - u) f_i^eq(rho0, u).
 *   R4  Eq. 27: G = (force_x, gbeta (theta - theta_ref)); theta is stored
 *       shifted so that the walls sit at +-0.5 and theta_ref defaults to 0.
 *   R5  Eqs. 40/43: with Ma = 0.1 the literal Eq. 40 forces a > 1, which the
 *       paper itself rules out.  Mode 0 keeps a fixed and solves Eq. 43 for
 *       sigma_k, with sigma_e = sigma_nu from Eq. 39.  Mode 1 is Eq. 40
 *       literally with a = 20 sqrt(3) alpha - 4, rejected unless -4 < a < 1.
 *   R6  Eq. 45: the anti-bounce-back constant is (4 + a)/10 theta_w, which
 *       equals the printed 2 sqrt(3) alpha theta_w when Eq. 40 holds.
 *   R7  Eq. 18: the wall gradient is the second-order one-sided difference
 *       through the wall value and the first two node centres.
 *
 * Besides the double MRT scheme the oracle runs the double LBGK scheme the
 * paper's introduction contrasts it with (one relaxation time for f and
 * one for g, He et al.'s double-distribution approach): the collision is
 * then done in distribution space, f* = f - (f - f^eq)/tau_f + F and
 * g* = g - (g - g^eq)/tau_g, with the textbook second-order equilibria and
 * 1/tau_f = s_nu (Eq. 32's viscosity relation), 1/tau_g = sigma_k (Eq. 43's
 * diffusivity relation).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_CAVITY = 0, ORC_PERIODIC = 1, ORC_CHANNEL_X = 2, ORC_ADIABATIC_BOX = 3 };
enum { ORC_Q5_FIXED_A = 0, ORC_Q5_PAPER = 1 };
enum { ORC_MRT = 0, ORC_LBGK = 1 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_EUNSTABLE = -2, ORC_ENOMEM = -3 };

typedef struct {
    int n;                       /* nodes per side; walls half a link outside */
    int bc;
    int collision;               /* ORC_MRT or ORC_LBGK */
    double rho0;
    /* physical parameters in lattice units */
    double H, nu, alpha, gbeta, force_x, theta_ref;
    double theta_hot, theta_cold;
    double a;                    /* D2Q5 equilibrium parameter, Eq. 42 */
    double S[9], Q[5];           /* Eqs. 31, 38 */
    double M[9][9], Minv[9][9];  /* Eq. 30 and its numerical inverse */
    double N[5][5], Ninv[5][5];  /* Eq. 37 (R2) and its numerical inverse */
    int e[9][2];                 /* Eq. 23 */
    int c5[5][2];                /* Eq. 35 */
    int opp9[9], opp5[5];
    double *theta_w;             /* hot-wall temperature per row */
    double *f, *g;               /* pre-collision state, AoS */
    double *fs, *gs;             /* post-collision state */
    double *fn, *gn;             /* streamed state */
    long steps;
} orc_t;

/* ---------------------------------------------------------------------- */
/* Parameter map: Eq. 9 with Eqs. 11-13 (lattice units, c = 1, c_s^2 = 1/3) */
/* out[12] = nu, alpha, gbeta, s_nu, s_q, sigma_k, sigma_e, sigma_nu, a,   */
/*           w0 (D2Q5 rest weight), wm (D2Q5 moving weight), H            */
/* ---------------------------------------------------------------------- */
int orc_derive(int n, double Ra, double Pr, double Ma, double theta_hot,
               double theta_cold, int q5_mode, double a_fixed,
               double gbeta_override, int collision, double *out)
{
    if (n < 2 || !out) return ORC_EINVAL;
    if (collision != ORC_MRT && collision != ORC_LBGK) return ORC_EINVAL;
    if (!isfinite(Ra) || !isfinite(Pr) || !isfinite(Ma) || !isfinite(theta_hot) ||
        !isfinite(theta_cold))
        return ORC_EINVAL;
    if (Ra <= 0.0 || Pr <= 0.0 || Ma <= 0.0) return ORC_EUNSTABLE;
    double H = (double)n;                    /* halfway walls at 0 and n */
    double dT = theta_hot - theta_cold;
    /* Ma = u_c / c_s with u_c^2 = g beta dT H, c_s^2 = 1/3  (Eq. 9) */
    double gbeta;
    if (isnan(gbeta_override)) {
        if (!(dT > 0.0)) return ORC_EINVAL;
        gbeta = Ma * Ma / 3.0 / H / dT;
    } else {
        gbeta = gbeta_override;
    }
    /* Eq. 11: nu / (c H) = Ma sqrt(Pr / (3 Ra));  Eq. 13: alpha = nu / Pr */
    double nu = Ma * H * sqrt(Pr / (3.0 * Ra));
    double alpha = nu / Pr;
    /* Eq. 32 */
    double s_nu = 2.0 / (6.0 * nu + 1.0);
    double s_q = 8.0 * (2.0 - s_nu) / (8.0 - s_nu);
    double a, sk, se, sn;
    if (q5_mode == ORC_Q5_PAPER) {
        /* Eq. 40 literally, then Eq. 43 solved for a */
        sk = 1.0 / (0.5 + sqrt(3.0) / 6.0);
        se = sn = 1.0 / (0.5 + sqrt(3.0) / 3.0);
        a = 10.0 * alpha / (1.0 / sk - 0.5) - 4.0;
    } else if (q5_mode == ORC_Q5_FIXED_A) {
        a = a_fixed;
        if (!isfinite(a)) return ORC_EINVAL;
        if (!(a > -4.0)) return ORC_EUNSTABLE;
        /* Eq. 43 solved for sigma_k, then Eq. 39 for sigma_nu = sigma_e */
        double lam_k = alpha * 10.0 / (4.0 + a);
        sk = 1.0 / (0.5 + lam_k);
        se = sn = 1.0 / (0.5 + 1.0 / (6.0 * lam_k));
    } else {
        return ORC_EINVAL;
    }
    if (collision == ORC_LBGK) {
        /* one relaxation time per distribution: every non-conserved moment
         * relaxes at the viscous rate (f) or at the diffusive rate (g) */
        s_q = s_nu;
        se = sn = sk;
    }
    if (!(a > -4.0 && a < 1.0)) return ORC_EUNSTABLE;   /* stability: a < 1 */
    double rel[5] = { s_nu, s_q, sk, se, sn };
    for (int k = 0; k < 5; ++k)
        if (!(rel[k] > 0.0 && rel[k] < 2.0)) return ORC_EUNSTABLE;
    out[0] = nu; out[1] = alpha; out[2] = gbeta; out[3] = s_nu; out[4] = s_q;
    out[5] = sk; out[6] = se; out[7] = sn; out[8] = a;
    out[9] = (1.0 - a) / 5.0; out[10] = (4.0 + a) / 20.0; out[11] = H;
    return ORC_OK;
}

/* Gauss-Jordan inversion with partial pivoting of an n x n matrix (n <= 9). */
static int invert(int n, const double *A, double *Ainv)
{
    double w[9][18];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            w[r][c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(w[r][col]) > fabs(w[piv][col])) piv = r;
        if (w[piv][col] == 0.0) return ORC_EINVAL;
        if (piv != col)
            for (int c = 0; c < 2 * n; ++c) {
                double t = w[col][c]; w[col][c] = w[piv][c]; w[piv][c] = t;
            }
        double d = w[col][col];
        for (int c = 0; c < 2 * n; ++c) w[col][c] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double fct = w[r][col];
            if (fct == 0.0) continue;
            for (int c = 0; c < 2 * n; ++c) w[r][c] -= fct * w[col][c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r * n + c] = w[r][n + c];
    return ORC_OK;
}

static void setup_lattice(orc_t *s)
{
    /* Eq. 23 (1-based i in the paper; 0-based here), c = 1 */
    const double pi = acos(-1.0);
    s->e[0][0] = 0; s->e[0][1] = 0;
    for (int i = 2; i <= 5; ++i) {
        s->e[i - 1][0] = (int)lround(-cos(i * pi / 2.0));
        s->e[i - 1][1] = (int)lround(-sin(i * pi / 2.0));
    }
    for (int i = 6; i <= 9; ++i) {
        s->e[i - 1][0] = (int)lround(sqrt(2.0) * -cos((2 * i + 1) * pi / 4.0));
        s->e[i - 1][1] = (int)lround(sqrt(2.0) * -sin((2 * i + 1) * pi / 4.0));
    }
    /* Eq. 35: the first five D2Q9 directions */
    for (int i = 0; i < 5; ++i) { s->c5[i][0] = s->e[i][0]; s->c5[i][1] = s->e[i][1]; }
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j)
            if (s->e[j][0] == -s->e[i][0] && s->e[j][1] == -s->e[i][1]) s->opp9[i] = j;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j)
            if (s->c5[j][0] == -s->c5[i][0] && s->c5[j][1] == -s->c5[i][1]) s->opp5[i] = j;

    /* Eq. 30 */
    static const double M[9][9] = {
        {  1,  1,  1,  1,  1,  1,  1,  1,  1 },
        {  0,  1,  0, -1,  0,  1, -1, -1,  1 },
        {  0,  0,  1,  0, -1,  1,  1, -1, -1 },
        { -4, -1, -1, -1, -1,  2,  2,  2,  2 },
        {  0,  1, -1,  1, -1,  0,  0,  0,  0 },
        {  0,  0,  0,  0,  0,  1, -1,  1, -1 },
        {  0, -2,  0,  2,  0,  1, -1, -1,  1 },
        {  0,  0, -2,  0,  2,  1,  1, -1, -1 },
        {  4, -2, -2, -2, -2,  1,  1,  1,  1 },
    };
    /* Eq. 37 with reading R2 for the last row */
    static const double N[5][5] = {
        {  1,  1,  1,  1,  1 },
        {  0,  1,  0, -1,  0 },
        {  0,  0,  1,  0, -1 },
        { -4,  1,  1,  1,  1 },
        {  0,  1, -1,  1, -1 },
    };
    memcpy(s->M, M, sizeof M);
    memcpy(s->N, N, sizeof N);
    invert(9, &s->M[0][0], &s->Minv[0][0]);
    invert(5, &s->N[0][0], &s->Ninv[0][0]);
}

void orc_destroy(orc_t *s)
{
    if (!s) return;
    free(s->theta_w); free(s->f); free(s->g); free(s->fs); free(s->gs);
    free(s->fn); free(s->gn); free(s);
}

orc_t *orc_create(int n, double Ra, double Pr, double Ma, double theta_hot,
                  double theta_cold, int q5_mode, double a_fixed, int bc,
                  double gbeta_override, double force_x, double theta_ref,
                  int collision, int *err)
{
    double d[12];
    int rc = orc_derive(n, Ra, Pr, Ma, theta_hot, theta_cold, q5_mode, a_fixed,
                        gbeta_override, collision, d);
    if (rc == ORC_OK && (bc < 0 || bc > 3 || !isfinite(force_x) || !isfinite(theta_ref)))
        rc = ORC_EINVAL;
    if (rc != ORC_OK) { if (err) *err = rc; return NULL; }
    orc_t *s = (orc_t *)calloc(1, sizeof(orc_t));
    if (!s) { if (err) *err = ORC_ENOMEM; return NULL; }
    s->n = n; s->bc = bc; s->rho0 = 1.0; s->collision = collision;
    s->nu = d[0]; s->alpha = d[1]; s->gbeta = d[2]; s->a = d[8]; s->H = d[11];
    s->force_x = force_x; s->theta_ref = theta_ref;
    s->theta_hot = theta_hot; s->theta_cold = theta_cold;
    /* Eq. 31: S = diag(0, 1, 1, s_e, s_nu, s_nu, s_q, s_q, s_eps), s_e = s_eps = s_nu */
    double Sv[9] = { 0.0, 1.0, 1.0, d[3], d[3], d[3], d[4], d[4], d[3] };
    /* Eq. 38: Q = diag(0, sigma_k, sigma_k, sigma_e, sigma_nu) */
    double Qv[5] = { 0.0, d[5], d[5], d[6], d[7] };
    memcpy(s->S, Sv, sizeof Sv);
    memcpy(s->Q, Qv, sizeof Qv);
    setup_lattice(s);
    size_t nn = (size_t)n * n;
    s->theta_w = (double *)malloc(n * sizeof(double));
    s->f = (double *)calloc(nn * 9, sizeof(double));
    s->g = (double *)calloc(nn * 5, sizeof(double));
    s->fs = (double *)calloc(nn * 9, sizeof(double));
    s->gs = (double *)calloc(nn * 5, sizeof(double));
    s->fn = (double *)calloc(nn * 9, sizeof(double));
    s->gn = (double *)calloc(nn * 5, sizeof(double));
    if (!s->theta_w || !s->f || !s->g || !s->fs || !s->gs || !s->fn || !s->gn) {
        orc_destroy(s);
        if (err) *err = ORC_ENOMEM;
        return NULL;
    }
    for (int y = 0; y < n; ++y) s->theta_w[y] = theta_hot;
    if (err) *err = ORC_OK;
    return s;
}

int orc_derived(const orc_t *s, double *out)
{
    /* nu, alpha, gbeta, S[0..8], Q[0..4], a */
    out[0] = s->nu; out[1] = s->alpha; out[2] = s->gbeta;
    for (int k = 0; k < 9; ++k) out[3 + k] = s->S[k];
    for (int k = 0; k < 5; ++k) out[12 + k] = s->Q[k];
    out[17] = s->a;
    return ORC_OK;
}

int orc_matrices(const orc_t *s, double *M, double *Minv, double *N, double *Ninv,
                 int *e9, int *e5)
{
    memcpy(M, s->M, sizeof s->M);
    memcpy(Minv, s->Minv, sizeof s->Minv);
    memcpy(N, s->N, sizeof s->N);
    memcpy(Ninv, s->Ninv, sizeof s->Ninv);
    for (int i = 0; i < 9; ++i) { e9[2 * i] = s->e[i][0]; e9[2 * i + 1] = s->e[i][1]; }
    for (int i = 0; i < 5; ++i) { e5[2 * i] = s->c5[i][0]; e5[2 * i + 1] = s->c5[i][1]; }
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Equilibria, Eq. 34 (R1) and Eq. 42                                      */
/* ---------------------------------------------------------------------- */
static void meq9(const orc_t *s, double drho, double u, double v, double *meq)
{
    double r0 = s->rho0, uu = u * u + v * v;
    meq[0] = drho;
    meq[1] = r0 * u;
    meq[2] = r0 * v;
    meq[3] = -2.0 * drho + 3.0 * r0 * uu;   /* R1 */
    meq[4] = r0 * (u * u - v * v);
    meq[5] = r0 * u * v;
    meq[6] = -r0 * u;
    meq[7] = -r0 * v;
    meq[8] = drho - 3.0 * r0 * uu;
}

static void neq5(const orc_t *s, double theta, double u, double v, double *neq)
{
    neq[0] = theta;
    neq[1] = u * theta;
    neq[2] = v * theta;
    neq[3] = s->a * theta;
    neq[4] = 0.0;
}

static void matvec(int n, const double *A, const double *x, double *y)
{
    for (int r = 0; r < n; ++r) {
        double acc = 0.0;
        for (int c = 0; c < n; ++c) acc += A[r * n + c] * x[c];
        y[r] = acc;
    }
}

/* Distribution-space equilibria: f^eq = M^-1 m^eq, g^eq = N^-1 n^eq */
static void feq9(const orc_t *s, double drho, double u, double v, double *feq)
{
    double meq[9];
    meq9(s, drho, u, v, meq);
    matvec(9, &s->Minv[0][0], meq, feq);
}

static void geq5(const orc_t *s, double theta, double u, double v, double *geq)
{
    double neq[5];
    neq5(s, theta, u, v, neq);
    matvec(5, &s->Ninv[0][0], neq, geq);
}

/* Eq. 26 with reading R3.  The rho0-based full equilibrium is M^-1 m^eq with
 * the density moment set to rho0 (m^eq is affine in the density moment).     */
int orc_force(const orc_t *s, double Gx, double Gy, double u, double v, double *F)
{
    double feq[9];
    feq9(s, s->rho0, u, v, feq);
    const double cs2 = 1.0 / 3.0;
    for (int i = 0; i < 9; ++i) {
        double gdot = Gx * (s->e[i][0] - u) + Gy * (s->e[i][1] - v);
        F[i] = gdot / (s->rho0 * cs2) * feq[i];
    }
    return ORC_OK;
}

/* One node: pre-collision f[9], g[5] -> post-collision fs[9], gs[5]. */
/* Double LBGK collision in distribution space.  The D2Q9 equilibrium is the
 * second-order polynomial w_i [drho + rho0 (3 e.u + 9/2 (e.u)^2 - 3/2 u^2)]
 * (f stored as the deviation from w_i rho0, as in Eq. 33); the D2Q5 one is
 * w_i theta + theta (c_i.u)/2, whose moments are those of Eq. 42. */
static void collide_lbgk(const orc_t *s, const double *f, const double *g, double *fs, double *gs)
{
    static const double w9[9] = { 4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36 };
    double drho = 0.0, jx = 0.0, jy = 0.0, theta = 0.0;
    for (int i = 0; i < 9; ++i) {
        drho += f[i];
        jx += s->e[i][0] * f[i];
        jy += s->e[i][1] * f[i];
    }
    for (int i = 0; i < 5; ++i) theta += g[i];
    double u = jx / s->rho0, v = jy / s->rho0, uu = u * u + v * v;
    double omega_f = s->S[4], omega_g = s->Q[1];
    double F[9];
    orc_force(s, s->force_x, s->gbeta * (theta - s->theta_ref), u, v, F);
    for (int i = 0; i < 9; ++i) {
        double eu = s->e[i][0] * u + s->e[i][1] * v;
        double feq = w9[i] * (drho + s->rho0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
        fs[i] = f[i] - omega_f * (f[i] - feq) + F[i];
    }
    double w0 = (1.0 - s->a) / 5.0, wm = (4.0 + s->a) / 20.0;
    for (int i = 0; i < 5; ++i) {
        double cu = s->c5[i][0] * u + s->c5[i][1] * v;
        double geq = (i == 0 ? w0 : wm) * theta + 0.5 * theta * cu;
        gs[i] = g[i] - omega_g * (g[i] - geq);
    }
}

/* Test hook: replace the relaxation rates of Eqs. 31 and 38. */
int orc_set_rates(orc_t *s, const double *S9, const double *Q5)
{
    memcpy(s->S, S9, sizeof s->S);
    memcpy(s->Q, Q5, sizeof s->Q);
    return ORC_OK;
}

int orc_collide(const orc_t *s, const double *f, const double *g, double *fs, double *gs)
{
    double m[9], meq[9], mst[9], n5[5], neq[5], nst[5], F[9];
    if (s->collision == ORC_LBGK) {
        collide_lbgk(s, f, g, fs, gs);
        return ORC_OK;
    }
    /* Eq. 33 and Eq. 41 */
    matvec(9, &s->M[0][0], f, m);
    double drho = m[0];
    double u = m[1] / s->rho0, v = m[2] / s->rho0;
    double theta = 0.0;
    for (int i = 0; i < 5; ++i) theta += g[i];
    /* Eq. 28 */
    meq9(s, drho, u, v, meq);
    for (int k = 0; k < 9; ++k) mst[k] = m[k] - s->S[k] * (m[k] - meq[k]);
    matvec(9, &s->Minv[0][0], mst, fs);
    /* Eqs. 26-27 */
    double Gx = s->force_x, Gy = s->gbeta * (theta - s->theta_ref);
    orc_force(s, Gx, Gy, u, v, F);
    for (int i = 0; i < 9; ++i) fs[i] += F[i];
    /* Eq. 36 */
    matvec(5, &s->N[0][0], g, n5);
    neq5(s, theta, u, v, neq);
    for (int k = 0; k < 5; ++k) nst[k] = n5[k] - s->Q[k] * (n5[k] - neq[k]);
    matvec(5, &s->Ninv[0][0], nst, gs);
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* State                                                                   */
/* ---------------------------------------------------------------------- */
int orc_set_equilibrium(orc_t *s, const double *drho, const double *U, const double *V,
                        const double *theta)
{
    size_t nn = (size_t)s->n * s->n;
    for (size_t k = 0; k < nn; ++k) {
        double r = drho ? drho[k] : 0.0, u = U ? U[k] : 0.0, v = V ? V[k] : 0.0;
        double th = theta ? theta[k] : 0.0;
        if (!isfinite(r) || !isfinite(u) || !isfinite(v) || !isfinite(th)) return ORC_EINVAL;
        feq9(s, r, u, v, &s->f[9 * k]);
        geq5(s, th, u, v, &s->g[5 * k]);
    }
    s->steps = 0;
    return ORC_OK;
}

int orc_set_hot_wall(orc_t *s, const double *theta_w)
{
    for (int y = 0; y < s->n; ++y) {
        if (!isfinite(theta_w[y])) return ORC_EINVAL;
        s->theta_w[y] = theta_w[y];
    }
    return ORC_OK;
}

int orc_get_state(const orc_t *s, double *f, double *g)
{
    size_t nn = (size_t)s->n * s->n;
    if (f) memcpy(f, s->f, nn * 9 * sizeof(double));
    if (g) memcpy(g, s->g, nn * 5 * sizeof(double));
    return ORC_OK;
}

int orc_set_state(orc_t *s, const double *f, const double *g)
{
    size_t nn = (size_t)s->n * s->n;
    if (f) memcpy(s->f, f, nn * 9 * sizeof(double));
    if (g) memcpy(s->g, g, nn * 5 * sizeof(double));
    return ORC_OK;
}

long orc_steps(const orc_t *s) { return s->steps; }

/* ---------------------------------------------------------------------- */
/* One time step: collide every node, push-stream, then the wall pass.     */
/* ---------------------------------------------------------------------- */
static int periodic_x(const orc_t *s) { return s->bc == ORC_PERIODIC || s->bc == ORC_CHANNEL_X; }
static int periodic_y(const orc_t *s) { return s->bc == ORC_PERIODIC; }

static void step_once(orc_t *s)
{
    const int n = s->n;
    const size_t nn = (size_t)n * n;
    /* collision (Eqs. 25, 36, right-hand sides) */
    for (size_t k = 0; k < nn; ++k)
        orc_collide(s, &s->f[9 * k], &s->g[5 * k], &s->fs[9 * k], &s->gs[5 * k]);

    /* streaming into the fresh arrays (left-hand sides of Eqs. 25, 36) */
    for (size_t k = 0; k < nn * 9; ++k) s->fn[k] = NAN;
    for (size_t k = 0; k < nn * 5; ++k) s->gn[k] = NAN;
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
            size_t k = (size_t)y * n + x;
            for (int i = 0; i < 9; ++i) {
                int tx = x + s->e[i][0], ty = y + s->e[i][1];
                if (periodic_x(s)) tx = (tx + n) % n;
                if (periodic_y(s)) ty = (ty + n) % n;
                if (tx >= 0 && tx < n && ty >= 0 && ty < n)
                    s->fn[9 * ((size_t)ty * n + tx) + i] = s->fs[9 * k + i];
            }
            for (int i = 0; i < 5; ++i) {
                int tx = x + s->c5[i][0], ty = y + s->c5[i][1];
                if (periodic_x(s)) tx = (tx + n) % n;
                if (periodic_y(s)) ty = (ty + n) % n;
                if (tx >= 0 && tx < n && ty >= 0 && ty < n)
                    s->gn[5 * ((size_t)ty * n + tx) + i] = s->gs[5 * k + i];
            }
        }

    /* wall pass: every link that left the domain returns to its own node
     * reversed (halfway bounce-back for f; Eq. 44 for g on adiabatic walls,
     * Eq. 45 with reading R6 on the isothermal left and right walls)       */
    const double wm2 = (4.0 + s->a) / 10.0;
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
            size_t k = (size_t)y * n + x;
            for (int i = 0; i < 9; ++i) {
                int tx = x + s->e[i][0], ty = y + s->e[i][1];
                int out = (!periodic_x(s) && (tx < 0 || tx >= n)) ||
                          (!periodic_y(s) && (ty < 0 || ty >= n));
                if (out) s->fn[9 * k + s->opp9[i]] = s->fs[9 * k + i];
            }
            for (int i = 0; i < 5; ++i) {
                int tx = x + s->c5[i][0], ty = y + s->c5[i][1];
                int out_x = !periodic_x(s) && (tx < 0 || tx >= n);
                int out_y = !periodic_y(s) && (ty < 0 || ty >= n);
                if (!out_x && !out_y) continue;
                double val = s->gs[5 * k + i];
                double res;
                if (out_x && s->bc == ORC_CAVITY) {
                    double thw = tx < 0 ? s->theta_w[y] : s->theta_cold;
                    res = wm2 * thw - val;                  /* Eq. 45 */
                } else {
                    res = val;                              /* Eq. 44 */
                }
                s->gn[5 * k + s->opp5[i]] = res;
            }
        }
    double *t;
    t = s->f; s->f = s->fn; s->fn = t;
    t = s->g; s->g = s->gn; s->gn = t;
    s->steps += 1;
}

int orc_step(orc_t *s, long nsteps)
{
    if (!s || nsteps < 0) return ORC_EINVAL;
    for (long k = 0; k < nsteps; ++k) step_once(s);
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Diagnostics                                                             */
/* ---------------------------------------------------------------------- */
/* Eq. 9 and Eq. 33 on the pre-collision state: U = u / (sqrt(3) c_s) = u,
 * V likewise, theta from Eq. 41, P = p / (3 rho c_s^2) with p = c_s^2 drho. */
int orc_fields(const orc_t *s, double *U, double *V, double *theta, double *P)
{
    size_t nn = (size_t)s->n * s->n;
    for (size_t k = 0; k < nn; ++k) {
        const double *f = &s->f[9 * k], *g = &s->g[5 * k];
        double drho = 0.0, jx = 0.0, jy = 0.0, th = 0.0;
        for (int i = 0; i < 9; ++i) {
            drho += f[i];
            jx += f[i] * s->e[i][0];
            jy += f[i] * s->e[i][1];
        }
        for (int i = 0; i < 5; ++i) th += g[i];
        if (U) U[k] = jx / s->rho0;
        if (V) V[k] = jy / s->rho0;
        if (theta) theta[k] = th;
        if (P) P[k] = drho / 3.0;
    }
    return ORC_OK;
}

/* Eqs. 18-19 with reading R7.  wall 0: hot (x = 0), wall 1: cold (x = H).
 * Nu(Y) = -d theta / d X at the wall, in units of the wall difference.     */
int orc_nusselt(const orc_t *s, int wall, double *nu_avg, double *nu_local)
{
    const int n = s->n;
    if (n < 2 || (wall != 0 && wall != 1)) return ORC_EINVAL;
    double dT = s->theta_hot - s->theta_cold;
    double sum = 0.0;
    for (int y = 0; y < n; ++y) {
        int x0 = wall == 0 ? 0 : n - 1, x1 = wall == 0 ? 1 : n - 2;
        double t0 = 0.0, t1 = 0.0;
        for (int i = 0; i < 5; ++i) {
            t0 += s->g[5 * ((size_t)y * n + x0) + i];
            t1 += s->g[5 * ((size_t)y * n + x1) + i];
        }
        double tw = wall == 0 ? s->theta_w[y] : s->theta_cold;
        /* quadratic through (0, tw), (1/2, t0), (3/2, t1) in lattice units,
         * slope at the wall pointing into the fluid                         */
        double slope_in = (9.0 * t0 - t1 - 8.0 * tw) / 3.0;
        /* heat flux along +x: -dtheta/dx; at the hot wall the inward
         * direction is +x, at the cold wall it is -x                        */
        double nu = (wall == 0 ? -slope_in : slope_in) * s->H / dT;
        if (nu_local) nu_local[y] = nu;
        sum += nu;
    }
    if (nu_avg) *nu_avg = sum / n;
    return ORC_OK;
}

/* Objective of the gradient problem: J = mean of the hot-wall Nu_avg
 * (Eqs. 18-19) over the last K of N steps taken from the current state. */
int orc_objective(orc_t *s, long N, long K, double *J)
{
    if (!s || N < 1 || K < 1 || K > N || !J) return ORC_EINVAL;
    double acc = 0.0;
    for (long m = 1; m <= N; ++m) {
        step_once(s);
        if (m > N - K) {
            double nu;
            orc_nusselt(s, 0, &nu, NULL);
            acc += nu;
        }
    }
    *J = acc / K;
    return ORC_OK;
}
