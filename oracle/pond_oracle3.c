/*
 * pond_oracle3.c -- TEST INFRASTRUCTURE ONLY (oracle), three-dimensional lattice.
 *
 * A plain, slow, FP64 CPU implementation of the D3Q27 time step of the
 * two-population Particles-on-Demand model of Reyhanian, Dorschner & Karlin,
 * "Thermokinetic model of compressible multiphase flows", arXiv:2002.09217, on a
 * periodic box.  Same method and the same readings (R1-R12 of pond_oracle.c, with the
 * same parity-unpinned ones) as the one- and two-dimensional oracle, written out for
 * three axes:
 *   - D3Q27 = C1 x C1 x C1, W_ijk = W_i W_j W_k, T_L = 1/3                        (App. B)
 *   - v_i = sqrt(theta) c_i + u, moments rho, rho u, 2 rho E                       (eqs. 1-2)
 *   - every donor of the 4x4x4 stencil is re-expressed in the receiver gauge with
 *     G = G_x (x) G_y (x) G_z (the 27 moments M_lmn factor per axis)               (App. C)
 *   - cubic Lagrange reconstruction per axis, x0 = floor(x) - 1                     (App. D)
 *   - BGK collisions with the force source, the force-extended g equilibrium
 *     (D = 3) and the sources g~ + phi                                             (eqs. 9, 16-22)
 *   - Korteweg stress (6 components), F = -div K, isotropic D3Q27 stencils         (eq. 18; App. F)
 * Only the test suite loads this file (through the same shared library as
 * pond_oracle.c, whose one-axis transfer and Lagrange routines it calls).
 *
 * Build: with pond_oracle.c, gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define T_L (1.0 / 3.0)
#define Q3 27

static const double W1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};

enum { ORC_OK = 0, ORC_E_INVALID = -1, ORC_E_NOMEM = -2, ORC_E_PRESSURE = -4, ORC_E_NONFINITE = -5 };

/* from pond_oracle.c: one-axis transfer G[k][i], cubic Lagrange weights and the
 * equation of state (kind, isothermal switch, double-well constants; R11) */
void orc_transfer_1d(double u_from, double th_from, double u_to, double th_to, double G[3][3]);
void orc_lagrange4(double t, double w[4]);
typedef struct {
    int kind, isothermal;
    double T0;
    double c[4];
} orc_eos;
double orc_eos_p(const orc_eos *E, double a, double b, double R, double rho, double T);
double orc_eos_e(const orc_eos *E, double a, double b, double R, double Cv, double rho, double T);
double orc_eos_T_of_e(const orc_eos *E, double a, double b, double R, double Cv, double rho, double e);
double orc_eos_T_of_p(const orc_eos *E, double a, double b, double R, double rho, double p);
int orc_eos_in_domain(const orc_eos *E, double b, double rho);
int orc_eos_valid(const orc_eos *E);

typedef struct {
    int nx, ny, nz;           /* periodic box */
    double a, b, R, delta;    /* EoS constants, C_v = R / delta */
    double omega, kappa, k_scale, dt;
    int n_pass;
    orc_eos eos;
} orc3_params;

/* direction q = 9 (cx + 1) + 3 (cy + 1) + (cz + 1) */
static int cxq(int q) { return q / 9 - 1; }
static int cyq(int q) { return (q / 3) % 3 - 1; }
static int czq(int q) { return q % 3 - 1; }
static double wq(int q) { return W1[q / 9] * W1[(q / 3) % 3] * W1[q % 3]; }

static double eos_p(const orc3_params *P, double rho, double T) { return orc_eos_p(&P->eos, P->a, P->b, P->R, rho, T); }
static double eos_e(const orc3_params *P, double rho, double T)
{
    return orc_eos_e(&P->eos, P->a, P->b, P->R, P->R / P->delta, rho, T);
}
static double eos_T_of_e(const orc3_params *P, double rho, double e)
{
    return orc_eos_T_of_e(&P->eos, P->a, P->b, P->R, P->R / P->delta, rho, e);
}
/* temperature of an initial state: T0 when isothermal */
static double state_T(const orc3_params *P, double T) { return P->eos.isothermal ? P->eos.T0 : T; }

static int thermo_bad(const orc3_params *P, double rho, double p)
{
    if (!isfinite(rho) || !isfinite(p)) return ORC_E_NONFINITE;
    if (p <= 0.0 || !orc_eos_in_domain(&P->eos, P->b, rho) || rho <= 0.0) return ORC_E_PRESSURE;
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* transfer (App. C): a gauge is (u_x, u_y, u_z, theta)                        */
/* ------------------------------------------------------------------------- */
static void transfer_axes(const double lf[4], const double lt[4], double G[3][3][3])
{
    for (int a = 0; a < 3; ++a) orc_transfer_1d(lf[a], lf[3], lt[a], lt[3], G[a]);
}

/* full population vector re-expressed from gauge lf to gauge lt */
void orc3_transfer_pop(const double lf[4], const double lt[4], const double *fin, double *fout)
{
    double G[3][3][3];
    transfer_axes(lf, lt, G);
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
            for (int m = 0; m < 3; ++m) {
                double s = 0.0;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j)
                        for (int n = 0; n < 3; ++n) s += G[0][k][i] * G[1][l][j] * G[2][m][n] * fin[9 * i + 3 * j + n];
                fout[9 * k + 3 * l + m] = s;
            }
}

/* ------------------------------------------------------------------------- */
/* equilibria and sources (eqs. 9, 16-22; App. F), D = 3                       */
/* ------------------------------------------------------------------------- */
void orc3_force_source(double rho, const double u[3], double theta, const double du[3], double *S)
{
    double feq[Q3], fs[Q3];
    double lf[4] = {u[0] + du[0], u[1] + du[1], u[2] + du[2], theta};
    double lt[4] = {u[0], u[1], u[2], theta};
    for (int q = 0; q < Q3; ++q) feq[q] = rho * wq(q);
    orc3_transfer_pop(lf, lt, feq, fs);
    for (int q = 0; q < Q3; ++q) S[q] = fs[q] - feq[q];
}

void orc3_geq(const orc3_params *P, double rho, const double u[3], double theta, double p, double E,
              const double uh[3], const double F[3], double *g)
{
    double Pr = p / rho, H = E + Pr, s = sqrt(theta);
    double X[3][3], M[3], N[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) X[a][b] = uh[a] * F[b] + F[a] * uh[b] + P->dt * F[a] * F[b] * E / (2.0 * p);
    for (int a = 0; a < 3; ++a) {
        double xu = 0.0;
        for (int b = 0; b < 3; ++b) xu += X[a][b] * u[b];
        M[a] = P->dt / Pr * (F[a] * H - xu);
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) N[a][b] = (a == b ? rho : 0.0) + P->dt / (2.0 * Pr) * X[a][b];
    for (int q = 0; q < Q3; ++q) {
        double c[3] = {(double)cxq(q), (double)cyq(q), (double)czq(q)}, v[3];
        for (int a = 0; a < 3; ++a) v[a] = u[a] + s * c[a];
        double t1 = 0.0, t2 = 0.0;
        for (int a = 0; a < 3; ++a) t1 += M[a] * (v[a] - u[a]);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) t2 += N[a][b] * (v[a] * v[b] - (a == b ? Pr : 0.0) - u[a] * u[b]);
        g[q] = wq(q) * (2.0 * rho * E + t1 + t2);
    }
}

void orc3_psi(double rho, const double u[3], double theta, double p, double *psi)
{
    double s = sqrt(theta);
    for (int q = 0; q < Q3; ++q) {
        double c[3] = {(double)cxq(q), (double)cyq(q), (double)czq(q)};
        double uc = 0.0, v2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double v = u[a] + s * c[a];
            uc += u[a] * c[a];
            v2 += v * v;
        }
        psi[q] = wq(q) * (1.0 + rho * uc * uc / (2.0 * p * T_L) - rho * v2 / (2.0 * p) + 1.5);
    }
}

typedef struct {
    double u[3], uh[3], e, T, p, theta, h, mu, kc;
} node3;

static void close_node(const orc3_params *P, double rho, const double j[3], double E, const double F[3], node3 *n)
{
    double uh2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        n->u[a] = j[a] / rho;
        n->uh[a] = n->u[a] + F[a] * P->dt / (2.0 * rho);
        uh2 += n->uh[a] * n->uh[a];
    }
    n->e = E - 0.5 * uh2;
    n->T = eos_T_of_e(P, rho, n->e);
    n->p = eos_p(P, rho, n->T);
    n->theta = n->p / (rho * T_L);
    n->h = n->e + n->p / rho;
    n->mu = (1.0 / P->omega - 0.5) * n->p * P->dt;
    n->kc = P->k_scale * n->mu * P->R * (1.0 + P->delta) / P->delta;
}

/* collision of one node in the gauge (u, theta_final) (R2) */
int orc3_collide(const orc3_params *P, const double lam_str[4], const double *fstr, const double *gstr,
                 const double F[3], double M0, double *fout, double *gout, double lam_out[4])
{
    double s_str = sqrt(lam_str[3]);
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, G2 = 0.0;
    for (int q = 0; q < Q3; ++q) {
        double c[3] = {(double)cxq(q), (double)cyq(q), (double)czq(q)};
        rho += fstr[q];
        for (int a = 0; a < 3; ++a) j[a] += fstr[q] * (lam_str[a] + s_str * c[a]);
        G2 += gstr[q];
    }
    double E = G2 / (2.0 * rho);
    node3 n;
    close_node(P, rho, j, E, F, &n);
    int bad = thermo_bad(P, rho, n.p);
    if (bad) return bad;
    double lam_c[4] = {n.u[0], n.u[1], n.u[2], n.theta};
    double f[Q3], g[Q3], S[Q3], geq[Q3], psi[Q3];
    orc3_transfer_pop(lam_str, lam_c, fstr, f);
    orc3_transfer_pop(lam_str, lam_c, gstr, g);
    double du[3] = {F[0] * P->dt / rho, F[1] * P->dt / rho, F[2] * P->dt / rho};
    orc3_force_source(rho, n.u, n.theta, du, S);
    for (int q = 0; q < Q3; ++q) fout[q] = f[q] + P->omega * (rho * wq(q) - f[q]) + S[q];
    orc3_geq(P, rho, n.u, n.theta, n.p, E, n.uh, F, geq);
    orc3_psi(rho, n.u, n.theta, n.p, psi);
    double work = 0.0;
    for (int a = 0; a < 3; ++a) work += 2.0 * n.uh[a] * F[a];
    for (int q = 0; q < Q3; ++q) gout[q] = g[q] + P->omega * (geq[q] - g[q]) + (M0 + work) * psi[q] * P->dt;
    for (int a = 0; a < 3; ++a) lam_out[a] = n.u[a];
    lam_out[3] = n.theta;
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* periodic box                                                                */
/* ------------------------------------------------------------------------- */
static int wrap(int i, int n) { return ((i % n) + n) % n; }
static int node_of(const orc3_params *P, int x, int y, int z)
{
    return wrap(x, P->nx) + P->nx * (wrap(y, P->ny) + P->ny * wrap(z, P->nz));
}

typedef struct {
    const double *f, *g, *ux, *uy, *uz, *th, *Fx, *Fy, *Fz;
} cstate3;

/* streaming of one receiver with the predictor-corrector (eqs. 1-4; R1, R3) */
static int stream_receiver(const orc3_params *P, const cstate3 *S, int x, int y, int z, double *fstr,
                           double *gstr, double lam_str[4], double *rho_o, double j_o[3], double *E_o)
{
    int N = P->nx * P->ny * P->nz;
    int node = x + P->nx * (y + P->ny * z);
    double lam[4] = {S->ux[node], S->uy[node], S->uz[node], S->th[node]};
    double Fp[3] = {S->Fx[node], S->Fy[node], S->Fz[node]};
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, E = 0.0;
    for (int pass = 0; pass < P->n_pass; ++pass) {
        double s = sqrt(lam[3]);
        for (int q = 0; q < Q3; ++q) {
            int c[3] = {cxq(q), cyq(q), czq(q)};
            int pos[3] = {x, y, z}, i0[3];
            double w[3][4];
            for (int a = 0; a < 3; ++a) {
                double X = (double)pos[a] - (lam[a] + s * (double)c[a]) * P->dt; /* departure point */
                double x0 = floor(X) - 1.0;                                      /* App. D */
                orc_lagrange4(X - x0, w[a]);
                i0[a] = (int)x0;
            }
            int k = c[0] + 1, l = c[1] + 1, m = c[2] + 1;
            double accf = 0.0, accg = 0.0;
            for (int dz = 0; dz < 4; ++dz)
                for (int dy = 0; dy < 4; ++dy)
                    for (int dx = 0; dx < 4; ++dx) {
                        int d = node_of(P, i0[0] + dx, i0[1] + dy, i0[2] + dz);
                        double ld[4] = {S->ux[d], S->uy[d], S->uz[d], S->th[d]};
                        double G[3][3][3];
                        transfer_axes(ld, lam, G);
                        /* component (k, l, m) of the donor populations in the receiver gauge */
                        double rf = 0.0, rg = 0.0;
                        for (int i = 0; i < 3; ++i)
                            for (int jj = 0; jj < 3; ++jj)
                                for (int n = 0; n < 3; ++n) {
                                    double gg = G[0][k][i] * G[1][l][jj] * G[2][m][n];
                                    int qi = 9 * i + 3 * jj + n;
                                    rf += gg * S->f[(size_t)qi * N + d];
                                    rg += gg * S->g[(size_t)qi * N + d];
                                }
                        double a_ = w[0][dx] * w[1][dy] * w[2][dz];
                        accf += a_ * rf;
                        accg += a_ * rg;
                    }
            fstr[q] = accf;
            gstr[q] = accg;
        }
        rho = 0.0;
        j[0] = j[1] = j[2] = 0.0;
        double G2 = 0.0;
        for (int q = 0; q < Q3; ++q) {
            double c[3] = {(double)cxq(q), (double)cyq(q), (double)czq(q)};
            rho += fstr[q];
            for (int a = 0; a < 3; ++a) j[a] += fstr[q] * (lam[a] + s * c[a]);
            G2 += gstr[q];
        }
        E = G2 / (2.0 * rho);
        node3 n;
        close_node(P, rho, j, E, Fp, &n);
        int bad = thermo_bad(P, rho, n.p);
        if (bad) return bad;
        memcpy(lam_str, lam, sizeof lam);
        for (int a = 0; a < 3; ++a) lam[a] = n.u[a];
        lam[3] = n.theta;
    }
    *rho_o = rho;
    memcpy(j_o, j, sizeof j);
    *E_o = E;
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* non-local terms (eq. 18; R5, R6)                                           */
/* ------------------------------------------------------------------------- */
/* K components: 0 xx, 1 xy, 2 xz, 3 yy, 4 yz, 5 zz */
static const int KIDX[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

static void korteweg(const orc3_params *P, const double *rho, double *K)
{
    int N = P->nx * P->ny * P->nz;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < N; ++n) {
        int x = n % P->nx, y = (n / P->nx) % P->ny, z = n / (P->nx * P->ny);
        double r0 = rho[n], gr[3] = {0.0, 0.0, 0.0}, lap = 0.0;
        for (int q = 0; q < Q3; ++q) {
            int c[3] = {cxq(q), cyq(q), czq(q)};
            double rq = rho[node_of(P, x + c[0], y + c[1], z + c[2])];
            for (int a = 0; a < 3; ++a) gr[a] += wq(q) * (double)c[a] * rq;
            lap += wq(q) * (rq - r0);
        }
        for (int a = 0; a < 3; ++a) gr[a] /= T_L;
        lap *= 2.0 / T_L;
        double iso = -P->kappa * (r0 * lap + 0.5 * (gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]));
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b)
                K[(size_t)KIDX[a][b] * N + n] = (a == b ? iso : 0.0) + P->kappa * gr[a] * gr[b];
    }
}

static void korteweg_force(const orc3_params *P, const double *K, double *F)
{
    int N = P->nx * P->ny * P->nz;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < N; ++n) {
        int x = n % P->nx, y = (n / P->nx) % P->ny, z = n / (P->nx * P->ny);
        double dv[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < Q3; ++q) {
            int c[3] = {cxq(q), cyq(q), czq(q)};
            int m = node_of(P, x + c[0], y + c[1], z + c[2]);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) dv[a] += wq(q) * K[(size_t)KIDX[a][b] * N + m] * (double)c[b];
        }
        for (int a = 0; a < 3; ++a) F[(size_t)a * N + n] = -dv[a] / T_L;
    }
}

static void heat_correction(const orc3_params *P, const double *T, const double *h, const double *mu,
                            const double *kc, double *M0)
{
    int N = P->nx * P->ny * P->nz;
#pragma omp parallel for schedule(static)
    for (int n = 0; n < N; ++n) {
        if (P->k_scale < 0.0) {
            M0[n] = 0.0;
            continue;
        }
        int x = n % P->nx, y = (n / P->nx) % P->ny, z = n / (P->nx * P->ny);
        double acc = 0.0;
        for (int q = 0; q < Q3; ++q) {
            int m = node_of(P, x + cxq(q), y + cyq(q), z + czq(q));
            double kmid = 0.5 * (kc[m] + kc[n]);
            double mmid = 0.5 * (mu[m] + mu[n]);
            acc += wq(q) * (kmid * (T[m] - T[n]) - mmid * (h[m] - h[n]));
        }
        M0[n] = 2.0 * (2.0 / T_L) * acc;
    }
}

static int valid(const orc3_params *P)
{
    if (P->nx < 1 || P->ny < 1 || P->nz < 1) return 0;
    if (!(P->delta > 0.0 && P->delta <= 2.0 / 3.0)) return 0;
    if (!(P->omega > 0.0 && P->omega < 2.0)) return 0;
    if (P->n_pass < 1 || !(P->dt > 0.0)) return 0;
    return orc_eos_valid(&P->eos);
}

/* Non-local closure and collision of every node (shared by the step and the initial
 * state).  lam: 4 planes of the streamed gauge; j: 3 planes; side output: u (3
 * planes), theta, F (3 planes). */
static int close_and_collide(const orc3_params *P, const double *fstr, const double *gstr, const double *lam,
                             const double *rho, const double *j, const double *E, double *f, double *g,
                             double *u, double *th, double *F)
{
    int N = P->nx * P->ny * P->nz, err = ORC_OK;
    double *K = malloc(sizeof(double) * 6 * N), *Fn = malloc(sizeof(double) * 3 * N);
    double *T = malloc(sizeof(double) * N), *h = malloc(sizeof(double) * N);
    double *mu = malloc(sizeof(double) * N), *kc = malloc(sizeof(double) * N);
    double *M0 = malloc(sizeof(double) * N);
    if (!K || !Fn || !T || !h || !mu || !kc || !M0) {
        err = ORC_E_NOMEM;
        goto done;
    }
    korteweg(P, rho, K);
    korteweg_force(P, K, Fn);
    for (int n = 0; n < N; ++n) {
        double jj[3] = {j[n], j[(size_t)N + n], j[(size_t)2 * N + n]};
        double Fv[3] = {Fn[n], Fn[(size_t)N + n], Fn[(size_t)2 * N + n]};
        node3 t;
        close_node(P, rho[n], jj, E[n], Fv, &t);
        int bad = thermo_bad(P, rho[n], t.p);
        if (bad) {
            err = bad;
            goto done;
        }
        T[n] = t.T;
        h[n] = t.h;
        mu[n] = t.mu;
        kc[n] = t.kc;
    }
    heat_correction(P, T, h, mu, kc, M0);
    for (int n = 0; n < N; ++n) {
        double ls[4], fs[Q3], gs[Q3], fo[Q3], go[Q3], lo[4];
        for (int a = 0; a < 4; ++a) ls[a] = lam[(size_t)a * N + n];
        for (int q = 0; q < Q3; ++q) {
            fs[q] = fstr[(size_t)q * N + n];
            gs[q] = gstr[(size_t)q * N + n];
        }
        double Fv[3] = {Fn[n], Fn[(size_t)N + n], Fn[(size_t)2 * N + n]};
        int bad = orc3_collide(P, ls, fs, gs, Fv, M0[n], fo, go, lo);
        if (bad) {
            err = bad;
            goto done;
        }
        for (int q = 0; q < Q3; ++q) {
            f[(size_t)q * N + n] = fo[q];
            g[(size_t)q * N + n] = go[q];
        }
        for (int a = 0; a < 3; ++a) {
            u[(size_t)a * N + n] = lo[a];
            F[(size_t)a * N + n] = Fv[a];
        }
        th[n] = lo[3];
    }
done:
    free(K); free(Fn); free(T); free(h); free(mu); free(kc); free(M0);
    return err;
}

/* Initial state from (rho, u_hat (3 planes), T) (R9).  u and F are 3 planes each. */
int orc3_init(const orc3_params *P, const double *rho, const double *uh_in, const double *Tin, double *f,
              double *g, double *u, double *th, double *F)
{
    if (!valid(P)) return ORC_E_INVALID;
    int N = P->nx * P->ny * P->nz, err = ORC_OK;
    double *K = malloc(sizeof(double) * 6 * N), *F0 = malloc(sizeof(double) * 3 * N);
    double *fe = malloc(sizeof(double) * Q3 * N), *ge = malloc(sizeof(double) * Q3 * N);
    double *lam = malloc(sizeof(double) * 4 * N), *j = malloc(sizeof(double) * 3 * N);
    double *Ev = malloc(sizeof(double) * N);
    if (!K || !F0 || !fe || !ge || !lam || !j || !Ev) {
        err = ORC_E_NOMEM;
        goto done;
    }
    korteweg(P, rho, K);
    korteweg_force(P, K, F0);
    for (int n = 0; n < N; ++n) {
        double r = rho[n], uh[3], Fv[3], uu[3];
        for (int a = 0; a < 3; ++a) {
            uh[a] = uh_in[(size_t)a * N + n];
            Fv[a] = F0[(size_t)a * N + n];
            uu[a] = uh[a] - Fv[a] * P->dt / (2.0 * r);
        }
        double Tn = state_T(P, Tin[n]);
        double p = eos_p(P, r, Tn);
        int bad = thermo_bad(P, r, p);
        if (bad) {
            err = bad;
            goto done;
        }
        double E = eos_e(P, r, Tn) + 0.5 * (uh[0] * uh[0] + uh[1] * uh[1] + uh[2] * uh[2]);
        double theta = p / (r * T_L), geq[Q3];
        orc3_geq(P, r, uu, theta, p, E, uh, Fv, geq);
        for (int q = 0; q < Q3; ++q) {
            fe[(size_t)q * N + n] = r * wq(q);
            ge[(size_t)q * N + n] = geq[q];
        }
        for (int a = 0; a < 3; ++a) {
            lam[(size_t)a * N + n] = uu[a];
            j[(size_t)a * N + n] = r * uu[a];
        }
        lam[(size_t)3 * N + n] = theta;
        Ev[n] = E;
    }
    err = close_and_collide(P, fe, ge, lam, rho, j, Ev, f, g, u, th, F);
done:
    free(K); free(F0); free(fe); free(ge); free(lam); free(j); free(Ev);
    return err;
}

/* Advance nsteps time steps; on error the state is that of the last completed step. */
int orc3_step(const orc3_params *P, int nsteps, double *f, double *g, double *u, double *th, double *F,
              int *done_steps)
{
    if (!valid(P)) return ORC_E_INVALID;
    int N = P->nx * P->ny * P->nz, err = ORC_OK;
    if (done_steps) *done_steps = 0;
    double *fstr = malloc(sizeof(double) * Q3 * N), *gstr = malloc(sizeof(double) * Q3 * N);
    double *lam = malloc(sizeof(double) * 4 * N), *rho = malloc(sizeof(double) * N);
    double *j = malloc(sizeof(double) * 3 * N), *E = malloc(sizeof(double) * N);
    int *errs = malloc(sizeof(int) * N);
    double *fn = malloc(sizeof(double) * Q3 * N), *gn = malloc(sizeof(double) * Q3 * N);
    double *un = malloc(sizeof(double) * 3 * N), *thn = malloc(sizeof(double) * N);
    double *Fn = malloc(sizeof(double) * 3 * N);
    if (!fstr || !gstr || !lam || !rho || !j || !E || !errs || !fn || !gn || !un || !thn || !Fn) {
        err = ORC_E_NOMEM;
        goto done;
    }
    for (int step = 0; step < nsteps; ++step) {
        cstate3 S = {f, g, u, u + N, u + 2 * (size_t)N, th, F, F + N, F + 2 * (size_t)N};
#pragma omp parallel for schedule(dynamic, 1)
        for (int n = 0; n < N; ++n) {
            int x = n % P->nx, y = (n / P->nx) % P->ny, z = n / (P->nx * P->ny);
            double fs[Q3] = {0}, gs[Q3] = {0}, ls[4] = {0}, jj[3] = {0}, r = 0.0, e_ = 0.0;
            errs[n] = stream_receiver(P, &S, x, y, z, fs, gs, ls, &r, jj, &e_);
            for (int q = 0; q < Q3; ++q) {
                fstr[(size_t)q * N + n] = fs[q];
                gstr[(size_t)q * N + n] = gs[q];
            }
            for (int a = 0; a < 4; ++a) lam[(size_t)a * N + n] = ls[a];
            for (int a = 0; a < 3; ++a) j[(size_t)a * N + n] = jj[a];
            rho[n] = r;
            E[n] = e_;
        }
        for (int n = 0; n < N; ++n)
            if (errs[n]) {
                err = errs[n];
                goto done;
            }
        err = close_and_collide(P, fstr, gstr, lam, rho, j, E, fn, gn, un, thn, Fn);
        if (err) goto done;
        memcpy(f, fn, sizeof(double) * Q3 * N);
        memcpy(g, gn, sizeof(double) * Q3 * N);
        memcpy(u, un, sizeof(double) * 3 * N);
        memcpy(th, thn, sizeof(double) * N);
        memcpy(F, Fn, sizeof(double) * 3 * N);
        if (done_steps) *done_steps = step + 1;
    }
done:
    free(fstr); free(gstr); free(lam); free(rho); free(j); free(E); free(errs);
    free(fn); free(gn); free(un); free(thn); free(Fn);
    return err;
}

/* rho = sum f, u_hat = u + F dt/(2 rho) (3 planes), T, p = rho theta T_L, E = e + u_hat^2/2 */
void orc3_moments(const orc3_params *P, const double *f, const double *u, const double *th, const double *F,
                  double *rho, double *uh, double *T, double *p, double *E)
{
    int N = P->nx * P->ny * P->nz;
    for (int n = 0; n < N; ++n) {
        double r = 0.0;
        for (int q = 0; q < Q3; ++q) r += f[(size_t)q * N + n];
        double h2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            double v = u[(size_t)a * N + n] + F[(size_t)a * N + n] * P->dt / (2.0 * r);
            uh[(size_t)a * N + n] = v;
            h2 += v * v;
        }
        double pr = r * th[n] * T_L;
        double Tn = orc_eos_T_of_p(&P->eos, P->a, P->b, P->R, r, pr);
        rho[n] = r;
        T[n] = Tn;
        p[n] = pr;
        E[n] = eos_e(P, r, Tn) + 0.5 * h2;
    }
}

/* exported views of the non-local operators, for the telescoping-sum tests */
void orc3_korteweg_force(const orc3_params *P, const double *rho, double *F)
{
    int N = P->nx * P->ny * P->nz;
    double *K = malloc(sizeof(double) * 6 * N);
    if (K) {
        korteweg(P, rho, K);
        korteweg_force(P, K, F);
    }
    free(K);
}

void orc3_heat_correction(const orc3_params *P, const double *T, const double *h, const double *mu,
                          const double *kc, double *M0)
{
    heat_correction(P, T, h, mu, kc, M0);
}
