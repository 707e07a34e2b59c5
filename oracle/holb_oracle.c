/*
 * holb_oracle.c -- FP64 CPU oracle for the high-order BGK lattice Boltzmann
 * step with Hermite source terms (arXiv:2411.10751).
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, obviously-correct reference used
 * to check the HIP path.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product never does.
 *
 * State is the shifted, pre-collision population f^ of Eq. (4.3).  One step
 * follows the order the paper's update implies:
 *   1. wall closure of the unknown populations (Section 4.3, Eqs. 4.7-4.8;
 *      the wall-node target solved from the boundary conditions),
 *   2. moments and macroscopic fields with the source shift (Eq. 4.5),
 *      including the pseudopotential force (Eq. 3.8) when enabled,
 *   3. temperature gradient by central finite differences (Section 3.2),
 *   4. sources F_i (Eq. 3.3), H_i (Eq. 3.7), P_i (Eq. 3.12),
 *   5. equilibrium (Eq. 2.2) and the BGK + trapezoidal-source collision (Eq. 4.4),
 *   6. push streaming f^(x + c_i, t+1) = f*(x, t) (left side of Eq. 4.4).
 * Everything is FP64 with no blocking or fusion.
 */
#include "holb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Lattices (Section 4.1, Table 1).                                         */
/* ------------------------------------------------------------------------ */

/* The velocity set is the union of symmetry orbits ("shells") of these
 * representatives.  D2Q37 shells follow the grouping of Table 1 (|c|^2 = 0, 1,
 * 2, 4, 5, 8, 9, 10; the |c|^2 = 5 shell is split in the table but shares one
 * weight).  D3Q39 is not in the paper: it is the standard degree-7 shell set
 * (0,0,0), (1,0,0), (1,1,1), (2,0,0), (2,2,0), (3,0,0). */
static const int shells_d2q37[8][3] = {
    {0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {2, 0, 0}, {2, 1, 0}, {2, 2, 0}, {3, 0, 0}, {3, 1, 0}};
static const int shells_d3q39[6][3] = {
    {0, 0, 0}, {1, 0, 0}, {1, 1, 1}, {2, 0, 0}, {2, 2, 0}, {3, 0, 0}};

/* Moment conditions: sum_i w_i c_i^p = c0^|p| * E[g^p] with g a unit normal
 * vector (all odd moments vanish by symmetry of the shells).  D2Q37 matches
 * every moment of degree <= 8 (8th-order isotropy, Section 4.1), D3Q39 every
 * moment of degree <= 6. */
static const int pows_d2q37[9][3] = {
    {0, 0, 0}, {2, 0, 0}, {4, 0, 0}, {2, 2, 0}, {6, 0, 0}, {4, 2, 0}, {8, 0, 0}, {6, 2, 0}, {4, 4, 0}};
static const int pows_d3q39[7][3] = {
    {0, 0, 0}, {2, 0, 0}, {4, 0, 0}, {2, 2, 0}, {6, 0, 0}, {4, 2, 0}, {2, 2, 2}};

static double dfact_odd(int n) /* (n)!! for odd n >= -1 */
{
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

static double gauss_moment(const int p[3], double c0sq)
{
    double m = 1.0;
    int deg = 0;
    for (int a = 0; a < 3; ++a) {
        if (p[a] % 2) return 0.0;
        m *= dfact_odd(p[a] - 1);
        deg += p[a];
    }
    return m * pow(c0sq, deg / 2);
}

static int cmp_vec(const int *a, const int *b)
{
    for (int k = 0; k < 3; ++k)
        if (a[k] != b[k]) return a[k] < b[k] ? -1 : 1;
    return 0;
}

/* Orbit of rep under axis permutations and sign flips, sorted, deduplicated. */
static int shell_orbit(int D, const int rep[3], int out[48][3])
{
    static const int perm2[2][3] = {{0, 1, 2}, {1, 0, 2}};
    static const int perm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int np = D == 2 ? 2 : 6;
    int n = 0;
    for (int ip = 0; ip < np; ++ip) {
        const int *pm = D == 2 ? perm2[ip] : perm3[ip];
        for (int s = 0; s < (1 << D); ++s) {
            int v[3] = {0, 0, 0};
            for (int a = 0; a < D; ++a) v[a] = ((s >> a) & 1 ? -1 : 1) * rep[pm[a]];
            int dup = 0;
            for (int k = 0; k < n; ++k)
                if (!cmp_vec(out[k], v)) { dup = 1; break; }
            if (!dup) { memcpy(out[n], v, sizeof v); ++n; }
        }
    }
    /* insertion sort, lexicographic */
    for (int i = 1; i < n; ++i)
        for (int j = i; j > 0 && cmp_vec(out[j - 1], out[j]) > 0; --j) {
            int t[3];
            memcpy(t, out[j], sizeof t);
            memcpy(out[j], out[j - 1], sizeof t);
            memcpy(out[j - 1], t, sizeof t);
        }
    return n;
}

/* Gaussian elimination with row pivoting on the (S+1) x S moment system.
 * The pivot order depends only on the shell sums, so the leftover residual is
 * a polynomial in c0^2; the lattice constant is its root. */
static double moment_residual(int S, const double A0[10][9], const double b0[10], double *W)
{
    double A[10][9], b[10];
    memcpy(A, A0, sizeof A);
    memcpy(b, b0, sizeof b);
    for (int k = 0; k < S; ++k) {
        int piv = k;
        for (int r = k + 1; r <= S; ++r)
            if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
        if (piv != k) {
            for (int j = 0; j < S; ++j) { double t = A[k][j]; A[k][j] = A[piv][j]; A[piv][j] = t; }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int r = k + 1; r <= S; ++r) {
            double fct = A[r][k] / A[k][k];
            for (int j = k; j < S; ++j) A[r][j] -= fct * A[k][j];
            b[r] -= fct * b[k];
        }
    }
    if (W) {
        for (int k = S - 1; k >= 0; --k) {
            double acc = b[k];
            for (int j = k + 1; j < S; ++j) acc -= A[k][j] * W[j];
            W[k] = acc / A[k][k];
        }
    }
    return b[S];
}

static void moment_system(int D, int S, const int (*reps)[3], const int (*pows)[3], double c0sq,
                          double A[10][9], double b[10])
{
    memset(A, 0, sizeof(double) * 10 * 9);
    for (int k = 0; k <= S; ++k) {
        for (int s = 0; s < S; ++s) {
            int orb[48][3];
            int n = shell_orbit(D, reps[s], orb);
            double acc = 0.0;
            for (int m = 0; m < n; ++m) {
                double t = 1.0;
                for (int a = 0; a < 3; ++a)
                    for (int e = 0; e < pows[k][a]; ++e) t *= orb[m][a];
                acc += t;
            }
            A[k][s] = acc;
        }
        b[k] = gauss_moment(pows[k], c0sq);
    }
}

int orc_lattice_get(int lattice, orc_lattice *L)
{
    int D, S;
    const int(*reps)[3];
    const int(*pows)[3];
    if (lattice == ORC_D2Q37) { D = 2; S = 8; reps = shells_d2q37; pows = pows_d2q37; }
    else if (lattice == ORC_D3Q39) { D = 3; S = 6; reps = shells_d3q39; pows = pows_d3q39; }
    else return ORC_EINVAL;

    /* Bisection for c0^2 on [0.5, 0.9]; the residual has a single sign change
     * there for both shell sets (the paper quotes c0 ~ 0.83543 for D2Q37). */
    double A[10][9], b[10];
    double lo = 0.5, hi = 0.9;
    moment_system(D, S, reps, pows, lo, A, b);
    double rlo = moment_residual(S, A, b, NULL);
    moment_system(D, S, reps, pows, hi, A, b);
    double rhi = moment_residual(S, A, b, NULL);
    if (rlo * rhi > 0) return ORC_ENUMERIC;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        moment_system(D, S, reps, pows, mid, A, b);
        double rm = moment_residual(S, A, b, NULL);
        if (rm == 0.0) { lo = hi = mid; break; }
        if ((rm < 0) == (rlo < 0)) { lo = mid; rlo = rm; }
        else hi = mid;
        if (hi - lo <= 1e-17) break;
    }
    double c0sq = 0.5 * (lo + hi);
    double W[9];
    moment_system(D, S, reps, pows, c0sq, A, b);
    moment_residual(S, A, b, W);

    memset(L, 0, sizeof *L);
    L->D = D;
    L->c0sq = c0sq;
    int q = 0;
    for (int s = 0; s < S; ++s) {
        int orb[48][3];
        int n = shell_orbit(D, reps[s], orb);
        for (int m = 0; m < n; ++m) {
            memcpy(L->c[q], orb[m], sizeof orb[m]);
            L->w[q] = W[s];
            ++q;
        }
    }
    L->Q = q;
    for (int i = 0; i < q; ++i) {
        L->opp[i] = -1;
        for (int j = 0; j < q; ++j)
            if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] && L->c[j][2] == -L->c[i][2])
                L->opp[i] = j;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Local kinetic algebra.  Lattice units outside; inside, the paper's Hermite */
/* units xi = c/c0, U = u/c0, Phi = F/c0 (Table 2 is the same in lattice    */
/* units).                                                                  */
/* ------------------------------------------------------------------------ */

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Eq. (2.2): fourth-order Hermite equilibrium of one discrete velocity. */
static double feq_one(int D, double w, const double xi[3], double rho, const double U[3], double theta)
{
    double xu = dot3(xi, U), uu = dot3(U, U), xx = dot3(xi, xi), thb = theta - 1.0;
    double t = 1.0 + xu + 0.5 * xu * xu - 0.5 * uu + 0.5 * thb * (xx - D)
             + xu * xu * xu / 6.0 - 0.5 * xu * uu + 0.5 * xu * thb * (xx - (D + 2))
             + xu * xu * xu * xu / 24.0 - 0.25 * xu * xu * uu + 0.125 * uu * uu
             + 0.25 * thb * (xu * xu * (xx - (D + 4)) + uu * ((D + 2) - xx))
             + 0.125 * thb * thb * (xx * xx - 2.0 * (D + 2) * xx + D * (D + 2));
    return w * rho * t;
}

/* Eq. (3.3): third-order Hermite body-force source of one discrete velocity.
 * The last term is -(xi.U)(U.Phi) as in Eq. (3.3); Table 2 prints a garbled
 * repeat of the second term instead. */
static double force_one(int D, double w, const double xi[3], const double U[3], const double Phi[3],
                        double theta)
{
    double xu = dot3(xi, U), uu = dot3(U, U), xx = dot3(xi, xi), thb = theta - 1.0;
    double xF = dot3(xi, Phi), UF = dot3(U, Phi);
    double t = xF + xu * xF - UF + 0.5 * xF * (xu * xu + thb * xx - uu - thb * (D + 2)) - xu * UF;
    return w * t;
}

/* Eq. (3.7): thermal-dissipation source, 0.5 w rho theta (1 - 1/Pr)
 * (|xi|^2 - D - 2) (c . grad theta), grad theta per lattice spacing. */
static double thermal_one(int D, double w, const double xi[3], const int c[3], double rho,
                          double theta, double prandtl, const double gT[3])
{
    double xx = dot3(xi, xi);
    double cg = c[0] * gT[0] + c[1] * gT[1] + c[2] * gT[2];
    return 0.5 * w * rho * theta * (1.0 - 1.0 / prandtl) * (xx - D - 2) * cg;
}

/* Eq. (3.12): pressure-tensor source, with tau = tau_hat - 1/2 (Eq. 4.3) and
 * |F^SC|^2 / (c0^2 G psi^2) the Hermite-consistent lattice-unit factor. */
static double ptensor_one(int D, double w, const double xi[3], double tau, double k, double G,
                          const double Fsc[3], double psi, double c0sq)
{
    double xx = dot3(xi, xi);
    double F2 = dot3(Fsc, Fsc);
    return -w * (k / (2.0 * D * tau)) * (F2 / (c0sq * G * psi * psi)) * (xx - D);
}

static const orc_lattice *lattice_cached(int lattice)
{
    static orc_lattice L[2];
    static int ready[2] = {0, 0};
    if (lattice < 0 || lattice > 1) return NULL;
    if (!ready[lattice]) {
#ifdef _OPENMP
#pragma omp critical(orc_lattice_init)
#endif
        {
            if (!ready[lattice] && orc_lattice_get(lattice, &L[lattice]) == ORC_OK) ready[lattice] = 1;
        }
    }
    return ready[lattice] ? &L[lattice] : NULL;
}

static void scaled(const orc_lattice *L, int i, double xi[3])
{
    double c0 = sqrt(L->c0sq);
    for (int a = 0; a < 3; ++a) xi[a] = L->c[i][a] / c0;
}

int orc_feq(int lattice, double rho, const double *u, double theta, double *out)
{
    const orc_lattice *L = lattice_cached(lattice);
    if (!L) return ORC_EINVAL;
    double c0 = sqrt(L->c0sq), U[3] = {0, 0, 0}, xi[3];
    for (int a = 0; a < L->D; ++a) U[a] = u[a] / c0;
    for (int i = 0; i < L->Q; ++i) {
        scaled(L, i, xi);
        out[i] = feq_one(L->D, L->w[i], xi, rho, U, theta);
    }
    return ORC_OK;
}

int orc_src_force(int lattice, const double *F, const double *u, double theta, double *out)
{
    const orc_lattice *L = lattice_cached(lattice);
    if (!L) return ORC_EINVAL;
    double c0 = sqrt(L->c0sq), U[3] = {0, 0, 0}, Phi[3] = {0, 0, 0}, xi[3];
    for (int a = 0; a < L->D; ++a) { U[a] = u[a] / c0; Phi[a] = F[a] / c0; }
    for (int i = 0; i < L->Q; ++i) {
        scaled(L, i, xi);
        out[i] = force_one(L->D, L->w[i], xi, U, Phi, theta);
    }
    return ORC_OK;
}

int orc_src_thermal(int lattice, double rho, double theta, double prandtl, const double *grad_theta,
                    double *out)
{
    const orc_lattice *L = lattice_cached(lattice);
    if (!L || !(prandtl > 0)) return ORC_EINVAL;
    double gT[3] = {0, 0, 0}, xi[3];
    for (int a = 0; a < L->D; ++a) gT[a] = grad_theta[a];
    for (int i = 0; i < L->Q; ++i) {
        scaled(L, i, xi);
        out[i] = thermal_one(L->D, L->w[i], xi, L->c[i], rho, theta, prandtl, gT);
    }
    return ORC_OK;
}

int orc_src_ptensor(int lattice, double tau_hat, double k, double G, const double *Fsc, double psi,
                    double *out)
{
    const orc_lattice *L = lattice_cached(lattice);
    if (!L || !(tau_hat > 0.5)) return ORC_EINVAL;
    double F[3] = {0, 0, 0}, xi[3];
    for (int a = 0; a < L->D; ++a) F[a] = Fsc[a];
    for (int i = 0; i < L->Q; ++i) {
        scaled(L, i, xi);
        out[i] = ptensor_one(L->D, L->w[i], xi, tau_hat - 0.5, k, G, F, psi, L->c0sq);
    }
    return ORC_OK;
}

/* van der Waals equation of state, p = rho T / (1 - b rho) - a rho^2. */
int orc_vdw_pressure(double a, double b, double T, double rho, double *p)
{
    if (!(rho > 0) || !(b * rho < 1.0)) return ORC_ENUMERIC;
    *p = rho * T / (1.0 - b * rho) - a * rho * rho;
    return ORC_OK;
}

/* Carnahan-Starling equation of state, Eq. (5.9) with R_g = 1:
 * p = rho T (1 + e + e^2 - e^3) / (1 - e)^3 - a rho^2, e = b rho / 4. */
int orc_cs_pressure(double a, double b, double T, double rho, double *p)
{
    double e = 0.25 * b * rho;
    if (!(rho > 0) || !(e < 1.0)) return ORC_ENUMERIC;
    double d = 1.0 - e;
    *p = rho * T * (1.0 + e + e * e - e * e * e) / (d * d * d) - a * rho * rho;
    return ORC_OK;
}

/* Pseudopotential of Eq. (3.8), psi = sqrt(2 (p_EOS - rho theta) / G) in
 * Hermite units with theta = 1 (the multiphase runs hold theta at 1, Section
 * 5.4); in lattice units rho theta -> rho c0^2 and the argument is divided by
 * c0^2, so that F^SC ~ -grad(p_EOS - rho c0^2). */
int orc_psi_eos(int lattice, int eos, double a, double b, double T, double G, double rho, double *psi)
{
    const orc_lattice *L = lattice_cached(lattice);
    if (!L) return ORC_EINVAL;
    double p;
    int rc;
    if (eos == ORC_EOS_VDW) rc = orc_vdw_pressure(a, b, T, rho, &p);
    else if (eos == ORC_EOS_CS) rc = orc_cs_pressure(a, b, T, rho, &p);
    else return ORC_EINVAL;
    if (rc) return rc;
    double arg = 2.0 * (p - rho * L->c0sq) / (G * L->c0sq);
    if (!(arg >= 0.0)) return ORC_ENUMERIC;
    *psi = sqrt(arg);
    return ORC_OK;
}

int orc_psi(int lattice, double a, double b, double T, double G, double rho, double *psi)
{
    return orc_psi_eos(lattice, ORC_EOS_VDW, a, b, T, G, rho, psi);
}

static long wrap(long x, long n)
{
    long r = x % n;
    return r < 0 ? r + n : r;
}

/* Eq. (3.8): F^SC(x) = -G psi(x) sum_i w_i psi(x + c_i) c_i, periodic. */
int orc_sc_force_field(int lattice, int nx, int ny, int nz, const double *psi, double G, double *Fsc)
{
    const orc_lattice *L = lattice_cached(lattice);
    if (!L || nx < 1 || ny < 1 || nz < 1) return ORC_EINVAL;
    long N = (long)nx * ny * nz;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (long cell = 0; cell < N; ++cell) {
        long x = cell % nx, y = (cell / nx) % ny, z = cell / ((long)nx * ny);
        double acc[3] = {0, 0, 0};
        for (int i = 0; i < L->Q; ++i) {
            long xs = wrap(x + L->c[i][0], nx), ys = wrap(y + L->c[i][1], ny), zs = wrap(z + L->c[i][2], nz);
            double ps = psi[xs + nx * (ys + (long)ny * zs)];
            for (int a = 0; a < 3; ++a) acc[a] += L->w[i] * ps * L->c[i][a];
        }
        for (int a = 0; a < 3; ++a) Fsc[a * N + cell] = -G * psi[cell] * acc[a];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Whole-grid simulation.                                                   */
/* ------------------------------------------------------------------------ */

struct orc_sim {
    orc_config cfg;
    const orc_lattice *L;
    int D, Q;
    long N;
    int dims[3];
    int wax;                /* wall-normal axis (last axis) */
    double *f;              /* [Q][N] pre-collision f^ */
    double *fpost;          /* [Q][N] post-collision */
    double *rho, *u, *theta;    /* stage-2 fields */
    double *force;          /* [3][N] total force density F */
    double *psi, *Fsc;      /* pseudopotential and its force */
    double *gradT;          /* [3][N] */
    double *theta_prev;     /* theta of the previous step (grad_lag) */
    int have_prev;
    double *jmom, *emom;    /* first moment [3][N] and energy moment [N] */
    double *trho, *tu, *ttheta; /* TMS targets: previous-step fields */
    long ncol;              /* cells per wall-normal layer */
    double *lost;           /* [2][ncol]: mass that left through each wall, per column, at the last streaming */
};

static void *xcalloc(long n, size_t sz)
{
    return calloc((size_t)(n > 0 ? n : 1), sz);
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->f); free(s->fpost); free(s->rho); free(s->u); free(s->theta); free(s->force);
    free(s->psi); free(s->Fsc); free(s->gradT); free(s->theta_prev); free(s->trho); free(s->tu); free(s->ttheta);
    free(s->jmom); free(s->emom); free(s->lost);
    free(s);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_create(const orc_config *cfg, orc_sim **out)
{
    *out = NULL;
    const orc_lattice *L = lattice_cached(cfg->lattice);
    if (!L) return ORC_EINVAL;
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return ORC_EINVAL;
    if (L->D == 2 && cfg->nz != 1) return ORC_EINVAL;
    if (!(cfg->tau_hat > 0.5)) return ORC_EINVAL;
    unsigned src = cfg->sources;
    if (src & ~(ORC_SRC_BODY | ORC_SRC_THERMAL | ORC_SRC_PTENSOR)) return ORC_EINVAL;
    if ((src & ORC_SRC_THERMAL) && (cfg->isothermal || !(cfg->prandtl > 0))) return ORC_EUNSUPPORTED;
    if (cfg->grad_lag != 0 && cfg->grad_lag != 1) return ORC_EINVAL;
    if ((src & ORC_SRC_PTENSOR) && (!cfg->isothermal || cfg->walls)) return ORC_EUNSUPPORTED;
    if (cfg->eos != ORC_EOS_VDW && cfg->eos != ORC_EOS_CS) return ORC_EINVAL;
    orc_sim *s = calloc(1, sizeof *s);
    if (!s) return ORC_EINVAL;
    s->cfg = *cfg;
    s->L = L;
    s->D = L->D;
    s->Q = L->Q;
    s->dims[0] = cfg->nx; s->dims[1] = cfg->ny; s->dims[2] = cfg->nz;
    s->wax = L->D - 1;
    if (cfg->walls && s->dims[s->wax] < 8) { free(s); return ORC_EINVAL; }
    s->N = (long)cfg->nx * cfg->ny * cfg->nz;
    long N = s->N;
    s->f = xcalloc(N * s->Q, sizeof(double));
    s->fpost = xcalloc(N * s->Q, sizeof(double));
    s->rho = xcalloc(N, sizeof(double));
    s->u = xcalloc(3 * N, sizeof(double));
    s->theta = xcalloc(N, sizeof(double));
    s->force = xcalloc(3 * N, sizeof(double));
    s->psi = xcalloc(N, sizeof(double));
    s->Fsc = xcalloc(3 * N, sizeof(double));
    s->gradT = xcalloc(3 * N, sizeof(double));
    s->theta_prev = xcalloc(N, sizeof(double));
    s->trho = xcalloc(N, sizeof(double));
    s->tu = xcalloc(3 * N, sizeof(double));
    s->ttheta = xcalloc(N, sizeof(double));
    s->jmom = xcalloc(3 * N, sizeof(double));
    s->emom = xcalloc(N, sizeof(double));
    s->ncol = N / s->dims[s->wax];
    s->lost = xcalloc(2 * s->ncol, sizeof(double));
    if (!s->jmom || !s->emom || !s->lost ||
        !s->f || !s->fpost || !s->rho || !s->u || !s->theta || !s->force || !s->psi || !s->Fsc ||
        !s->gradT || !s->trho || !s->tu || !s->ttheta || !s->theta_prev) {
        orc_destroy(s);
        return ORC_EINVAL;
    }
    *out = s;
    return ORC_OK;
}

static void coords(const orc_sim *s, long cell, long x[3])
{
    x[0] = cell % s->dims[0];
    x[1] = (cell / s->dims[0]) % s->dims[1];
    x[2] = cell / ((long)s->dims[0] * s->dims[1]);
}

static long cell_of(const orc_sim *s, const long x[3])
{
    return x[0] + s->dims[0] * (x[1] + (long)s->dims[1] * x[2]);
}

static void wall_outflow(orc_sim *s, const double *fp);

/* Initial state f^0 = f^eq(rho, u, theta) (Section 5 initial fields). */
int orc_init(orc_sim *s, const double *rho, const double *u, const double *theta)
{
    long N = s->N;
    int bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : bad)
#endif
    for (long cell = 0; cell < N; ++cell) {
        double uu[3] = {0, 0, 0}, fe[ORC_QMAX];
        for (int a = 0; a < s->D; ++a) uu[a] = u[a * N + cell];
        double th = s->cfg.isothermal ? 1.0 : theta[cell];
        if (!(rho[cell] > 0) || !(th > 0)) { bad = 1; continue; }
        orc_feq(s->cfg.lattice, rho[cell], uu, th, fe);
        for (int i = 0; i < s->Q; ++i) s->f[i * N + cell] = fe[i];
        s->trho[cell] = rho[cell];
        for (int a = 0; a < 3; ++a) s->tu[a * N + cell] = uu[a];
        s->ttheta[cell] = th;
    }
    if (bad) return ORC_EINVAL;
    s->have_prev = 0;
    /* Before the first step no population has left yet; the wall closure of
     * step 0 balances the mass the initial equilibrium would send out, as if
     * it were the post-collision state of a step before. */
    wall_outflow(s, s->f);
    return ORC_OK;
}

/* Mass that leaves the domain through each wall in the streaming of the
 * post-collision state fp: for every column along the wall-normal axis, the
 * populations of its first three nodes next to the wall that point out of the
 * domain (summed in node order, then velocity order). */
static void wall_outflow(orc_sim *s, const double *fp)
{
    if (!s->cfg.walls) return;
    const orc_lattice *L = s->L;
    long N = s->N, ncol = s->ncol;
    int nax = s->dims[s->wax];
    for (long col = 0; col < ncol; ++col)
        for (int wall = 0; wall < 2; ++wall) {
            double m = 0.0;
            for (int d = 0; d < 3; ++d) {
                long k = wall == 0 ? d : nax - 1 - d;
                long cell = col + k * ncol;
                for (int i = 0; i < L->Q; ++i) {
                    long dst = k + L->c[i][s->wax];
                    if (dst < 0 || dst >= nax) m += fp[i * N + cell];
                }
            }
            s->lost[wall * ncol + col] = m;
        }
}

/* Eq. (4.7) at one boundary node: the unknown populations (bit set in unknown)
 * become f_i = f_ibar + f^eq_i(tgt) - f^eq_ibar(loc), where loc is the state of
 * Eq. (4.8): the known populations plus the target equilibrium in the unknown
 * slots, with the shifted velocity (rho u = sum c f + F/2, F = rho g) and the
 * temperature of Eq. (4.5).  The local equilibrium is taken at the opposite
 * index (non-equilibrium bounce-back): a node already at the target state is
 * left unchanged, and a moving wall imposes its velocity (Section 5.1); with
 * the index i on both equilibria the unknowns reduce to plain bounce-back at
 * that state.  The node's populations f[Q] are read and the result written to
 * out[Q]; the mass of the rebuilt populations is returned. */
static double tms_node(const orc_sim *s, const double *f, const int *unknown, double rt, const double ut[3],
                       double tt, double *out)
{
    const orc_lattice *L = s->L;
    if (s->cfg.isothermal) tt = 1.0;
    double fet[ORC_QMAX], fel[ORC_QMAX];
    orc_feq(s->cfg.lattice, rt, ut, tt, fet);
    double rl = 0, jl[3] = {0, 0, 0}, el = 0;
    for (int i = 0; i < L->Q; ++i) {
        double fi = unknown[i] ? fet[i] : f[i];
        rl += fi;
        for (int a = 0; a < 3; ++a) jl[a] += fi * L->c[i][a];
        el += fi * (L->c[i][0] * L->c[i][0] + L->c[i][1] * L->c[i][1] + L->c[i][2] * L->c[i][2]);
    }
    double Fl[3], ul[3];
    for (int a = 0; a < 3; ++a) {
        Fl[a] = ((s->cfg.sources & ORC_SRC_BODY) && a < s->D) ? rl * s->cfg.g[a] : 0.0;
        ul[a] = (jl[a] + 0.5 * Fl[a]) / rl;
    }
    double tl = s->cfg.isothermal ? 1.0 : (el - rl * dot3(ul, ul) + dot3(ul, Fl)) / (rl * s->D * L->c0sq);
    orc_feq(s->cfg.lattice, rl, ul, tl, fel);
    double m = 0.0;
    for (int i = 0; i < L->Q; ++i) {
        out[i] = unknown[i] ? f[L->opp[i]] + fet[i] - fel[L->opp[i]] : f[i];
        if (unknown[i]) m += out[i];
    }
    return m;
}

/* Macroscopic state of Eq. (4.5) of one node's populations f[Q]. */
static void node_macro(const orc_sim *s, const double *f, double *rho, double u[3], double *theta)
{
    const orc_lattice *L = s->L;
    double r = 0, j[3] = {0, 0, 0}, e = 0;
    for (int i = 0; i < L->Q; ++i) {
        r += f[i];
        for (int a = 0; a < 3; ++a) j[a] += f[i] * L->c[i][a];
        e += f[i] * (L->c[i][0] * L->c[i][0] + L->c[i][1] * L->c[i][1] + L->c[i][2] * L->c[i][2]);
    }
    double F[3];
    for (int a = 0; a < 3; ++a) {
        F[a] = ((s->cfg.sources & ORC_SRC_BODY) && a < s->D) ? r * s->cfg.g[a] : 0.0;
        u[a] = (j[a] + 0.5 * F[a]) / r;
    }
    *rho = r;
    *theta = s->cfg.isothermal ? 1.0 : (e - r * dot3(u, u) + dot3(u, F)) / (r * s->D * L->c0sq);
}

/* Unknown set of the node at wall-normal index k: the populations whose
 * source node x - c_i lies outside the domain.  Returns their number. */
static int unknown_set(const orc_sim *s, long k, int *unknown)
{
    int n = 0, nax = s->dims[s->wax];
    for (int i = 0; i < s->L->Q; ++i) {
        long src = k - s->L->c[i][s->wax];
        unknown[i] = (src < 0 || src >= nax);
        n += unknown[i];
    }
    return n;
}

/* Target of a wall node (Section 4.3: computed from the boundary condition).
 * The wall node lies outside the fluid, half-way across the wall from the
 * first fluid node, so the boundary values hold half-way between the two:
 *   - impermeability: the populations the closure rebuilds along this column
 *     (wall node and fluid boundary nodes) carry exactly the mass that left
 *     through the wall in the last streaming, which fixes rho_tgt;
 *   - no slip and the wall temperature: after the closure the wall node holds
 *     the reflection 2 u_wall - u_1 (components along the wall) and
 *     2 theta_wall - theta_1 of the first fluid node's previous-step fields,
 *     which fixes the tangential u_tgt and theta_tgt;
 *   - the wall-normal u_tgt is the reflection itself.
 * These conditions (D + 1 equations; D in the isothermal mode) are solved by
 * Newton's method with a finite-difference Jacobian, started from the node's
 * previous-step density and the reflected fields.  v = (rho, tangential u,
 * theta) in that order. */
static int wall_target(const orc_sim *s, const double *f, const int *unknown, double mass_want,
                       const double udes[3], double thdes, double rprev, double rt_out[1], double ut_out[3],
                       double *tt_out)
{
    const int D = s->D, wax = s->wax;
    int idx[5], nv = 0; /* -1: rho, 0..2: u component, 3: theta */
    idx[nv++] = -1;
    for (int a = 0; a < D; ++a)
        if (a != wax) idx[nv++] = a;
    if (!s->cfg.isothermal) idx[nv++] = 3;
    double v[5];
    for (int q = 0; q < nv; ++q) v[q] = idx[q] == -1 ? rprev : idx[q] == 3 ? thdes : udes[idx[q]];
    double out[ORC_QMAX];
    for (int it = 0; it < 60; ++it) {
        double R[5], J[5][5];
        for (int col = -1; col < nv; ++col) {
            double vv[5];
            memcpy(vv, v, sizeof vv);
            double h = 0.0;
            if (col >= 0) {
                h = 1e-7 * (fabs(v[col]) + (idx[col] == -1 || idx[col] == 3 ? 0.0 : 1e-2));
                vv[col] += h;
            }
            double rt = rprev, ut[3] = {udes[0], udes[1], udes[2]}, tt = thdes;
            for (int q = 0; q < nv; ++q) {
                if (idx[q] == -1) rt = vv[q];
                else if (idx[q] == 3) tt = vv[q];
                else ut[idx[q]] = vv[q];
            }
            double m = tms_node(s, f, unknown, rt, ut, tt, out);
            double ra, ua[3], tha;
            node_macro(s, out, &ra, ua, &tha);
            double res[5];
            for (int q = 0; q < nv; ++q)
                res[q] = idx[q] == -1 ? m - mass_want : idx[q] == 3 ? tha - thdes : ua[idx[q]] - udes[idx[q]];
            if (col < 0) memcpy(R, res, sizeof R);
            else for (int q = 0; q < nv; ++q) J[q][col] = (res[q] - R[q]) / h;
        }
        /* J dv = -R by Gaussian elimination with partial pivoting */
        double A[5][6], dv[5];
        for (int q = 0; q < nv; ++q) {
            for (int c = 0; c < nv; ++c) A[q][c] = J[q][c];
            A[q][nv] = -R[q];
        }
        for (int k = 0; k < nv; ++k) {
            int piv = k;
            for (int q = k + 1; q < nv; ++q)
                if (fabs(A[q][k]) > fabs(A[piv][k])) piv = q;
            for (int c = 0; c <= nv; ++c) { double t = A[k][c]; A[k][c] = A[piv][c]; A[piv][c] = t; }
            if (A[k][k] == 0.0) return ORC_ENUMERIC;
            for (int q = k + 1; q < nv; ++q) {
                double fct = A[q][k] / A[k][k];
                for (int c = k; c <= nv; ++c) A[q][c] -= fct * A[k][c];
            }
        }
        for (int k = nv - 1; k >= 0; --k) {
            double acc = A[k][nv];
            for (int c = k + 1; c < nv; ++c) acc -= A[k][c] * dv[c];
            dv[k] = acc / A[k][k];
        }
        int done = 1;
        for (int q = 0; q < nv; ++q) {
            v[q] += dv[q];
            if (!isfinite(v[q])) return ORC_ENUMERIC;
            if (fabs(dv[q]) > 1e-14 * (1.0 + fabs(v[q]))) done = 0;
        }
        if (done) {
            rt_out[0] = rprev;
            for (int a = 0; a < 3; ++a) ut_out[a] = udes[a];
            *tt_out = thdes;
            for (int q = 0; q < nv; ++q) {
                if (idx[q] == -1) rt_out[0] = v[q];
                else if (idx[q] == 3) *tt_out = v[q];
                else ut_out[idx[q]] = v[q];
            }
            return ORC_OK;
        }
    }
    return ORC_ENUMERIC;
}

/* Section 4.3, Eqs. (4.7)-(4.8): TMS closure of the populations streamed in
 * from outside the walls.  Boundary nodes are the first three layers next to
 * each wall (the lattice reaches three nodes).  The first layer holds the
 * wall nodes, outside the fluid: the wall lies half-way between them and the
 * first fluid layer, so the fluid between the walls is n - 2 nodes high
 * (Sections 5.1 and 5.2: 54 of 56).  Fluid boundary nodes (second and third
 * layers) target their own previous-step fields; wall nodes take the target
 * that the boundary conditions fix (wall_target).  Per column, the fluid
 * boundary nodes are closed first, because the wall node's mass balance
 * counts what they rebuild. */
static int tms_fill(orc_sim *s)
{
    if (!s->cfg.walls) return ORC_OK;
    const orc_lattice *L = s->L;
    long N = s->N, ncol = s->ncol;
    int nax = s->dims[s->wax], D = s->D;
    int bad = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : bad)
#endif
    for (long col = 0; col < ncol; ++col) {
        for (int wall = 0; wall < 2; ++wall) {
            double f[ORC_QMAX], out[ORC_QMAX];
            int unknown[ORC_QMAX];
            double mass_fluid = 0.0;
            for (int d = 1; d < 3; ++d) {
                long k = wall == 0 ? d : nax - 1 - d;
                long cell = col + k * ncol;
                if (!unknown_set(s, k, unknown)) continue;
                for (int i = 0; i < L->Q; ++i) f[i] = s->f[i * N + cell];
                double ut[3] = {s->tu[cell], s->tu[N + cell], s->tu[2 * N + cell]};
                mass_fluid += tms_node(s, f, unknown, s->trho[cell], ut, s->ttheta[cell], out);
                for (int i = 0; i < L->Q; ++i) s->f[i * N + cell] = out[i];
            }
            long k = wall == 0 ? 0 : nax - 1;
            long cell = col + k * ncol;
            long c1 = col + (wall == 0 ? 1 : nax - 2) * ncol;
            unknown_set(s, k, unknown);
            for (int i = 0; i < L->Q; ++i) f[i] = s->f[i * N + cell];
            double udes[3] = {0, 0, 0};
            for (int a = 0; a < D; ++a) udes[a] = 2.0 * s->cfg.u_wall[wall][a] - s->tu[a * N + c1];
            double thdes = s->cfg.isothermal ? 1.0 : 2.0 * s->cfg.theta_wall[wall] - s->ttheta[c1];
            double rt, ut[3], tt;
            if (wall_target(s, f, unknown, s->lost[wall * ncol + col] - mass_fluid, udes, thdes, s->trho[cell],
                            &rt, ut, &tt)) {
                bad = 1;
                continue;
            }
            tms_node(s, f, unknown, rt, ut, tt, out);
            for (int i = 0; i < L->Q; ++i) s->f[i * N + cell] = out[i];
        }
    }
    return bad ? ORC_ENUMERIC : ORC_OK;
}

/* Eq. (4.5): rho = F^_0, rho u = F^_1 + F/2 (G_1 = F exactly), and
 * rho D c0^2 theta = tr F^_2 - rho |u|^2 + tr G_2 / 2 with tr G_2 = 2 u.F for
 * the body force; theta = 1 in the isothermal (multiphase) mode. */
static int macroscopic(orc_sim *s)
{
    const orc_lattice *L = s->L;
    const orc_config *cf = &s->cfg;
    long N = s->N;
    int bad = 0;
    double *j = s->jmom, *e = s->emom;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (long cell = 0; cell < N; ++cell) {
        double r = 0, jj[3] = {0, 0, 0}, ee = 0;
        for (int i = 0; i < L->Q; ++i) {
            double fi = s->f[i * N + cell];
            r += fi;
            for (int a = 0; a < 3; ++a) jj[a] += fi * L->c[i][a];
            ee += fi * (L->c[i][0] * L->c[i][0] + L->c[i][1] * L->c[i][1] + L->c[i][2] * L->c[i][2]);
        }
        s->rho[cell] = r;
        for (int a = 0; a < 3; ++a) j[a * N + cell] = jj[a];
        e[cell] = ee;
    }
    if (cf->sources & ORC_SRC_PTENSOR) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : bad)
#endif
        for (long cell = 0; cell < N; ++cell)
            if (orc_psi_eos(cf->lattice, cf->eos, cf->eos_a, cf->eos_b, cf->eos_T, cf->sc_G, s->rho[cell], &s->psi[cell]))
                bad = 1;
        if (bad) return ORC_ENUMERIC;
        orc_sc_force_field(cf->lattice, s->dims[0], s->dims[1], s->dims[2], s->psi, cf->sc_G, s->Fsc);
    }
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : bad)
#endif
    for (long cell = 0; cell < N; ++cell) {
        double r = s->rho[cell];
        if (!(r > 0)) { bad = 1; continue; }
        double F[3], uu[3];
        for (int a = 0; a < 3; ++a) {
            F[a] = 0.0;
            if (a < s->D) {
                if (cf->sources & ORC_SRC_BODY) F[a] += r * cf->g[a];
                if (cf->sources & ORC_SRC_PTENSOR) F[a] += s->Fsc[a * N + cell];
            }
            s->force[a * N + cell] = F[a];
            uu[a] = (j[a * N + cell] + 0.5 * F[a]) / r;
        }
        double th = cf->isothermal ? 1.0 : (e[cell] - r * dot3(uu, uu) + dot3(uu, F)) / (r * s->D * L->c0sq);
        if (!isfinite(th) || !(th > 0)) bad = 1;
        for (int a = 0; a < 3; ++a) s->u[a * N + cell] = uu[a];
        s->theta[cell] = th;
    }
    return bad ? ORC_ENUMERIC : ORC_OK;
}

/* Section 3.2: grad theta by second-order central differences; along the
 * wall-normal axis the wall layers use a one-sided first difference.  The
 * section leaves the time level open: theta of the same step, or with
 * grad_lag of the previous step (the initial state's before the first). */
static void grad_theta(orc_sim *s)
{
    long N = s->N;
    const double *theta = (s->cfg.grad_lag && s->have_prev) ? s->theta_prev : s->theta;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (long cell = 0; cell < N; ++cell) {
        long x[3];
        coords(s, cell, x);
        for (int a = 0; a < 3; ++a) {
            double g = 0.0;
            if (a < s->D) {
                long n = s->dims[a];
                long xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
                if (s->cfg.walls && a == s->wax) {
                    if (x[a] == 0) { xp[a] = 1; xm[a] = 0; g = theta[cell_of(s, xp)] - theta[cell_of(s, xm)]; }
                    else if (x[a] == n - 1) { xp[a] = n - 1; xm[a] = n - 2; g = theta[cell_of(s, xp)] - theta[cell_of(s, xm)]; }
                    else { xp[a] = x[a] + 1; xm[a] = x[a] - 1; g = 0.5 * (theta[cell_of(s, xp)] - theta[cell_of(s, xm)]); }
                } else {
                    xp[a] = wrap(x[a] + 1, n);
                    xm[a] = wrap(x[a] - 1, n);
                    g = 0.5 * (theta[cell_of(s, xp)] - theta[cell_of(s, xm)]);
                }
            }
            s->gradT[a * N + cell] = g;
        }
    }
}

/* Eq. (4.4) right-hand side: f* = f^ - (f^ - f^eq)/tau_hat + (1 - 1/(2 tau_hat)) S. */
static void collide(orc_sim *s, double *fpost)
{
    const orc_lattice *L = s->L;
    const orc_config *cf = &s->cfg;
    long N = s->N;
    double c0 = sqrt(L->c0sq);
    double th_ = cf->tau_hat;
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (long cell = 0; cell < N; ++cell) {
        double r = s->rho[cell], th = s->theta[cell];
        double U[3], Phi[3], gT[3], Fsc[3];
        for (int a = 0; a < 3; ++a) {
            U[a] = s->u[a * N + cell] / c0;
            Phi[a] = s->force[a * N + cell] / c0;
            gT[a] = s->gradT[a * N + cell];
            Fsc[a] = s->Fsc[a * N + cell];
        }
        for (int i = 0; i < L->Q; ++i) {
            double xi[3];
            scaled(L, i, xi);
            double fe = feq_one(s->D, L->w[i], xi, r, U, th);
            double S = 0.0;
            if (cf->sources & (ORC_SRC_BODY | ORC_SRC_PTENSOR))
                S += force_one(s->D, L->w[i], xi, U, Phi, th);
            if (cf->sources & ORC_SRC_THERMAL)
                S += thermal_one(s->D, L->w[i], xi, L->c[i], r, th, cf->prandtl, gT);
            if (cf->sources & ORC_SRC_PTENSOR)
                S += ptensor_one(s->D, L->w[i], xi, th_ - 0.5, cf->ptensor_k, cf->sc_G, Fsc, s->psi[cell], L->c0sq);
            double fi = s->f[i * N + cell];
            fpost[i * N + cell] = fi - (fi - fe) / th_ + (1.0 - 1.0 / (2.0 * th_)) * S;
        }
    }
}

/* Left-hand side of Eq. (4.4): push streaming, periodic except across walls,
 * where populations leaving the domain are dropped (their slots are rebuilt
 * by the wall closure at the next step). */
static void stream(orc_sim *s, const double *fpost)
{
    const orc_lattice *L = s->L;
    long N = s->N;
    if (s->cfg.walls) {
        for (long k = 0; k < N * s->Q; ++k) s->f[k] = NAN;
    }
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (long cell = 0; cell < N; ++cell) {
        long x[3];
        coords(s, cell, x);
        for (int i = 0; i < L->Q; ++i) {
            long y[3];
            int out = 0;
            for (int a = 0; a < 3; ++a) {
                long t = x[a] + L->c[i][a];
                if (s->cfg.walls && a == s->wax) {
                    if (t < 0 || t >= s->dims[a]) out = 1;
                    y[a] = t;
                } else {
                    y[a] = wrap(t, s->dims[a]);
                }
            }
            if (!out) s->f[i * N + cell_of(s, y)] = fpost[i * N + cell];
        }
    }
}

static int stages_to_collision(orc_sim *s)
{
    int rc = tms_fill(s);
    if (rc) return rc;
    rc = macroscopic(s);
    if (rc) return rc;
    if (s->cfg.sources & ORC_SRC_THERMAL) grad_theta(s);
    else memset(s->gradT, 0, sizeof(double) * 3 * s->N);
    return ORC_OK;
}

int orc_step(orc_sim *s, int nsteps)
{
    for (int n = 0; n < nsteps; ++n) {
        int rc = stages_to_collision(s);
        if (rc) return rc;
        collide(s, s->fpost);
        if (s->cfg.grad_lag) {
            memcpy(s->theta_prev, s->theta, sizeof(double) * s->N);
            s->have_prev = 1;
        }
        if (s->cfg.walls) {
            memcpy(s->trho, s->rho, sizeof(double) * s->N);
            memcpy(s->tu, s->u, sizeof(double) * 3 * s->N);
            memcpy(s->ttheta, s->theta, sizeof(double) * s->N);
            wall_outflow(s, s->fpost);
        }
        stream(s, s->fpost);
    }
    return ORC_OK;
}

int orc_collide_only(orc_sim *s, double *fpost)
{
    int rc = stages_to_collision(s);
    if (rc) return rc;
    collide(s, fpost);
    return ORC_OK;
}

int orc_fields(orc_sim *s, double *rho, double *u, double *theta)
{
    int rc = stages_to_collision(s);
    if (rc) return rc;
    long N = s->N;
    memcpy(rho, s->rho, sizeof(double) * N);
    for (int a = 0; a < s->D; ++a) memcpy(u + a * N, s->u + a * N, sizeof(double) * N);
    memcpy(theta, s->theta, sizeof(double) * N);
    return ORC_OK;
}

/* Global totals: mass sum rho, momentum sum rho u = sum (F^_1 + F/2), and
 * energy sum (rho |u|^2 + rho D c0^2 theta)/2 = sum (tr F^_2 + u.F)/2. */
int orc_reduce(orc_sim *s, double out[5])
{
    int rc = stages_to_collision(s);
    if (rc) return rc;
    long N = s->N;
    double m = 0, p[3] = {0, 0, 0}, en = 0;
    for (long cell = 0; cell < N; ++cell) {
        double r = s->rho[cell];
        double uu[3] = {s->u[cell], s->u[N + cell], s->u[2 * N + cell]};
        m += r;
        for (int a = 0; a < 3; ++a) p[a] += r * uu[a];
        en += 0.5 * (r * dot3(uu, uu) + r * s->D * s->L->c0sq * s->theta[cell]);
    }
    out[0] = m;
    out[1] = p[0];
    out[2] = p[1];
    out[3] = p[2];
    out[4] = en;
    return ORC_OK;
}

int orc_get_state(orc_sim *s, double *f)
{
    memcpy(f, s->f, sizeof(double) * s->N * s->Q);
    return ORC_OK;
}

int orc_set_state(orc_sim *s, const double *f)
{
    memcpy(s->f, f, sizeof(double) * s->N * s->Q);
    return ORC_OK;
}
