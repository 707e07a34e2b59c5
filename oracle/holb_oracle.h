/*
 * holb_oracle.h -- FP64 CPU oracle for the high-order BGK lattice Boltzmann
 * step with Hermite source terms (Li, Wan, Gui, Yang, Tu, Jiang,
 * "Constructing the body source for high-order lattice Boltzmann method",
 * arXiv:2411.10751).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct CPU
 * implementation used to check the HIP path.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * Layout: populations f[i*N + cell], fields rho[cell], u[a*N + cell],
 * theta[cell], with cell = x + nx*(y + ny*z) and N = nx*ny*nz.
 * Every function returns 0 on success and a negative ORC_E* code on error.
 */
#ifndef HOLB_ORACLE_H
#define HOLB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENUMERIC (-4)
#define ORC_EUNSUPPORTED (-5)

#define ORC_D2Q37 0
#define ORC_D3Q39 1

#define ORC_SRC_BODY 1u
#define ORC_SRC_THERMAL 2u
#define ORC_SRC_PTENSOR 4u

#define ORC_EOS_VDW 0        /* p = rho*T/(1-b*rho) - a*rho^2 */
#define ORC_EOS_CS 1         /* Carnahan-Starling, Eq. (5.9), R_g = 1 */

#define ORC_QMAX 39

typedef struct {
    int lattice;           /* ORC_D2Q37 or ORC_D3Q39 */
    int nx, ny, nz;        /* nz == 1 for D2Q37 */
    double tau_hat;        /* shifted relaxation time, Eq. (4.3) */
    unsigned sources;      /* ORC_SRC_* mask */
    int isothermal;        /* 1: theta held at 1 (Section 5.4) */
    double g[3];           /* body-force acceleration, F = rho*g */
    double prandtl;        /* Pr of the thermal-dissipation source */
    double eos_a, eos_b, eos_T; /* parameters a, b, T of the equation of state (field eos) */
    double sc_G;           /* pseudopotential coupling G (paper: -1) */
    double ptensor_k;      /* free parameter k of Eq. (3.12) */
    int walls;             /* 0: periodic; 1: TMS walls normal to last axis */
    double theta_wall[2];  /* [0] low wall (index 0), [1] high wall */
    double u_wall[2][3];   /* wall velocities, same order */
    int eos;               /* ORC_EOS_VDW or ORC_EOS_CS */
    int grad_lag;          /* 1: the thermal source takes grad theta of the previous step's theta */
} orc_config;

typedef struct {
    int D, Q;
    int c[ORC_QMAX][3];
    double w[ORC_QMAX];
    double c0sq;
    int opp[ORC_QMAX];
} orc_lattice;

typedef struct orc_sim orc_sim;

/* Velocity set and weights, derived from the isotropy (moment) equations. */
int orc_lattice_get(int lattice, orc_lattice *out);

/* Single-node kinetic algebra (Hermite units inside, lattice units outside). */
int orc_feq(int lattice, double rho, const double *u, double theta, double *out);
int orc_src_force(int lattice, const double *F, const double *u, double theta, double *out);
int orc_src_thermal(int lattice, double rho, double theta, double prandtl,
                    const double *grad_theta, double *out);
int orc_src_ptensor(int lattice, double tau_hat, double k, double G,
                    const double *Fsc, double psi, double *out);
int orc_vdw_pressure(double a, double b, double T, double rho, double *p);
int orc_cs_pressure(double a, double b, double T, double rho, double *p);
int orc_psi(int lattice, double a, double b, double T, double G, double rho, double *psi);
/* psi of Eq. (3.8) for either equation of state (orc_psi is the van der Waals case). */
int orc_psi_eos(int lattice, int eos, double a, double b, double T, double G, double rho, double *psi);
/* F^SC of Eq. (3.8) for a periodic psi field (nz == 1 for 2D). */
int orc_sc_force_field(int lattice, int nx, int ny, int nz, const double *psi, double G,
                       double *Fsc);

/* Whole-grid time stepping. */
int orc_create(const orc_config *cfg, orc_sim **out);
int orc_init(orc_sim *s, const double *rho, const double *u, const double *theta);
int orc_step(orc_sim *s, int nsteps);
int orc_fields(orc_sim *s, double *rho, double *u, double *theta);
int orc_reduce(orc_sim *s, double out[5]);
/* The populations f[Q*N] only: with walls, the previous-step targets and the
 * mass that left through each wall stay as they are. */
int orc_get_state(orc_sim *s, double *f);
int orc_set_state(orc_sim *s, const double *f);
int orc_collide_only(orc_sim *s, double *fpost);
void orc_destroy(orc_sim *s);
int orc_num_threads(void);
/* Threads of the following OpenMP regions (n > 0; timing of the CPU baseline). */
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
