/*
 * Declarations of the CPU FP64 oracle of the sG-PM particle method.
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product library.
 */
#ifndef SGPM_ORACLE_H
#define SGPM_ORACLE_H
#include <stdint.h>

#define ORC_QMAX 128
#define ORC_PMAX 128
#define ORC_NTHETA 32
#define ORC_EDGE_TRIES 64

typedef struct {
    int dim_z;          /* 0, 1 or 2 uncertain inputs                         */
    int degree;         /* gPC total degree M                                 */
    int nodes_1d;       /* Gauss-Legendre nodes per uncertain dimension       */
    long n_particles;
    int gap_mode;       /* 0: gap [eV] = gap0 (1 + gap_rel z); 1: width [nm]  */
    int gap_dim;        /* which z drives the gap/width, -1 = deterministic    */
    double gap0, gap_rel;
    int field_dim;      /* which z drives the field, -1 = deterministic        */
    double field0, field_rel;  /* V/m */
    double fermi_eV, temp_K, alpha;
    int nk;             /* histogram cells per axis                           */
    double lk_eV;       /* half-width of the grid, L_k hbar v_F               */
    int pauli;          /* 1: Pauli acceptance on                              */
    int final_state;    /* 0: energy conserving, 1: paper-literal |k| +/- w/v_F */
    double rate_scale[6];
    uint64_t seed;
    uint32_t instance;
    int c_max;          /* cap on collisions per particle per step            */
    int splitting;      /* 0: drift dt then collisions (the paper's first-order
                           splitting); 1: Strang, drift dt/2, collisions, drift
                           dt/2 (Sec. 3 mentions higher-order splittings)      */
    double init_temp_K; /* temperature of the Fermi-Dirac initial datum (and of
                           the density n used for J); 0 = temp_K              */
} orc_params;

typedef struct {
    long long collisions, events, pauli_rejected, edge_exhausted, cmax_hits, out_of_grid;
} orc_counters;

typedef struct {
    orc_params p;
    int P, Q;
    double hbar, kT_eV;     /* lattice k_B T: Bose factors, acoustic rate       */
    double kT0_eV;          /* k_B T of the Fermi-Dirac initial datum           */
    double *z, *w, *psi, *Ehat, *eps0, *width, *field, *density;
    double C_ac, C_O, C_K, n_O, n_K, hw_O, hw_K, edge_kappa_coef;
    double *C_edge;
    double dk;
    double gl10_x[10], gl10_w[10];
    int *cdf_np;
    double **cdf_x, **cdf_lo, **cdf_hi;
    double *kx, *ky;        /* [P][N] coefficients, kappa units (eV) */
    uint32_t *H, *Hmax;     /* [Q][nk*nk] histogram of the current state, [Q] max */
    uint32_t *cap;          /* [Q] maximum occupation: the largest cell count of the
                               state given to init / set_state, per node       */
    uint32_t *excess;       /* [Q] particles above the cap in the current histogram */
    long step;
    orc_counters counters;
    int threads;
} orc_sim;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u52(uint32_t whi, uint32_t wlo);
void orc_gauss_legendre(int n, double *x, double *w);
double orc_legendre_orthonormal(int k, double x);
int orc_num_modes(int dim_z, int degree);
orc_sim *orc_create(const orc_params *p);
void orc_destroy(orc_sim *s);
double orc_fd_inverse_cdf(const orc_sim *s, int q, uint32_t whi, uint32_t wlo);
double orc_edge_integral(double kap, double c);
void orc_rates(const orc_sim *s, int q, double kx, double ky, double out[6]);
double orc_theta_ac(double u1, double u2);
long orc_cell(const orc_sim *s, double x, double y);
void orc_collide_particle(const orc_sim *s, long i, uint32_t step, double dt,
                          double *chx, double *chy, orc_counters *cnt);
void orc_moments(const orc_sim *s, double *out);
void orc_init(orc_sim *s);
void orc_run(orc_sim *s, double dt, int n_steps, double *moments_out, uint32_t *excess_out);
void orc_reconstruct_f(const orc_sim *s, int nbins, double emin, double emax,
                       double *nodes_out, double *modes_out);
/* Moments at points z ([nz][dim_z]) of the particle expansion: out[nz][4] =
 * V_x, V_y (m/s), mean energy (eV), J_x (A/m). */
void orc_moments_at(const orc_sim *s, int nz, const double *z, double *out);
/* Equilibrium electron density (1/m^2) of a band with minimum e0 (eV), in
 * closed form with the dilogarithm. */
double orc_density_closed(double e0, double mu, double kT, double hbar);
void orc_reconstruct_f_at(const orc_sim *s, const double *z, int nbins, double emin,
                          double emax, double *out);

#endif
