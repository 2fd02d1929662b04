/*
 * Plain CPU FP64 oracle for the stochastic-Galerkin particle method (sG-PM)
 * of Medaglia, Nastasi, Romano, Zanella, "Uncertainty quantification for
 * charge transport in GNRs through particle Galerkin methods for the
 * semiclassical Boltzmann equation" (arXiv:2404.19602).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file.  It exists so that the tests, the smoke check and
 * the CPU-baseline leg of the benchmark can compare the HIP library with a
 * slow, sequential, obviously correct implementation written directly from
 * the paper.  It shares no code, header, table or constant with the HIP
 * library.
 *
 * Units used throughout:
 *   energies                       eV
 *   wave-vectors  kappa = hbar v_F k   eV   (the paper's grid is stated in these
 *                                        units: L_k hbar v_F = 5 eV, Sec. 5)
 *   rates                          1/s
 *   times                          s
 *   electric field                 V/m
 * The drift of kappa in one step is then v_F * E * dt (in eV).
 *
 * Readings of points where the paper is silent, garbled or ambiguous are
 * marked "Reading:" below; each is listed in the design notes of the
 * repository.
 *
 * Parity status: every function here is pinned by a CPU test (closed forms,
 * invariants, special cases, library routines, brute force).  The absolute
 * time curves V_x(t), E(t) cannot be pinned to the paper (its figures are
 * absent and its tables only give relative errors against a solver it does
 * not describe): "parity unpinned" for those absolute curves.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "sgpm_oracle.h"

/* ------------------------------------------------------------------------ */
/* Physical constants: SI 2019 exact values.                                */
/* ------------------------------------------------------------------------ */
static const double Q_E = 1.602176634e-19;   /* elementary charge, C       */
static const double H_PLANCK = 6.62607015e-34;/* Planck constant, J s      */
static const double K_B = 1.380649e-23;      /* Boltzmann constant, J/K     */
#define PI_D 3.14159265358979323846

/* Table 1 of the paper (Sec. 5), converted to SI. */
static const double V_F = 1.0e6;              /* 1e8 cm/s                   */
static const double SIGMA_M = 7.6e-7;         /* 7.6e-8 g/cm^2 -> kg/m^2    */
static const double HW_O_EV = 0.1646;         /* 164.6 meV                  */
static const double HW_K_EV = 0.124;          /* 124 meV                    */
static const double V_P = 2.0e4;              /* 2e6 cm/s                   */
static const double D_AC_EV = 6.8;            /* eV                         */
static const double D_O_EV_PER_M = 1.0e11;    /* 1e9 eV/cm                  */
static const double D_K_EV_PER_M = 3.5e10;    /* 3.5e8 eV/cm                */
static const double N_I = 1.0e6;              /* 1e4 1/cm -> 1/m            */
static const double V0_EV_M2 = 4.56e-18;      /* 4.56e-14 eV cm^2 -> eV m^2 */
static const double A_EDGE = 1.0e-10;         /* 1e-8 cm -> m               */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), from its published     */
/* definition.  Counter layout (a convention of this code, which the GPU     */
/* path follows by definition only): c0 = particle, c1 = step (0xFFFFFFFF   */
/* during initialisation),                                                   */
/* c2 = (collision << 8) | purpose, c3 = instance; key = seed.               */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

enum { PUR_XI = 0, PUR_SEL = 1, PUR_ANG = 2, PUR_EDGE0 = 16, PUR_INIT = 255 };

/* Open-interval uniform in (0,1) from two words, 52 bits:
 *   m = ((w_hi << 32) | w_lo) >> 12,  u = (m + 1/2) 2^-52,
 * every value exactly representable, so 0 < u < 1 strictly.                */
static uint64_t u52_int(uint32_t whi, uint32_t wlo)
{
    return ((((uint64_t)whi) << 32) | (uint64_t)wlo) >> 12;
}
double orc_u52(uint32_t whi, uint32_t wlo)
{
    return ((double)u52_int(whi, wlo) + 0.5) * 0x1p-52;
}

static void draw(const orc_sim *s, uint32_t particle, uint32_t step,
                 uint32_t coll, uint32_t purpose, uint32_t out[4])
{
    uint32_t ctr[4] = { particle, step, (coll << 8) | purpose, s->p.instance };
    uint32_t key[2] = { (uint32_t)(s->p.seed & 0xffffffffu), (uint32_t)(s->p.seed >> 32) };
    orc_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre quadrature on [-1,1] by Newton's method on P_n.            */
/* ------------------------------------------------------------------------ */
/* P_n(z) and P_{n-1}(z) by the three-term recurrence */
static void legendre_pair(int n, double z, double *pn, double *pnm1)
{
    double p0 = 1.0, p1 = z;
    if (n == 1) { *pn = z; *pnm1 = 1.0; return; }
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1; p1 = p2;
    }
    *pn = p1; *pnm1 = p0;
}

void orc_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        /* initial guess for the i-th largest root */
        double z = cos(PI_D * (i + 0.75) / (n + 0.5));
        double pn, pnm1, dp;
        for (int it = 0; it < 100; ++it) {
            legendre_pair(n, z, &pn, &pnm1);
            dp = n * (z * pn - pnm1) / (z * z - 1.0);   /* P_n'(z) */
            double dz = pn / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        legendre_pair(n, z, &pn, &pnm1);
        dp = n * (z * pn - pnm1) / (z * z - 1.0);
        x[n - 1 - i] = z;                               /* ascending */
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Orthonormal Legendre polynomial psi_k(x) = sqrt(2k+1) P_k(x), orthonormal
 * for the uniform density 1/2 on [-1,1] (Wiener-Askey choice for a uniform
 * random input, Sec. 4.1). */
double orc_legendre_orthonormal(int k, double x)
{
    double p0 = 1.0, p1 = x;
    if (k == 0) return 1.0;
    for (int j = 2; j <= k; ++j) {
        double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1; p1 = p2;
    }
    return sqrt(2.0 * k + 1.0) * p1;
}

/* Multi-index of basis function h: for d_z = 2 the total-degree basis in
 * graded order (t = 0..M; within t the first exponent runs from t down to 0). */
static void multi_index(int dim_z, int h, int *a1, int *a2)
{
    if (dim_z <= 1) { *a1 = h; *a2 = 0; return; }
    int t = 0, start = 0;
    while (start + (t + 1) <= h) { start += t + 1; ++t; }
    int off = h - start;
    *a1 = t - off;
    *a2 = off;
}

static double basis_eval(int dim_z, int h, const double *z)
{
    if (dim_z == 0) return 1.0;
    int a1, a2;
    multi_index(dim_z, h, &a1, &a2);
    if (dim_z == 1) return orc_legendre_orthonormal(a1, z[0]);
    return orc_legendre_orthonormal(a1, z[0]) * orc_legendre_orthonormal(a2, z[1]);
}

int orc_num_modes(int dim_z, int degree)
{
    if (dim_z == 0) return 1;
    if (dim_z == 1) return degree + 1;
    return (degree + 1) * (degree + 2) / 2;
}

/* ------------------------------------------------------------------------ */
/* Fermi-Dirac energy density and its CDF (initial condition).              */
/* The initial datum is Fermi-Dirac in k (Sec. 2 and Sec. 4).  In polar      */
/* coordinates dk = eps/(hbar v_F)^2 d eps d theta (Appendix Jacobian), so   */
/* the particle energy has density proportional to eps f_FD(eps) on          */
/* [eps0, inf) and the angle is uniform.                                     */
/* ------------------------------------------------------------------------ */
static double fd_weight(const orc_sim *s, double e)
{
    return e / (1.0 + exp((e - s->p.fermi_eV) / s->kT0_eV));
}

/* integral of eps f_FD over [a, b] by 10-point Gauss-Legendre */
static double fd_integral(const orc_sim *s, double a, double b)
{
    double c = 0.5 * (a + b), h = 0.5 * (b - a), acc = 0.0;
    for (int j = 0; j < 10; ++j) acc += s->gl10_w[j] * fd_weight(s, c + h * s->gl10_x[j]);
    return acc * h;
}

/* Per node: panels of width kT/2 from eps0 to max(eps_F, eps0) + 80 kT
 * (T the temperature of the initial datum),
 * with cumulative integrals from below (lo) and from above (hi).  The
 * neglected tail is about e^-80 of the total, below 1e-18 of the smallest
 * upper-tail probability a 52-bit uniform can ask for (2^-53 ~ e^-36.7). */
static void build_cdf_tables(orc_sim *s)
{
    int Q = s->Q;
    s->cdf_np = (int *)calloc((size_t)Q, sizeof(int));
    s->cdf_x = (double **)calloc((size_t)Q, sizeof(double *));
    s->cdf_lo = (double **)calloc((size_t)Q, sizeof(double *));
    s->cdf_hi = (double **)calloc((size_t)Q, sizeof(double *));
    for (int q = 0; q < Q; ++q) {
        double a = s->eps0[q];
        double top = (s->p.fermi_eV > a ? s->p.fermi_eV : a) + 80.0 * s->kT0_eV;
        double hpan = 0.5 * s->kT0_eV;
        int np = (int)ceil((top - a) / hpan);
        s->cdf_np[q] = np;
        s->cdf_x[q] = (double *)malloc(sizeof(double) * (size_t)(np + 1));
        s->cdf_lo[q] = (double *)malloc(sizeof(double) * (size_t)(np + 1));
        s->cdf_hi[q] = (double *)malloc(sizeof(double) * (size_t)(np + 1));
        for (int j = 0; j <= np; ++j) s->cdf_x[q][j] = a + hpan * j;
        double *pan = (double *)malloc(sizeof(double) * (size_t)np);
        for (int j = 0; j < np; ++j) pan[j] = fd_integral(s, s->cdf_x[q][j], s->cdf_x[q][j + 1]);
        s->cdf_lo[q][0] = 0.0;
        for (int j = 0; j < np; ++j) s->cdf_lo[q][j + 1] = s->cdf_lo[q][j] + pan[j];
        s->cdf_hi[q][np] = 0.0;
        for (int j = np - 1; j >= 0; --j) s->cdf_hi[q][j] = s->cdf_hi[q][j + 1] + pan[j];
        free(pan);
    }
}

/* Solve F_q(eps) = u, given u as the integer m of orc_u52 (u = (m+1/2)2^-52).
 * For u <= 1/2 the lower cumulative integral is matched to u Z; above, the
 * upper one is matched to (1-u) Z, computed exactly from the integer, so the
 * tail keeps full relative precision.  Bisection until the bracket cannot
 * shrink. */
static double fd_inverse_cdf_m(const orc_sim *s, int q, uint64_t m)
{
    int np = s->cdf_np[q];
    const double *x = s->cdf_x[q], *lo = s->cdf_lo[q], *hi = s->cdf_hi[q];
    double Z = lo[np];
    int upper = (m >= (1ull << 51));
    double target;
    if (!upper) target = ((double)m + 0.5) * 0x1p-52 * Z;
    else        target = ((double)((1ull << 52) - 1ull - m) + 0.5) * 0x1p-52 * Z;
    /* locate the panel */
    int j;
    if (!upper) {
        j = 0;
        while (j < np - 1 && lo[j + 1] <= target) ++j;
    } else {
        j = np - 1;
        while (j > 0 && hi[j] <= target) --j;
    }
    double a = x[j], b = x[j + 1];
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (a + b);
        if (mid <= a || mid >= b) break;
        if (!upper) {
            double F = lo[j] + fd_integral(s, x[j], mid);
            if (F < target) a = mid; else b = mid;
        } else {
            double G = fd_integral(s, mid, x[j + 1]) + hi[j + 1];
            if (G > target) a = mid; else b = mid;
        }
    }
    return 0.5 * (a + b);
}

double orc_fd_inverse_cdf(const orc_sim *s, int q, uint32_t whi, uint32_t wlo)
{
    return fd_inverse_cdf_m(s, q, u52_int(whi, wlo));
}

/* Electron density n(z) = g_s g_v/(2 pi)^2 int f(0,k,z) dk  (Sec. 3 eq. den,
 * Sec. 4.2), g_s = g_v = 2:  n = (2/pi) (hbar v_F)^-2 int eps f_FD d eps.   */
static double density_m2(const orc_sim *s, int q)
{
    double hvf_eV_m = s->hbar * V_F / Q_E;       /* hbar v_F in eV m */
    double Z = s->cdf_lo[q][s->cdf_np[q]];       /* eV^2 */
    return (2.0 / PI_D) * Z / (hvf_eV_m * hvf_eV_m);
}

/* ------------------------------------------------------------------------ */
/* Instance set-up.                                                         */
/* ------------------------------------------------------------------------ */
static double z_coord(const orc_sim *s, int q, int d) { return s->z[q * 2 + d]; }

orc_sim *orc_create(const orc_params *p)
{
    if (p->dim_z < 0 || p->dim_z > 2) return NULL;
    if (p->splitting != 0 && p->splitting != 1) return NULL;
    if (p->degree < 0 || p->nodes_1d < 1) return NULL;
    if (p->n_particles < 1) return NULL;
    if (p->temp_K <= 0 || p->nk < 1 || p->lk_eV <= 0 || p->alpha < 0) return NULL;
    if (!(p->init_temp_K >= 0)) return NULL;
    if (p->gap_dim >= p->dim_z || p->field_dim >= p->dim_z) return NULL;
    if (p->c_max < 1 || p->c_max > 255) return NULL;

    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->p = *p;
    s->hbar = H_PLANCK / (2.0 * PI_D);
    s->kT_eV = K_B * p->temp_K / Q_E;
    s->kT0_eV = K_B * (p->init_temp_K > 0 ? p->init_temp_K : p->temp_K) / Q_E;
    s->P = orc_num_modes(p->dim_z, p->degree);
    int n1 = p->nodes_1d;
    s->Q = (p->dim_z == 0) ? 1 : (p->dim_z == 1 ? n1 : n1 * n1);
    int P = s->P, Q = s->Q;

    /* quadrature nodes and weights for the uniform density on [-1,1]^d_z */
    double *gx = (double *)malloc(sizeof(double) * (size_t)n1);
    double *gw = (double *)malloc(sizeof(double) * (size_t)n1);
    orc_gauss_legendre(n1, gx, gw);
    s->z = (double *)calloc((size_t)Q * 2, sizeof(double));
    s->w = (double *)calloc((size_t)Q, sizeof(double));
    for (int q = 0; q < Q; ++q) {
        if (p->dim_z == 0) { s->w[q] = 1.0; continue; }
        int q1 = q % n1, q2 = q / n1;
        s->z[q * 2 + 0] = gx[q1];
        s->w[q] = 0.5 * gw[q1];
        if (p->dim_z == 2) {
            s->z[q * 2 + 1] = gx[q2];
            s->w[q] *= 0.5 * gw[q2];
        }
    }
    free(gx); free(gw);

    s->psi = (double *)calloc((size_t)Q * P, sizeof(double));
    for (int q = 0; q < Q; ++q)
        for (int h = 0; h < P; ++h)
            s->psi[q * P + h] = basis_eval(p->dim_z, h, &s->z[q * 2]);

    /* uncertain inputs at the nodes */
    double hvf_eV_m = s->hbar * V_F / Q_E;
    s->eps0 = (double *)calloc((size_t)Q, sizeof(double));
    s->width = (double *)calloc((size_t)Q, sizeof(double));
    s->field = (double *)calloc((size_t)Q, sizeof(double));
    for (int q = 0; q < Q; ++q) {
        double zg = (p->gap_dim >= 0) ? z_coord(s, q, p->gap_dim) : 0.0;
        double zf = (p->field_dim >= 0) ? z_coord(s, q, p->field_dim) : 0.0;
        if (p->gap_mode == 0) {
            /* Reading: the band gap is the full gap 2 eps0 of the symmetric
             * dispersion eps = hbar v_F sqrt(k^2 + (pi/W)^2) (Sec. 2). */
            double gap = p->gap0 * (1.0 + p->gap_rel * zg);
            if (!(gap > 0)) { orc_destroy(s); return NULL; }
            s->eps0[q] = 0.5 * gap;
            s->width[q] = PI_D * hvf_eV_m / s->eps0[q];
        } else {
            double W = p->gap0 * 1e-9 * (1.0 + p->gap_rel * zg);
            if (!(W > 0)) { orc_destroy(s); return NULL; }
            s->width[q] = W;
            s->eps0[q] = PI_D * hvf_eV_m / W;
        }
        s->field[q] = p->field0 * (1.0 + p->field_rel * zf);
    }

    /* Galerkin field coefficients  E_h = int E(z) Psi_h(z) p(z) dz  (Sec. 4.1,
     * electric forcing), by the same quadrature.  E is linear in z and Psi_h
     * a polynomial of degree <= M, so the Gauss rule is exact for the
     * integrand: a sum that lies within its own rounding bound
     * (4 Q eps sum_q |w_q E_q Psi_h(z_q)|) is the integral's exact zero. */
    s->Ehat = (double *)calloc((size_t)P, sizeof(double));
    for (int h = 0; h < P; ++h) {
        double acc = 0.0, mag = 0.0;
        for (int q = 0; q < Q; ++q) {
            acc += s->w[q] * s->field[q] * s->psi[q * P + h];
            mag += fabs(s->w[q] * s->field[q] * s->psi[q * P + h]);
        }
        s->Ehat[h] = fabs(acc) <= 4.0 * Q * DBL_EPSILON * mag ? 0.0 : acc;
    }

    /* Scattering-rate prefactors, Appendix closed forms, energies in eV.
     * Reading: optical prefactor 2/(2 pi)^2 (the printed 2/(2 pi^2) is a typo;
     * the Appendix closed form is normative); the K-phonon rate uses omega_K. */
    double e = Q_E, hb = s->hbar;
    double kT_J = K_B * p->temp_K;
    double Dac = D_AC_EV * e;
    double DO = D_O_EV_PER_M * e, DK = D_K_EV_PER_M * e;
    double wO = HW_O_EV * e / hb, wK = HW_K_EV * e / hb;
    /* Gamma_ac = D_ac^2 k_B T eps / (4 hbar^3 v_F^2 sigma v_p^2); eps in J = eps_eV e */
    s->C_ac = Dac * Dac * kT_J / (4.0 * hb * hb * hb * V_F * V_F * SIGMA_M * V_P * V_P) * e;
    /* Gamma_O(-/+) = D_O^2/(hbar^2 v_F^2 sigma omega_O) (n+1 | n) (eps -/+ hbar w) */
    s->C_O = DO * DO / (hb * hb * V_F * V_F * SIGMA_M * wO) * e;
    s->C_K = DK * DK / (hb * hb * V_F * V_F * SIGMA_M * wK) * e;
    s->n_O = 1.0 / (exp(HW_O_EV / s->kT_eV) - 1.0);
    s->n_K = 1.0 / (exp(HW_K_EV / s->kT_eV) - 1.0);
    s->hw_O = HW_O_EV;
    s->hw_K = HW_K_EV;
    /* Gamma_edg = (hbar v_F)^-2 N_i V0^2/(2 pi hbar W) eps int exp(-2 a^2 |k|^2 (cos t' - cos t)^2) dt' */
    double V0 = V0_EV_M2 * e;
    double hvf_J_m = hb * V_F;
    s->C_edge = (double *)calloc((size_t)Q, sizeof(double));
    for (int q = 0; q < Q; ++q)
        s->C_edge[q] = N_I * V0 * V0 / (2.0 * PI_D * hb * s->width[q] * hvf_J_m * hvf_J_m) * e;
    /* 2 a^2 |k|^2 with |k| = kappa/(hbar v_F), kappa in eV */
    s->edge_kappa_coef = 2.0 * A_EDGE * A_EDGE / (hvf_eV_m * hvf_eV_m);

    s->dk = 2.0 * p->lk_eV / p->nk;

    orc_gauss_legendre(10, s->gl10_x, s->gl10_w);
    build_cdf_tables(s);
    s->density = (double *)calloc((size_t)Q, sizeof(double));
    for (int q = 0; q < Q; ++q) s->density[q] = density_m2(s, q);

    size_t N = (size_t)p->n_particles;
    s->kx = (double *)calloc((size_t)P * N, sizeof(double));
    s->ky = (double *)calloc((size_t)P * N, sizeof(double));
    s->H = (uint32_t *)calloc((size_t)Q * p->nk * p->nk, sizeof(uint32_t));
    s->Hmax = (uint32_t *)calloc((size_t)Q, sizeof(uint32_t));
    s->cap = (uint32_t *)calloc((size_t)Q, sizeof(uint32_t));
    s->excess = (uint32_t *)calloc((size_t)Q, sizeof(uint32_t));
    s->threads = 1;
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    if (s->cdf_x) for (int q = 0; q < s->Q; ++q) { free(s->cdf_x[q]); free(s->cdf_lo[q]); free(s->cdf_hi[q]); }
    free(s->cdf_x); free(s->cdf_lo); free(s->cdf_hi); free(s->cdf_np);
    free(s->z); free(s->w); free(s->psi); free(s->eps0); free(s->width); free(s->field);
    free(s->Ehat); free(s->C_edge); free(s->density);
    free(s->kx); free(s->ky); free(s->H); free(s->Hmax); free(s->cap); free(s->excess);
    free(s);
}

/* ------------------------------------------------------------------------ */
/* Dispersion, velocity and scattering rates at one node.                   */
/* ------------------------------------------------------------------------ */
/* eps(k) = hbar v_F sqrt(k_x^2 + k_y^2 + (pi/W)^2)   (Sec. 2) */
static double energy(double kx, double ky, double eps0)
{
    return sqrt(kx * kx + ky * ky + eps0 * eps0);
}

/* edge angular integral  I = int_0^{2pi} exp(-kap (cos t' - c)^2) dt'  by the
 * trapezoid rule (Appendix).  Reading: 32 uniform points on [0, 2 pi). */
double orc_edge_integral(double kap, double c)
{
    double acc = 0.0;
    for (int j = 0; j < ORC_NTHETA; ++j) {
        double d = cos(2.0 * PI_D * j / ORC_NTHETA) - c;
        acc += exp(-kap * d * d);
    }
    return acc * (2.0 * PI_D / ORC_NTHETA);
}

/* The six physical rates in the order of the mechanism vector (Sec. 3 eq.
 * lambda): AC, OP-, OP+, K-, K+, edge.  Appendix closed forms; each one
 * multiplied by its test scale. */
void orc_rates(const orc_sim *s, int q, double kx, double ky, double out[6])
{
    const double *sc = s->p.rate_scale;
    double e0 = s->eps0[q];
    double k2 = kx * kx + ky * ky;
    double eps = energy(kx, ky, e0);
    double on = (eps - e0 >= 0.0) ? 1.0 : 0.0;
    out[0] = sc[0] * s->C_ac * eps * on;
    double eOm = eps - s->hw_O, eOp = eps + s->hw_O;
    double eKm = eps - s->hw_K, eKp = eps + s->hw_K;
    out[1] = (eOm - e0 >= 0.0) ? sc[1] * s->C_O * (s->n_O + 1.0) * eOm : 0.0;
    out[2] = (eOp - e0 >= 0.0) ? sc[2] * s->C_O * s->n_O * eOp : 0.0;
    out[3] = (eKm - e0 >= 0.0) ? sc[3] * s->C_K * (s->n_K + 1.0) * eKm : 0.0;
    out[4] = (eKp - e0 >= 0.0) ? sc[4] * s->C_K * s->n_K * eKp : 0.0;
    double kabs = sqrt(k2);
    double c = (kabs > 0.0) ? kx / kabs : 1.0;   /* Reading: |k| = 0 -> theta_in = 0 */
    double kap = s->edge_kappa_coef * k2;
    out[5] = sc[5] * s->C_edge[q] * eps * orc_edge_integral(kap, c) * on;
}

/* ------------------------------------------------------------------------ */
/* Angle samplers (deterministic maps from uniforms).                        */
/* Reading: AC angle with density (1 + cos t)/(2 pi): twice the polar angle  */
/* of a uniform point of the unit disk centred at (1,0); K angle = AC angle  */
/* + pi (density 1 - cos t); OP angle = 2 pi u1.                             */
/* ------------------------------------------------------------------------ */
double orc_theta_ac(double u1, double u2)
{
    double r = sqrt(u1), phi = 2.0 * PI_D * u2;
    return 2.0 * atan2(r * sin(phi), 1.0 + r * cos(phi));
}

/* Rotate the incoming direction by theta and give the new vector length mag
 * (the h maps of Sec. 3).  Reading: for |k| = 0 the incoming direction is
 * (1, 0). */
static void rotate(double kx, double ky, double theta, double mag, double *ox, double *oy)
{
    double kabs = sqrt(kx * kx + ky * ky);
    double cin = (kabs > 0.0) ? kx / kabs : 1.0;
    double sin_ = (kabs > 0.0) ? ky / kabs : 0.0;
    double ct = cos(theta), st = sin(theta);
    *ox = mag * (ct * cin - st * sin_);
    *oy = mag * (st * cin + ct * sin_);
}

/* length of the final wave-vector after a phonon of energy dE is absorbed
 * (dE > 0) or emitted (dE < 0). */
static double final_magnitude(const orc_sim *s, double kx, double ky, double eps0, double dE)
{
    if (s->p.final_state == 1) {
        /* paper-literal:  |k| +/- omega/v_F  */
        return sqrt(kx * kx + ky * ky) + dE;
    }
    /* Reading (default): energy-conserving final state on the gapped band,
     * eps' = eps + dE, |kappa'| = sqrt(eps'^2 - eps0^2). */
    double e1 = energy(kx, ky, eps0) + dE;
    return sqrt((e1 - eps0) * (e1 + eps0));
}

/* ------------------------------------------------------------------------ */
/* Histogram and Pauli lookup.                                               */
/* ------------------------------------------------------------------------ */
/* cell index of (x, y) on [-L_k, L_k]^2 split in nk x nk cells (Sec. 3);
 * -1 if outside (zero boundary condition). */
long orc_cell(const orc_sim *s, double x, double y)
{
    double L = s->p.lk_eV;
    double fr = floor((x + L) / s->dk), fl = floor((y + L) / s->dk);
    if (!(fr >= 0.0 && fr < s->p.nk && fl >= 0.0 && fl < s->p.nk)) return -1;
    return (long)fr * s->p.nk + (long)fl;
}

/* f^n_{N,rl}(z_q) = N_rl / max N_rl at the cell of the candidate, on the grid
 * moved with the drift of this step (Sec. 3, Lagrangian grid).
 * Reading: the histogram counts k^n on the fixed grid; after the drift by
 * -D the grid moved by -D holds the same particles, so the candidate k' is
 * looked up at cell(k' + D) with D = v_F E(z_q) dt x^.  Outside the grid
 * f = 0. */
static double pauli_f(const orc_sim *s, int q, double kx, double ky, double dt)
{
    if (s->Hmax[q] == 0) return 0.0;
    double D = V_F * s->field[q] * dt;
    long c = orc_cell(s, kx + D, ky);
    if (c < 0) return 0.0;
    return (double)s->H[(size_t)q * s->p.nk * s->p.nk + c] / (double)s->Hmax[q];
}

/* ------------------------------------------------------------------------ */
/* gPC evaluation and projection.                                            */
/* ------------------------------------------------------------------------ */
static void evaluate(const orc_sim *s, const double *chx, const double *chy,
                     double *nx, double *ny)
{
    int P = s->P;
    for (int q = 0; q < s->Q; ++q) {
        double ax = 0.0, ay = 0.0;
        for (int h = 0; h < P; ++h) {
            ax += chx[h] * s->psi[q * P + h];
            ay += chy[h] * s->psi[q * P + h];
        }
        nx[q] = ax; ny[q] = ay;
    }
}

/* k_h = int k(z) Psi_h(z) p(z) dz  by the nodal quadrature (Sec. 4.1,
 * eq. update_sG; Reading: the collisional integrals eq. M1, M2 use the same
 * Gauss quadrature). */
static void project(const orc_sim *s, const double *nx, const double *ny,
                    double *chx, double *chy)
{
    int P = s->P;
    for (int h = 0; h < P; ++h) {
        double ax = 0.0, ay = 0.0;
        for (int q = 0; q < s->Q; ++q) {
            ax += s->w[q] * s->psi[q * P + h] * nx[q];
            ay += s->w[q] * s->psi[q * P + h] * ny[q];
        }
        chx[h] = ax; chy[h] = ay;
    }
}

/* ------------------------------------------------------------------------ */
/* Collision step of one particle (Algorithm 2; Algorithm 1 when Q = 1).     */
/* Input: the coefficients after the drift.  Output in place.                */
/* ------------------------------------------------------------------------ */
void orc_collide_particle(const orc_sim *s, long i, uint32_t step, double dt,
                          double *chx, double *chy, orc_counters *cnt)
{
    int Q = s->Q;
    double nx[ORC_QMAX], ny[ORC_QMAX], newx[ORC_QMAX], newy[ORC_QMAX];
    double rates[ORC_QMAX][6], S[ORC_QMAX];
    double tc = 0.0;
    uint32_t c = 0;
    for (;;) {
        evaluate(s, chx, chy, nx, ny);
        /* Gamma~ = (1 + alpha) max_q sum_nu Gamma^nu(z_q)  (eq. gamma_tot,
         * eq. deltat; Reading: the max over z is taken over the nodes). */
        double Smax = 0.0;
        for (int q = 0; q < Q; ++q) {
            orc_rates(s, q, nx[q], ny[q], rates[q]);
            S[q] = 0.0;
            for (int m = 0; m < 6; ++m) S[q] += rates[q][m];
            if (S[q] > Smax) Smax = S[q];
        }
        double G = (1.0 + s->p.alpha) * Smax;
        uint32_t r[4];
        draw(s, (uint32_t)i, step, c, PUR_XI, r);
        double xi = orc_u52(r[0], r[1]);
        double dtc = -log(xi) / G;          /* eq. dt with the node maximum */
        /* Reading: the free-flight time is drawn afresh after every
         * collision, at the current state. */
        if (!(tc + dtc < dt)) break;

        draw(s, (uint32_t)i, step, c, PUR_SEL, r);
        double su = orc_u52(r[0], r[1]);    /* s_i: mechanism selection */
        double eta = orc_u52(r[2], r[3]);   /* eta_i: Pauli acceptance  */
        draw(s, (uint32_t)i, step, c, PUR_ANG, r);
        double u1 = orc_u52(r[0], r[1]), u2 = orc_u52(r[2], r[3]);
        double th_ac = orc_theta_ac(u1, u2);
        double th_k = th_ac + PI_D;
        double th_op = 2.0 * PI_D * u1;
        cnt->collisions += 1;

        for (int q = 0; q < Q; ++q) {
            /* mechanism vector Lambda (eq. lambda) with the node's
             * self-scattering Gamma~ - S_q.  Reading: G^l normalised by
             * Gamma~, intervals half-open. */
            double lam[7];
            for (int m = 0; m < 6; ++m) lam[m] = rates[q][m];
            lam[6] = G - S[q];
            int ell = 7;
            double cum = 0.0;
            for (int m = 0; m < 6; ++m) {
                cum += lam[m];
                if (su < cum / G) { ell = m + 1; break; }
            }
            double kx = nx[q], ky = ny[q], e0 = s->eps0[q];
            double px = kx, py = ky;  /* candidate k' (eq. update) */
            int exhausted = 0;
            switch (ell) {
            case 1: rotate(kx, ky, th_ac, sqrt(kx * kx + ky * ky), &px, &py); break;
            case 2: rotate(kx, ky, th_op, final_magnitude(s, kx, ky, e0, -s->hw_O), &px, &py); break;
            case 3: rotate(kx, ky, th_op, final_magnitude(s, kx, ky, e0, +s->hw_O), &px, &py); break;
            case 4: rotate(kx, ky, th_k, final_magnitude(s, kx, ky, e0, -s->hw_K), &px, &py); break;
            case 5: rotate(kx, ky, th_k, final_magnitude(s, kx, ky, e0, +s->hw_K), &px, &py); break;
            case 6: {
                /* Reading: absolute final angle t' with density
                 * exp(-2 a^2 |k|^2 (cos t_in - cos t')^2) (eq. transport_el_edg),
                 * by rejection from shared uniform proposals. */
                double kabs = sqrt(kx * kx + ky * ky);
                double cin = (kabs > 0.0) ? kx / kabs : 1.0;
                double kap = s->edge_kappa_coef * (kx * kx + ky * ky);
                exhausted = 1;
                for (uint32_t j = 0; j < ORC_EDGE_TRIES; ++j) {
                    uint32_t rr[4];
                    draw(s, (uint32_t)i, step, c, PUR_EDGE0 + j, rr);
                    double tp = 2.0 * PI_D * orc_u52(rr[0], rr[1]);
                    double v = orc_u52(rr[2], rr[3]);
                    double d = cos(tp) - cin;
                    if (v < exp(-kap * d * d)) {
                        px = kabs * cos(tp); py = kabs * sin(tp);
                        exhausted = 0;
                        break;
                    }
                }
                if (exhausted) { px = kx; py = ky; cnt->edge_exhausted += 1; }
                break;
            }
            default: break;  /* self-scattering: h_7(k) = k */
            }
            if (ell == 7 || exhausted) {
                newx[q] = kx; newy[q] = ky;
                continue;
            }
            cnt->events += 1;
            /* Pauli acceptance against the previous-step distribution
             * (eq. Pauli / Pauli_gPC). */
            double f = s->p.pauli ? pauli_f(s, q, px, py, s->p.splitting ? 0.5 * dt : dt) : 0.0;
            if (f < eta) { newx[q] = px; newy[q] = py; }
            else { newx[q] = kx; newy[q] = ky; cnt->pauli_rejected += 1; }
        }
        project(s, newx, newy, chx, chy);
        tc += dtc;
        c += 1;
        if (c >= (uint32_t)s->p.c_max) { cnt->cmax_hits += 1; break; }
    }
}

/* ------------------------------------------------------------------------ */
/* Histogram, moments.                                                       */
/* ------------------------------------------------------------------------ */
static void rebuild_histogram(orc_sim *s)
{
    int Q = s->Q, P = s->P;
    size_t N = (size_t)s->p.n_particles, cells = (size_t)s->p.nk * s->p.nk;
    memset(s->H, 0, sizeof(uint32_t) * cells * Q);
    double ch_x[ORC_PMAX], ch_y[ORC_PMAX], nx[ORC_QMAX], ny[ORC_QMAX];
    for (size_t i = 0; i < N; ++i) {
        for (int h = 0; h < P; ++h) { ch_x[h] = s->kx[h * N + i]; ch_y[h] = s->ky[h * N + i]; }
        evaluate(s, ch_x, ch_y, nx, ny);
        for (int q = 0; q < Q; ++q) {
            long c = orc_cell(s, nx[q], ny[q]);
            if (c < 0) { s->counters.out_of_grid += 1; continue; }
            s->H[q * cells + c] += 1;
        }
    }
    for (int q = 0; q < Q; ++q) {
        uint32_t m = 0;
        for (size_t c = 0; c < cells; ++c) if (s->H[q * cells + c] > m) m = s->H[q * cells + c];
        s->Hmax[q] = m;
    }
    /* Pauli violation (Sec. 5 Test 1): particles above the maximum occupation
     * number of a cell, summed over the cells of each node */
    for (int q = 0; q < Q; ++q) {
        uint32_t ex = 0;
        for (size_t c = 0; c < cells; ++c)
            if (s->H[q * cells + c] > s->cap[q]) ex += s->H[q * cells + c] - s->cap[q];
        s->excess[q] = ex;
    }
}

/* the maximum occupation number per node: the largest cell count of the
 * current histogram (the initial datum, or a state set from outside) */
static void take_cap(orc_sim *s)
{
    for (int q = 0; q < s->Q; ++q) { s->cap[q] = s->Hmax[q]; s->excess[q] = 0; }
}

/* per node: V_x, V_y (m/s), mean energy (eV)  (Sec. 3 eq. Vx, eq. en; Sec. 4.2) */
void orc_moments(const orc_sim *s, double *out)
{
    int Q = s->Q, P = s->P;
    size_t N = (size_t)s->p.n_particles;
    double ch_x[ORC_PMAX], ch_y[ORC_PMAX], nx[ORC_QMAX], ny[ORC_QMAX];
    for (int q = 0; q < Q; ++q) { out[q * 3 + 0] = 0; out[q * 3 + 1] = 0; out[q * 3 + 2] = 0; }
    for (size_t i = 0; i < N; ++i) {
        for (int h = 0; h < P; ++h) { ch_x[h] = s->kx[h * N + i]; ch_y[h] = s->ky[h * N + i]; }
        evaluate(s, ch_x, ch_y, nx, ny);
        for (int q = 0; q < Q; ++q) {
            double eps = energy(nx[q], ny[q], s->eps0[q]);
            /* v = grad_k eps / hbar = v_F kappa / eps  (Sec. 2) */
            out[q * 3 + 0] += V_F * nx[q] / eps;
            out[q * 3 + 1] += V_F * ny[q] / eps;
            out[q * 3 + 2] += eps;
        }
    }
    for (int q = 0; q < Q; ++q) for (int k = 0; k < 3; ++k) out[q * 3 + k] /= (double)N;
}

/* ------------------------------------------------------------------------ */
/* Initial condition: Fermi-Dirac at every node (Sec. 4 uncertain IC).       */
/* Reading: one energy uniform and one angle uniform per particle, shared    */
/* by all nodes (the quantile map is smooth in z), then the nodal quadrature */
/* projection onto the gPC modes.                                            */
/* ------------------------------------------------------------------------ */
static void init_one(const orc_sim *s, long i, double *chx, double *chy)
{
    double nx[ORC_QMAX], ny[ORC_QMAX];
    uint32_t r[4];
    draw(s, (uint32_t)i, 0xFFFFFFFFu, 0, PUR_INIT, r);
    uint64_t m = u52_int(r[0], r[1]);
    double theta = 2.0 * PI_D * orc_u52(r[2], r[3]);
    for (int q = 0; q < s->Q; ++q) {
        double eps = fd_inverse_cdf_m(s, q, m);
        double e0 = s->eps0[q];
        double kabs = sqrt((eps - e0) * (eps + e0));
        nx[q] = kabs * cos(theta);
        ny[q] = kabs * sin(theta);
    }
    project(s, nx, ny, chx, chy);
}

/* initial coefficients of the listed particles: out[count][P] */
void orc_init_particles(const orc_sim *s, const long *idx, long count, double *kx, double *ky)
{
    for (long t = 0; t < count; ++t) init_one(s, idx[t], kx + t * s->P, ky + t * s->P);
}

void orc_init(orc_sim *s)
{
    int P = s->P;
    size_t N = (size_t)s->p.n_particles;
    double chx[ORC_PMAX], chy[ORC_PMAX];
    for (size_t i = 0; i < N; ++i) {
        init_one(s, (long)i, chx, chy);
        for (int h = 0; h < P; ++h) { s->kx[h * N + i] = chx[h]; s->ky[h * N + i] = chy[h]; }
    }
    s->step = 0;
    memset(&s->counters, 0, sizeof(s->counters));
    rebuild_histogram(s);
    take_cap(s);
}

/* One or more time steps: drift (Sec. 4.1 sG electric forcing), collisions
 * (Algorithm 2) against the histogram of the previous step, then the new
 * histogram and the moments at t^{n+1}.  moments_out: [n_steps][Q][3]. */
void orc_run(orc_sim *s, double dt, int n_steps, double *moments_out, uint32_t *excess_out)
{
    int P = s->P, Q = s->Q;
    size_t N = (size_t)s->p.n_particles;
    for (int n = 0; n < n_steps; ++n) {
        uint32_t step = (uint32_t)s->step;
        double drift[ORC_PMAX];
        for (int h = 0; h < P; ++h) drift[h] = V_F * dt * s->Ehat[h];
        orc_counters tot;
        memset(&tot, 0, sizeof(tot));
        long long c_coll = 0, c_ev = 0, c_rej = 0, c_exh = 0, c_cmax = 0;
#pragma omp parallel for schedule(static) num_threads(s->threads) reduction(+:c_coll,c_ev,c_rej,c_exh,c_cmax)
        for (long i = 0; i < (long)N; ++i) {
            double chx[ORC_PMAX], chy[ORC_PMAX];
            orc_counters loc;
            memset(&loc, 0, sizeof(loc));
            for (int h = 0; h < P; ++h) {
                /* k_h -= (e/hbar) dt E_h, in kappa units (dt/2 with Strang) */
                chx[h] = s->kx[h * N + i] - (s->p.splitting ? 0.5 * drift[h] : drift[h]);
                chy[h] = s->ky[h * N + i];
            }
            orc_collide_particle(s, i, step, dt, chx, chy, &loc);
            if (s->p.splitting)   /* the second half of the drift */
                for (int h = 0; h < P; ++h) chx[h] -= 0.5 * drift[h];
            for (int h = 0; h < P; ++h) { s->kx[h * N + i] = chx[h]; s->ky[h * N + i] = chy[h]; }
            c_coll += loc.collisions; c_ev += loc.events; c_rej += loc.pauli_rejected;
            c_exh += loc.edge_exhausted; c_cmax += loc.cmax_hits;
        }
        s->counters.collisions += c_coll; s->counters.events += c_ev;
        s->counters.pauli_rejected += c_rej; s->counters.edge_exhausted += c_exh;
        s->counters.cmax_hits += c_cmax;
        rebuild_histogram(s);
        s->step += 1;
        if (moments_out) orc_moments(s, moments_out + (size_t)n * Q * 3);
        if (excess_out) memcpy(excess_out + (size_t)n * Q, s->excess, sizeof(uint32_t) * Q);
    }
}

/* Energy distribution per node and its gPC modes:
 *   F_q(b) = #{i : eps(k_i(z_q)) in bin b} / (N * bin width),
 *   f_h(b) = sum_q w_q Psi_h(z_q) F_q(b)
 * (reconstruction of the distribution from the particles, Sec. 4.1 eq. f_gPC,
 * binned in energy). */
void orc_reconstruct_f(const orc_sim *s, int nbins, double emin, double emax,
                       double *nodes_out, double *modes_out)
{
    int Q = s->Q, P = s->P;
    size_t N = (size_t)s->p.n_particles;
    double width = (emax - emin) / nbins;
    memset(nodes_out, 0, sizeof(double) * (size_t)Q * nbins);
    double chx[ORC_PMAX], chy[ORC_PMAX], nx[ORC_QMAX], ny[ORC_QMAX];
    for (size_t i = 0; i < N; ++i) {
        for (int h = 0; h < P; ++h) { chx[h] = s->kx[h * N + i]; chy[h] = s->ky[h * N + i]; }
        evaluate(s, chx, chy, nx, ny);
        for (int q = 0; q < Q; ++q) {
            double eps = energy(nx[q], ny[q], s->eps0[q]);
            double fb = floor((eps - emin) / width);
            if (fb >= 0 && fb < nbins) nodes_out[q * nbins + (long)fb] += 1.0;
        }
    }
    for (int q = 0; q < Q; ++q)
        for (int b = 0; b < nbins; ++b) nodes_out[q * nbins + b] /= ((double)N * width);
    for (int h = 0; h < P; ++h)
        for (int b = 0; b < nbins; ++b) {
            double acc = 0.0;
            for (int q = 0; q < Q; ++q) acc += s->w[q] * s->psi[q * P + h] * nodes_out[q * nbins + b];
            modes_out[h * nbins + b] = acc;
        }
}

/* Energy distribution of the particles reconstructed at an arbitrary z:
 * k_i^M(z) = sum_h k_h Psi_h(z) (eq. gPC), eps with eps0(z). */
void orc_reconstruct_f_at(const orc_sim *s, const double *z, int nbins, double emin,
                          double emax, double *out)
{
    int P = s->P;
    size_t N = (size_t)s->p.n_particles;
    double width = (emax - emin) / nbins;
    double psi[ORC_PMAX];
    for (int h = 0; h < P; ++h) psi[h] = basis_eval(s->p.dim_z, h, z);
    double zg = (s->p.gap_dim >= 0) ? z[s->p.gap_dim] : 0.0;
    double hvf_eV_m = s->hbar * V_F / Q_E;
    double e0;
    if (s->p.gap_mode == 0) e0 = 0.5 * s->p.gap0 * (1.0 + s->p.gap_rel * zg);
    else e0 = PI_D * hvf_eV_m / (s->p.gap0 * 1e-9 * (1.0 + s->p.gap_rel * zg));
    memset(out, 0, sizeof(double) * (size_t)nbins);
    for (size_t i = 0; i < N; ++i) {
        double ax = 0.0, ay = 0.0;
        for (int h = 0; h < P; ++h) { ax += s->kx[h * N + i] * psi[h]; ay += s->ky[h * N + i] * psi[h]; }
        double eps = energy(ax, ay, e0);
        double fb = floor((eps - emin) / width);
        if (fb >= 0 && fb < nbins) out[(long)fb] += 1.0;
    }
    for (int b = 0; b < nbins; ++b) out[b] /= ((double)N * width);
}

/* Dilogarithm Li2(w) for 0 <= w <= 1/2 by its power series sum w^k / k^2
 * (terms shrink at least as 2^-k). */
static double dilog_small(double w)
{
    double term = w, sum = 0.0;
    for (int k = 1; k < 200 && term > 1e-20 * fabs(sum + 1e-300); ++k) {
        sum += term / ((double)k * (double)k);
        term *= w;
    }
    return sum;
}

/* Li2(-x) for x >= 0: Landen's identity Li2(-x) = -Li2(x/(1+x)) - ln^2(1+x)/2
 * maps 0 <= x <= 1 onto the series range; the inversion formula
 * Li2(-x) = -pi^2/6 - ln^2(x)/2 - Li2(-1/x) takes x > 1 there. */
static double dilog_neg(double x)
{
    if (x <= 1.0) {
        double l = log1p(x);
        return -dilog_small(x / (1.0 + x)) - 0.5 * l * l;
    }
    double l = log(x);
    return -PI_D * PI_D / 6.0 - 0.5 * l * l - dilog_neg(1.0 / x);
}

/* Equilibrium density of a band with minimum e0 (Sec. 3 eq. den with the
 * Fermi-Dirac datum of Sec. 2), in closed form:
 *   int_e0^inf eps / (1 + exp((eps - mu)/kT)) d eps
 *     = kT e0 ln(1 + e^eta) - kT^2 Li2(-e^eta),   eta = (mu - e0)/kT,
 * (integrate by parts; the Fermi-Dirac integral of order 1), then
 *   n = (2/pi) (hbar v_F)^-2 times it. */
double orc_density_closed(double e0, double mu, double kT, double hbar)
{
    double eta = (mu - e0) / kT;
    double lg = eta > 30.0 ? eta + log1p(exp(-eta)) : log1p(exp(eta));
    double z = kT * e0 * lg - kT * kT * dilog_neg(exp(eta));
    double hvf = hbar * V_F / Q_E;
    return (2.0 / PI_D) * z / (hvf * hvf);
}

/* Moments of the particle expansion at points z (Sec. 4.2): every particle's
 * wave-vector evaluated at z, k_i(z) = sum_h k_h Psi_h(z), on the band of
 * that z; out[j] = (V_x, V_y, mean energy, J_x = -e n(z) V_x). */
void orc_moments_at(const orc_sim *s, int nz, const double *z, double *out)
{
    int P = s->P, dz = s->p.dim_z;
    size_t N = (size_t)s->p.n_particles;
    double hvf_eV_m = s->hbar * V_F / Q_E;
    for (int j = 0; j < nz; ++j) {
        double zz[2] = {0.0, 0.0}, psi[ORC_PMAX];
        for (int d = 0; d < dz; ++d) zz[d] = z[(size_t)j * dz + d];
        for (int h = 0; h < P; ++h) psi[h] = basis_eval(dz, h, zz);
        double zg = (s->p.gap_dim >= 0) ? zz[s->p.gap_dim] : 0.0;
        double e0;
        if (s->p.gap_mode == 0) e0 = 0.5 * s->p.gap0 * (1.0 + s->p.gap_rel * zg);
        else e0 = PI_D * hvf_eV_m / (s->p.gap0 * 1e-9 * (1.0 + s->p.gap_rel * zg));
        double vx = 0.0, vy = 0.0, en = 0.0;
        for (size_t i = 0; i < N; ++i) {
            double ax = 0.0, ay = 0.0;
            for (int h = 0; h < P; ++h) { ax += s->kx[h * N + i] * psi[h]; ay += s->ky[h * N + i] * psi[h]; }
            double eps = energy(ax, ay, e0);
            vx += V_F * ax / eps;
            vy += V_F * ay / eps;
            en += eps;
        }
        double n = orc_density_closed(e0, s->p.fermi_eV, s->kT0_eV, s->hbar);
        out[j * 4 + 0] = vx / (double)N;
        out[j * 4 + 1] = vy / (double)N;
        out[j * 4 + 2] = en / (double)N;
        out[j * 4 + 3] = -Q_E * n * out[j * 4 + 0];
    }
}

/* ------------------------------------------------------------------------ */
/* Accessors for the test wrapper.                                           */
/* ------------------------------------------------------------------------ */
int orc_P(const orc_sim *s) { return s->P; }
int orc_Q(const orc_sim *s) { return s->Q; }
long orc_step_count(const orc_sim *s) { return s->step; }
void orc_set_threads(orc_sim *s, int t) { s->threads = t > 0 ? t : 1; }

void orc_tables(const orc_sim *s, double *z, double *w, double *psi, double *ehat,
                double *eps0, double *width, double *field, double *density)
{
    int P = s->P, Q = s->Q;
    if (z) memcpy(z, s->z, sizeof(double) * (size_t)Q * 2);
    if (w) memcpy(w, s->w, sizeof(double) * (size_t)Q);
    if (psi) memcpy(psi, s->psi, sizeof(double) * (size_t)Q * P);
    if (ehat) memcpy(ehat, s->Ehat, sizeof(double) * (size_t)P);
    if (eps0) memcpy(eps0, s->eps0, sizeof(double) * (size_t)Q);
    if (width) memcpy(width, s->width, sizeof(double) * (size_t)Q);
    if (field) memcpy(field, s->field, sizeof(double) * (size_t)Q);
    if (density) memcpy(density, s->density, sizeof(double) * (size_t)Q);
}

void orc_get_state(const orc_sim *s, double *kx, double *ky)
{
    size_t n = (size_t)s->P * (size_t)s->p.n_particles;
    memcpy(kx, s->kx, sizeof(double) * n);
    memcpy(ky, s->ky, sizeof(double) * n);
}

/* set the coefficients and rebuild the histogram of that state */
void orc_set_state(orc_sim *s, const double *kx, const double *ky, long step)
{
    size_t n = (size_t)s->P * (size_t)s->p.n_particles;
    memcpy(s->kx, kx, sizeof(double) * n);
    memcpy(s->ky, ky, sizeof(double) * n);
    s->step = step;
    rebuild_histogram(s);
    take_cap(s);
}

void orc_get_histogram(const orc_sim *s, uint32_t *H, uint32_t *Hmax)
{
    size_t cells = (size_t)s->p.nk * s->p.nk;
    if (H) memcpy(H, s->H, sizeof(uint32_t) * cells * s->Q);
    if (Hmax) memcpy(Hmax, s->Hmax, sizeof(uint32_t) * s->Q);
}

/* replace the histogram used by the Pauli check (sampled full-size parity:
 * the step of one particle depends only on its state and on H^n) */
void orc_set_histogram(orc_sim *s, const uint32_t *H, const uint32_t *Hmax)
{
    size_t cells = (size_t)s->p.nk * s->p.nk;
    memcpy(s->H, H, sizeof(uint32_t) * cells * s->Q);
    memcpy(s->Hmax, Hmax, sizeof(uint32_t) * s->Q);
}

void orc_get_counters(const orc_sim *s, long long *out)
{
    out[0] = s->counters.collisions;
    out[1] = s->counters.events;
    out[2] = s->counters.pauli_rejected;
    out[3] = s->counters.edge_exhausted;
    out[4] = s->counters.cmax_hits;
    out[5] = s->counters.out_of_grid;
}

/* Step a list of particles given their coefficients at t^n (before the
 * drift), with the histogram currently held (orc_set_histogram). */
void orc_step_particles(const orc_sim *s, const long *idx, long count, uint32_t step,
                        double dt, double *kx, double *ky, long long *ncoll)
{
    int P = s->P;
    for (long t = 0; t < count; ++t) {
        double chx[ORC_PMAX], chy[ORC_PMAX];
        orc_counters loc;
        memset(&loc, 0, sizeof(loc));
        for (int h = 0; h < P; ++h) {
            double d = V_F * dt * s->Ehat[h];
            chx[h] = kx[t * P + h] - (s->p.splitting ? 0.5 * d : d);
            chy[h] = ky[t * P + h];
        }
        orc_collide_particle(s, idx[t], step, dt, chx, chy, &loc);
        if (s->p.splitting)
            for (int h = 0; h < P; ++h) chx[h] -= 0.5 * (V_F * dt * s->Ehat[h]);
        for (int h = 0; h < P; ++h) { kx[t * P + h] = chx[h]; ky[t * P + h] = chy[h]; }
        if (ncoll) ncoll[t] = loc.collisions;
    }
}

/* rates and angle helpers exposed for the pins */
void orc_rates_at(const orc_sim *s, int q, const double *kx, const double *ky, long n, double *out)
{
    for (long t = 0; t < n; ++t) orc_rates(s, q, kx[t], ky[t], out + t * 6);
}

void orc_theta_ac_many(const double *u1, const double *u2, long n, double *out)
{
    for (long t = 0; t < n; ++t) out[t] = orc_theta_ac(u1[t], u2[t]);
}

void orc_fd_inverse_many(const orc_sim *s, int q, const uint32_t *whi, const uint32_t *wlo,
                         long n, double *out)
{
    for (long t = 0; t < n; ++t) out[t] = orc_fd_inverse_cdf(s, q, whi[t], wlo[t]);
}

void orc_philox_many(const uint32_t *ctr, const uint32_t *key, long n, uint32_t *out)
{
    for (long t = 0; t < n; ++t) orc_philox4x32_10(ctr + 4 * t, key + 2 * t, out + 4 * t);
}

/* one edge collision at one node for the sampler pin: the final absolute
 * angle for the given incoming vector, from the particle's shared proposals */
double orc_edge_angle(const orc_sim *s, long i, uint32_t step, uint32_t coll, double kx, double ky)
{
    double kabs = sqrt(kx * kx + ky * ky);
    double cin = (kabs > 0.0) ? kx / kabs : 1.0;
    double kap = s->edge_kappa_coef * (kx * kx + ky * ky);
    for (uint32_t j = 0; j < ORC_EDGE_TRIES; ++j) {
        uint32_t rr[4];
        draw(s, (uint32_t)i, step, coll, PUR_EDGE0 + j, rr);
        double tp = 2.0 * PI_D * orc_u52(rr[0], rr[1]);
        double v = orc_u52(rr[2], rr[3]);
        double d = cos(tp) - cin;
        if (v < exp(-kap * d * d)) return tp;
    }
    return NAN;
}

double orc_edge_kappa_coef(const orc_sim *s) { return s->edge_kappa_coef; }

/* Pauli occupation looked up for a candidate at node q (for the pins). */
double orc_pauli_lookup(const orc_sim *s, int q, double kx, double ky, double dt)
{
    return pauli_f(s, q, kx, ky, dt);
}
