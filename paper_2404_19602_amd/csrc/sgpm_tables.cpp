// Host FP64 set-up tables of one sG-PM instance: quadrature nodes and
// weights, the orthonormal Legendre basis, the Galerkin field coefficients
// (Sec. 4.1), the scattering-rate constants of the Appendix, the electron
// density and the Fermi-Dirac CDF tables of the initial datum.
#include <cfloat>
#include <cmath>
#include <cstring>

#include "sgpm_internal.h"

namespace sgpm {
namespace {

// SI 2019 exact constants.
constexpr double kE = 1.602176634e-19;
constexpr double kH = 6.62607015e-34;
constexpr double kKB = 1.380649e-23;
constexpr double kPi = 3.14159265358979323846;

// Table 1 (Sec. 5) in SI; energies of phonons in eV.
constexpr double kVF = 1.0e6;          // 1e8 cm/s
constexpr double kSigma = 7.6e-7;      // 7.6e-8 g/cm^2
constexpr double kHwO = 0.1646;        // eV
constexpr double kHwK = 0.124;         // eV
constexpr double kVp = 2.0e4;          // 2e6 cm/s
constexpr double kDac = 6.8;           // eV
constexpr double kDO = 1.0e11;         // 1e9 eV/cm in eV/m
constexpr double kDK = 3.5e10;         // 3.5e8 eV/cm in eV/m
constexpr double kNi = 1.0e6;          // 1e4 /cm in /m
constexpr double kV0 = 4.56e-18;       // 4.56e-14 eV cm^2 in eV m^2
constexpr double kA = 1.0e-10;         // 1e-8 cm in m

// Roots and weights of the n-point Gauss-Legendre rule: Newton iteration on
// P_n from the asymptotic root estimate, derivative from the recurrence.
void gauss_legendre(int n, double* x, double* w) {
    const int half = (n + 1) / 2;
    for (int k = 0; k < half; ++k) {
        double r = std::cos(kPi * (4.0 * k + 3.0) / (4.0 * n + 2.0));
        double d = 0.0;
        for (int it = 0; it < 64; ++it) {
            double pm = 1.0, p = r;            // P_0, P_1
            for (int j = 1; j < n; ++j) {
                double pn = ((2 * j + 1) * r * p - j * pm) / (j + 1);
                pm = p;
                p = pn;
            }
            if (n == 1) { p = r; pm = 1.0; }
            d = n * (pm - r * p) / (1.0 - r * r);   // P_n'(r)
            double step = p / d;
            r -= step;
            if (std::fabs(step) <= 4e-17) {
                // refresh the derivative at the accepted root
                pm = 1.0; p = r;
                for (int j = 1; j < n; ++j) {
                    double pn = ((2 * j + 1) * r * p - j * pm) / (j + 1);
                    pm = p;
                    p = pn;
                }
                if (n == 1) { p = r; pm = 1.0; }
                d = n * (pm - r * p) / (1.0 - r * r);
                break;
            }
        }
        double wk = 2.0 / ((1.0 - r * r) * d * d);
        x[n - 1 - k] = r;  w[n - 1 - k] = wk;
        x[k] = -r;         w[k] = wk;
    }
    if (n % 2 == 1) x[n / 2] = 0.0;
}

// Orthonormal Legendre polynomial of degree k at x (uniform density 1/2),
// by the normalised three-term recurrence.
double legendre_on(int k, double x) {
    double a = 1.0;                 // degree 0
    if (k == 0) return a;
    double b = std::sqrt(3.0) * x;  // degree 1
    for (int j = 1; j < k; ++j) {
        double c1 = std::sqrt((2.0 * j + 1.0) * (2.0 * j + 3.0)) / (j + 1.0);
        double c0 = (j / (j + 1.0)) * std::sqrt((2.0 * j + 3.0) / (2.0 * j - 1.0));
        double c = c1 * x * b - c0 * a;
        a = b;
        b = c;
    }
    return b;
}

void exponents(int dim_z, int h, int* e1, int* e2) {
    if (dim_z < 2) { *e1 = h; *e2 = 0; return; }
    int t = 0;
    while ((t + 1) * (t + 2) / 2 <= h) ++t;    // total degree of mode h
    int pos = h - t * (t + 1) / 2;               // position inside degree t
    *e1 = t - pos;
    *e2 = pos;
}

double fd_density(double e, double mu, double kT) {
    return e / (1.0 + std::exp((e - mu) / kT));
}

}  // namespace

int num_modes(int dim_z, int degree) {
    if (dim_z <= 0) return 1;
    if (dim_z == 1) return degree + 1;
    return (degree + 1) * (degree + 2) / 2;
}

double basis_at(int dim_z, int h, const double* z) {
    if (dim_z == 0) return 1.0;
    int e1, e2;
    exponents(dim_z, h, &e1, &e2);
    double v = legendre_on(e1, z[0]);
    if (dim_z == 2) v *= legendre_on(e2, z[1]);
    return v;
}

void eval_basis_all(int dim_z, int P, const double* z, double* out) {
    for (int h = 0; h < P; ++h) out[h] = basis_at(dim_z, h, z);
}

const char* build_tables(const sgpm_instance_desc& d, HostTables& t) {
    if (d.dim_z < 0 || d.dim_z > 2) return "dim_z must be 0, 1 or 2";
    if (d.degree < 0) return "degree must be >= 0";
    if (d.dim_z > 0 && d.nodes_1d < 1) return "nodes_1d must be >= 1";
    if (d.n_particles < 1) return "n_particles must be >= 1";
    if (d.n_particles > (int64_t)2000000000) return "n_particles above 2e9";
    if (!(d.temp_K > 0) || !std::isfinite(d.temp_K)) return "temp_K must be > 0";
    if (!(d.init_temp_K >= 0) || !std::isfinite(d.init_temp_K)) return "init_temp_K must be >= 0";
    if (d.nk < 2 || d.nk > 4096) return "nk must be in [2, 4096]";
    if (!(d.lk_eV > 0)) return "lk_eV must be > 0";
    if (!(d.alpha >= 0) || !std::isfinite(d.alpha)) return "alpha must be >= 0";
    if (d.gap_dim >= d.dim_z || d.gap_dim < -1) return "gap_dim out of range";
    if (d.field_dim >= d.dim_z || d.field_dim < -1) return "field_dim out of range";
    if (d.c_max < 1 || d.c_max > 255) return "c_max must be in [1, 255]";
    if (d.precision != SGPM_FP64 && d.precision != SGPM_FP32) return "unknown precision";
    if (d.pauli != 0 && d.pauli != 1) return "pauli must be 0 or 1";
    if (d.final_state != 0 && d.final_state != 1) return "final_state must be 0 or 1";
    if (d.splitting != 0 && d.splitting != 1) return "splitting must be 0 or 1";
    if (d.gap_mode != 0 && d.gap_mode != 1) return "gap_mode must be 0 or 1";
    if (d.max_steps < 0) return "max_steps must be >= 0";
    if (!std::isfinite(d.field0) || !std::isfinite(d.field_rel) || !std::isfinite(d.fermi_eV))
        return "non-finite field or Fermi level";
    for (int m = 0; m < 6; ++m)
        if (!(d.rate_scale[m] >= 0) || !std::isfinite(d.rate_scale[m]))
            return "rate_scale entries must be finite and >= 0";

    t.dim_z = d.dim_z;
    t.nodes_1d = d.dim_z == 0 ? 1 : d.nodes_1d;
    t.P = num_modes(d.dim_z, d.degree);
    t.Q = d.dim_z == 0 ? 1 : (d.dim_z == 1 ? t.nodes_1d : t.nodes_1d * t.nodes_1d);
    if (t.P > kMaxP) return "too many gPC modes (the kernels take P <= 32)";
    if (t.Q > kMaxQ) return "too many nodes (the kernels take Q <= 128)";
    // cell offsets of H^n and the overflow grid are 32-bit byte offsets
    if ((int64_t)t.Q * d.nk * d.nk >= ((int64_t)1 << 30)) return "Q nk^2 must be below 2^30";
    const int P = t.P, Q = t.Q, n1 = t.nodes_1d;

    std::vector<double> gx(n1), gw(n1);
    gauss_legendre(n1, gx.data(), gw.data());
    t.z.assign(2 * Q, 0.0);
    t.w.assign(Q, 1.0);
    for (int q = 0; q < Q; ++q) {
        if (d.dim_z == 0) break;
        int i1 = q % n1, i2 = q / n1;
        t.z[2 * q] = gx[i1];
        t.w[q] = 0.5 * gw[i1];
        if (d.dim_z == 2) {
            t.z[2 * q + 1] = gx[i2];
            t.w[q] *= 0.5 * gw[i2];
        }
    }
    t.psi.assign(Q * P, 0.0);
    t.wpsi.assign(Q * P, 0.0);
    for (int q = 0; q < Q; ++q)
        for (int h = 0; h < P; ++h) {
            t.psi[q * P + h] = basis_at(d.dim_z, h, &t.z[2 * q]);
            t.wpsi[q * P + h] = t.w[q] * t.psi[q * P + h];
        }

    const double hbar = kH / (2.0 * kPi);
    const double hvf_eVm = hbar * kVF / kE;      // hbar v_F in eV m
    t.v_f = kVF;
    t.kT = kKB * d.temp_K / kE;
    t.kT_init = kKB * (d.init_temp_K > 0 ? d.init_temp_K : d.temp_K) / kE;
    t.eps0.assign(Q, 0.0);
    t.width.assign(Q, 0.0);
    t.field.assign(Q, 0.0);
    for (int q = 0; q < Q; ++q) {
        double zg = d.gap_dim >= 0 ? t.z[2 * q + d.gap_dim] : 0.0;
        double zf = d.field_dim >= 0 ? t.z[2 * q + d.field_dim] : 0.0;
        double g = d.gap0 * (1.0 + d.gap_rel * zg);
        if (!(g > 0) || !std::isfinite(g)) return "band gap / width must be > 0 at every node";
        if (d.gap_mode == 0) {
            t.eps0[q] = 0.5 * g;                  // gap = 2 eps0
            t.width[q] = kPi * hvf_eVm / t.eps0[q];
        } else {
            t.width[q] = g * 1e-9;
            t.eps0[q] = kPi * hvf_eVm / t.width[q];
        }
        t.field[q] = d.field0 * (1.0 + d.field_rel * zf);
    }
    // Galerkin field coefficients (Sec. 4.1) by the Gauss rule, exact for the
    // polynomial integrand E(z) Psi_h(z): sums within their rounding bound are
    // the exact zeros of the modes E(z) does not reach, and the drift leaves
    // those modes untouched.
    t.ehat.assign(P, 0.0);
    for (int h = 0; h < P; ++h) {
        double s = 0.0, mag = 0.0;
        for (int q = 0; q < Q; ++q) {
            s += t.wpsi[q * P + h] * t.field[q];
            mag += std::fabs(t.wpsi[q * P + h] * t.field[q]);
        }
        t.ehat[h] = std::fabs(s) <= 4.0 * Q * DBL_EPSILON * mag ? 0.0 : s;
    }

    // Appendix closed forms; rate = c * energy[eV] * (occupation factors)
    const double kTJ = kKB * d.temp_K;
    const double dac = kDac * kE, dO = kDO * kE, dK = kDK * kE;
    const double wO = kHwO * kE / hbar, wK = kHwK * kE / hbar;
    t.c_ac = kE * dac * dac * kTJ / (4.0 * hbar * hbar * hbar * kVF * kVF * kSigma * kVp * kVp);
    t.c_o = kE * dO * dO / (hbar * hbar * kVF * kVF * kSigma * wO);
    t.c_k = kE * dK * dK / (hbar * hbar * kVF * kVF * kSigma * wK);
    t.hw_o = kHwO;
    t.hw_k = kHwK;
    t.n_o = 1.0 / std::expm1(kHwO / t.kT);
    t.n_k = 1.0 / std::expm1(kHwK / t.kT);
    const double hvfJ = hbar * kVF;
    const double v0 = kV0 * kE;
    t.cedge.assign(Q, 0.0);
    for (int q = 0; q < Q; ++q)
        t.cedge[q] = kE * kNi * v0 * v0 / (2.0 * kPi * hbar * t.width[q] * hvfJ * hvfJ);
    t.edge_kap = 2.0 * kA * kA / (hvf_eVm * hvf_eVm);
    for (int j = 0; j <= kEdgePts / 2; ++j) t.edge_cos[j] = std::cos(2.0 * kPi * j / kEdgePts);
    t.edge_cos[kEdgePts / 4] = 0.0;   // cos(pi/2): the exact value
    t.edge_cos[kEdgePts / 2] = -1.0;

    gauss_legendre(10, t.gl10_x, t.gl10_w);

    // Fermi-Dirac energy CDF per node (density eps f_FD on [eps0, inf)) at the
    // temperature of the initial datum: panels of kT/2 up to max(mu, eps0) +
    // 80 kT, 10-point Gauss per panel.
    double e0min = t.eps0[0], e0max = t.eps0[0];
    for (int q = 1; q < Q; ++q) {
        e0min = std::fmin(e0min, t.eps0[q]);
        e0max = std::fmax(e0max, t.eps0[q]);
    }
    t.cdf_h = 0.5 * t.kT_init;
    double top = std::fmax(d.fermi_eV, e0max) + 80.0 * t.kT_init;
    t.cdf_np = (int)std::ceil((top - e0min) / t.cdf_h);
    if (t.cdf_np < 4) t.cdf_np = 4;
    const int np = t.cdf_np;
    t.cdf_lo.assign((size_t)Q * (np + 1), 0.0);
    t.cdf_hi.assign((size_t)Q * (np + 1), 0.0);
    t.density.assign(Q, 0.0);
    std::vector<double> pan(np);
    for (int q = 0; q < Q; ++q) {
        for (int j = 0; j < np; ++j) {
            double a = t.eps0[q] + j * t.cdf_h, b = a + t.cdf_h;
            double c = 0.5 * (a + b), hw = 0.5 * (b - a), s = 0.0;
            for (int k = 0; k < 10; ++k)
                s += t.gl10_w[k] * fd_density(c + hw * t.gl10_x[k], d.fermi_eV, t.kT_init);
            pan[j] = s * hw;
        }
        double* lo = &t.cdf_lo[(size_t)q * (np + 1)];
        double* hi = &t.cdf_hi[(size_t)q * (np + 1)];
        lo[0] = 0.0;
        for (int j = 0; j < np; ++j) lo[j + 1] = lo[j] + pan[j];
        hi[np] = 0.0;
        for (int j = np - 1; j >= 0; --j) hi[j] = hi[j + 1] + pan[j];
        // n = g_s g_v/(2 pi)^2 int f dk = (2/pi) (hbar v_F)^-2 int eps f_FD d eps
        t.density[q] = (2.0 / kPi) * lo[np] / (hvf_eVm * hvf_eVm);
    }
    return "";
}

// Equilibrium density of a band with minimum eps0 (Sec. 3 eq. den with the
// Fermi-Dirac datum): n = (2/pi) (hbar v_F)^-2 int_eps0^inf eps f_FD d eps, by
// panels of kT/2 up to max(mu, eps0) + 80 kT with 10-point Gauss per panel.
double density_at(double eps0, double mu, double kT) {
    double gx[10], gw[10];
    gauss_legendre(10, gx, gw);
    const double h = 0.5 * kT, top = std::fmax(mu, eps0) + 80.0 * kT;
    const int np = (int)std::ceil((top - eps0) / h);
    double z = 0.0;
    for (int j = 0; j < np; ++j) {
        const double a = eps0 + j * h, c = a + 0.5 * h, hw = 0.5 * h;
        double s = 0.0;
        for (int k = 0; k < 10; ++k) s += gw[k] * fd_density(c + hw * gx[k], mu, kT);
        z += s * hw;
    }
    const double hvf_eVm = kH / (2.0 * kPi) * kVF / kE;
    return (2.0 / kPi) * z / (hvf_eVm * hvf_eVm);
}

}  // namespace sgpm
