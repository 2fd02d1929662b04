// Internal types of the sG-PM library: host set-up tables and the argument
// blocks of the gfx950 kernels.  Not part of the C-ABI.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/sgpm.h"

namespace sgpm {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kQueueCap = 2 * kBlock;  // LDS candidate queue
constexpr int kMaxP = 32;            // largest gPC basis the kernels accept
constexpr int kMaxQ = 128;           // largest node count
constexpr int kEdgePts = 32;         // trapezoid points of the edge integral
constexpr int kEdgeTries = 64;       // edge-angle proposals per collision
constexpr int kNumBatches = 32;      // batch-means batches of the moment record
constexpr int kLdsHistBytes = 56 * 1024;  // LDS budget of the histogram window

// Host FP64 set-up of one instance (Sec. 4.1 tables, Appendix rate constants).
struct HostTables {
    int dim_z = 0, P = 1, Q = 1, nodes_1d = 1;
    std::vector<double> z;      // [Q][2]
    std::vector<double> w;      // [Q]
    std::vector<double> psi;    // [Q][P]
    std::vector<double> wpsi;   // [Q][P]  w_q Psi_h(z_q)
    std::vector<double> ehat;   // [P]     int E(z) Psi_h p dz  (V/m)
    std::vector<double> eps0;   // [Q] band minimum, eV
    std::vector<double> width;  // [Q] ribbon width, m
    std::vector<double> field;  // [Q] V/m
    std::vector<double> density;// [Q] electrons per m^2
    std::vector<double> cedge;  // [Q] edge prefactor, 1/(s eV), per unit angular integral
    double c_ac = 0, c_o = 0, c_k = 0;   // 1/(s eV)
    double n_o = 0, n_k = 0, hw_o = 0, hw_k = 0, kT = 0;
    double edge_kap = 0;        // 2 a^2 / (hbar v_F)^2 in 1/eV^2
    double v_f = 0;             // m/s
    double gl10_x[10], gl10_w[10];
    double edge_cos[kEdgePts / 2 + 1];   // cos(2 pi j / 32), j = 0..16
    // Fermi-Dirac CDF tables per node: panels of width cdf_h from eps0[q]
    int cdf_np = 0;             // panels per node (same count for every node)
    double cdf_h = 0;
    std::vector<double> cdf_lo; // [Q][np+1] cumulative from below (eV^2)
    std::vector<double> cdf_hi; // [Q][np+1] cumulative from above
};

// Builds the tables; returns an empty string or the reason of a rejection.
const char* build_tables(const sgpm_instance_desc& d, HostTables& t);
int num_modes(int dim_z, int degree);
double basis_at(int dim_z, int h, const double* z);
void eval_basis_all(int dim_z, int P, const double* z, double* out);

// Device table blob of one instance (arrays are offsets into the blob).
template <typename T>
struct DevTab {
    const T* psi;      // [Q][P]
    const T* wpsi;     // [Q][P]
    const T* eps0;     // [Q]
    const T* eps0sq;   // [Q]
    const T* cedge;    // [Q] edge prefactor times its rate scale
    const T* vfield;   // [Q] v_F E(z_q), eV/s
    const T* edge_cos; // [17]
};

template <typename T>
struct StepArgs {
    T* kx;
    T* ky;
    int64_t n;
    int P, Q;
    DevTab<T> tab;
    T drift[kMaxP];      // v_F dt E_h, eV
    uint32_t drift_mask; // modes with a nonzero drift (h < 32)
    T dt;
    T c_ac, c_om, c_op, c_km, c_kp;   // rate coefficients incl. Bose factors and scales
    T hw_o, hw_k;
    T edge_kap;          // 2 a^2/(hbar v_F)^2
    T alpha1;            // 1 + alpha
    T v_f;               // m/s
    // rigorous upper bound of max_q sum_nu Gamma^nu as a function of eps_max
    T b_ac, b_om, b_op, b_km, b_kp, b_edge, b_thr_o, b_thr_k, b_margin;
    T lk, dk, inv_dk;
    int nk;
    int pauli, final_state, c_max;
    uint32_t seed_lo, seed_hi, instance, step;
    // histogram buffers: read H^n, accumulate H^{n+1}, clear the stale one
    const uint32_t* h_read;
    const uint32_t* hmax_read;
    uint32_t* h_acc;
    uint32_t* hmax_acc;
    uint32_t* h_clr;
    uint32_t* hmax_clr;
    int64_t clear_vec4;  // uint4 stores to clear the stale buffer
    int win, win_r0, win_l0, hwin_words;
    // moments
    double* partial;     // [nwg][Q][3]
    double* record;      // [NB][Q][3] of this time index
    uint32_t* done;
    int nb;
    unsigned long long* counters;  // [SGPM_N_COUNTERS]
    int64_t chunk;
    int nwg;
    int do_drift, do_collide;
};

struct InitArgs {
    double* kx64; double* ky64;   // one of the two pairs is used
    float* kx32; float* ky32;
    int64_t n;
    int P, Q;
    const double* wpsi;   // [Q][P]
    const double* eps0;   // [Q]
    const double* cdf_lo; // [Q][np+1]
    const double* cdf_hi;
    const double* gl;     // [20]: 10 nodes then 10 weights
    int cdf_np;
    double cdf_h, mu, kT;
    uint32_t seed_lo, seed_hi, instance;
};

struct EnergyHistArgs {
    const void* kx; const void* ky;
    int fp32;
    int64_t n;
    int P, Q;            // Q evaluation points
    const double* psi;   // [Q][P]
    const double* eps0;  // [Q]
    int nbins;
    double emin, width;
    unsigned long long* bins;  // [Q][nbins]
};

// Kernel launchers (sgpm_kernels.hip).  Return hipError_t as int.
int launch_step_f64(const StepArgs<double>& a, int pmax_bucket, void* stream);
int launch_step_f32(const StepArgs<float>& a, int pmax_bucket, void* stream);
int launch_init(const InitArgs& a, void* stream);
int launch_energy_hist(const EnergyHistArgs& a, void* stream);
int launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n,
                  void* stream);
size_t step_lds_bytes(int Q, int hwin_words);

}  // namespace sgpm
