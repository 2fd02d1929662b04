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
constexpr int kMaxP = 32;            // largest gPC basis the kernels accept
constexpr int kMaxQ = 128;           // largest node count
constexpr int kEdgePts = 32;         // trapezoid points of the edge integral
constexpr int kEdgeTries = 64;       // edge-angle proposals per collision
constexpr int kNumBatches = 32;      // batch-means batches of the moment record
constexpr int kLdsK1Bytes = 80 * 1024;   // default LDS budget of a stream workgroup

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
    double n_o = 0, n_k = 0, hw_o = 0, hw_k = 0;
    double kT = 0;              // lattice k_B T (eV): Bose factors, acoustic rate
    double kT_init = 0;         // k_B T (eV) of the Fermi-Dirac initial datum and density
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

// Per-instance constants of the step kernels, resident in device memory and
// staged into LDS by every workgroup (keeps them out of scalar registers).
template <typename T>
struct Consts {
    T c_ac, c_om, c_op, c_km, c_kp;   // rate coefficients incl. Bose factors and scales
    T hw_o, hw_k;
    T edge_kap;                       // 2 a^2 / (hbar v_F)^2, 1/eV^2
    T alpha1;                         // 1 + alpha
    T v_f;                            // m/s
    // upper bound of max_q sum_nu Gamma^nu as a function of an energy bound
    T b_ac, b_om, b_op, b_km, b_kp, b_edge, b_thr_o, b_thr_k, b_margin;
    T eps0max_sq;
    T lk, dk, inv_dk;
    int32_t nk, pauli, final_state, c_max;
    int32_t splitting;                // 1: Strang (half drift before and after the collisions)
    int32_t pad_;
};

// Device tables of one instance in one precision (all [Q][P] row-major).
template <typename T>
struct DevTab {
    const T* psi;      // [Q][P]
    const T* wpsi;     // [Q][P]   w_q Psi_h(z_q)
    const T* eps0;     // [Q]
    const T* eps0sq;   // [Q]
    const T* cedge;    // [Q] edge prefactor times its rate scale
    const T* vfield;   // [Q] v_F E(z_q)
    const T* edge_cos; // [17]
    const T* psimax;   // [P] max_q |Psi_h(z_q)|
    const Consts<T>* consts;
};

constexpr int kWaves1 = 16;           // most waves per workgroup of the stream kernel
constexpr int kBlock1 = 64 * kWaves1; // chunk quantum: a multiple of every stream block size

// Waves per stream workgroup for a precision, mode bucket and node bucket:
// sixteen (1024 threads, four waves per SIMD, so at most 128 VGPRs) where the
// kernel fits that with at most a few spilled registers, else eight.  The
// generic path for more than 12 nodes keeps eight: its per-wave moment sums
// live in LDS beside a histogram window that is already small.
constexpr int k1_waves(bool fp32, int pmax, int qmax) {
    return (qmax == 0 ||
            (fp32 ? ((pmax >= 16 && qmax == 12) || (pmax == 32 && qmax == 8))
                  : (qmax == 12 ? pmax > 1 : (qmax == 8 ? pmax > 6 : pmax > 16))))
               ? 8 : 16;
}
// Threads per workgroup of the stream kernel with mirror node pairs for a
// precision and bucket (1024, 768 or 512: four, three or two waves per SIMD,
// one workgroup per compute unit); alt: the other form the autotuner may pick.
int k1p_block(int fp32, int pmax, int qmax, int alt);
constexpr int kLdsPairBudget = 150 * 1024;   // LDS bytes of a mirror-pair stream workgroup
// its largest chunk (longer than the 65535 a 16-bit window count holds: the
// kernel moves large counts to the overflow grid between segments)
constexpr int64_t kMaxPairChunk = (int64_t)1 << 24;
// Mode and node buckets the mirror-pair stream kernel is built for.
constexpr bool k1p_buckets(int pmax, int qmax) {
    return (qmax == 8 || qmax == 12) && (pmax == 3 || pmax == 6 || pmax == 9 || pmax == 16);
}
constexpr int kMaxStreamWG = 4096;    // cap on stream workgroups of one instance (sizes the slabs)
constexpr int kMaxChunk = 8192;       // cap on particles per stream workgroup (LDS list)
static_assert(kMaxChunk <= 65535, "the generic stream kernel's 16-bit window counts");
constexpr int kK2Grid = 1024;         // persistent collider workgroups of one launch

// Per-instance values that change from step to step, resident in device
// memory.  The kernels of a step read them instead of taking them as launch
// arguments, so the launches of every step are identical and a captured graph
// can replay them.
//
// The global step counter n (random streams, buffer parity) is kept in three
// copies, one per step kernel, each advanced by the kernel that runs after its
// reader: the finalize kernel of step n advances the stream kernel's copy, the
// collider the finalize kernel's, the next stream kernel the collider's.  So a
// copy never changes while its reader runs, and no kernel has to find out
// when all of its workgroups are done.  Before the stream kernel of step n:
// step_k1 = step_k3 = n, step_k2 = n - 1.  Bins-only passes advance nothing.
struct Dyn {
    uint32_t step_k1;    // n as read by the stream kernel
    uint32_t step_k3;    // n as read by the finalize kernel
    uint32_t step_k2;    // n as read by the collider
    uint32_t rec_base;   // value of n at record index 0
    double dt;           // time step, s
    double vfdt;         // v_F dt, m: the drift of mode h is vfdt * ehat[h]
    double v_f;          // m/s
    double pad2;
};

// Stream kernel: every particle of a chunk, lane per particle.  From the
// state at t^n it bins H^n and sums the moments at t^n; then it applies the
// Galerkin drift and decides with a rigorous rate bound whether the particle
// may collide in this step; candidates go to a global work list.  One launch
// covers the instances of a group; the descriptors live in device memory.
template <typename T>
struct K1Args {
    T* kx;
    T* ky;
    int64_t n;
    int P, Q;
    DevTab<T> tab;
    const double* ehat;     // [P] Galerkin field coefficients (V/m)
    Dyn* dyn;
    uint32_t seed_lo, seed_hi, instance, pad;
    uint32_t* extra;        // overflow grid of H^n (outside the LDS window)
    uint32_t* slabs;        // [nwg][hwin_words] window slabs of H^n
    int win, win_r0, win_l0, hwin_words;
    double* partial;        // [nwg][Q][3] moment sums at t^n
    int* cand;              // global list of collision candidates
    uint32_t* qc;           // [2][2] candidate count (and a spare word), by step parity
    unsigned long long* counters;
    int64_t chunk;
    uint32_t* excess;       // [max_steps + 1][Q]: this time's slot is cleared here
};

// Collider kernel: a group of G lanes per candidate, one node per lane;
// the passes of the instances' candidate lists dealt out round-robin.
template <typename T>
struct K2Args {
    T* kx;
    T* ky;
    int64_t n;
    int P, Q, G, pad;       // G: lanes per candidate (power of two)
    DevTab<T> tab;
    const double* ehat;
    Dyn* dyn;
    uint32_t seed_lo, seed_hi, instance, pad2;
    const uint32_t* H;      // [3][hstride] histograms, H^n at n mod 3
    const uint32_t* Hmax;   // [3][hmstride] their per-node maxima
    int64_t hstride;
    int64_t hmstride;
    const int* cand;
    uint32_t* qc;
    unsigned long long* counters;
};

// Finalize kernel: H^n from the slabs and the overflow grid, its maximum,
// the moment record of t^n, and the reset of the next step's counters.
constexpr int kK3Words = 64;      // window words per finalize workgroup
constexpr int kK3Lanes = 16;      // slab lanes per column of four words
constexpr int kK3Rest = 2048;     // cells per workgroup of the outside part
constexpr int kK3Direct = 16;     // at most this many slabs: a thread sums whole words itself

struct K3Args {
    int Q, nk;
    const uint32_t* slabs;  // [nwg][hwin_words]
    int hwin_words, win, win_r0, win_l0;
    uint32_t* extra;        // [Q][nk][nk] overflow counts (zeroed here)
    uint32_t* H;            // [3][hstride]
    uint32_t* Hmax;         // [3][hmstride]
    int64_t hstride, hmstride;
    uint32_t* qc;           // [2][2] counters by step parity
    int n_win_wg;           // workgroups of the window part
    int nwg, nb;            // stream workgroups and moment batches
    int fold;               // window blocks of kK3Words words per workgroup
    const double* partial;  // [nwg][Q][3]
    double* record;         // [max_steps + 1][kNumBatches][Q][3], batches b < nb used
    Dyn* dyn;
    const uint32_t* cap;    // [Q] maximum occupation number per node
    uint32_t* excess;       // [max_steps + 1][Q] particles above it, per time
    int mirror;             // window layout: 0 node q in half q & 1 of plane q >> 1;
                            // 1 (mirror pairs) pair p in plane p, node p low, Q-1-p high
    int pad_;
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

// Moments of the particle expansion at up to kMomZ points z per launch.
constexpr int kMomZ = 8;          // points per launch
constexpr int kMomWG = 256;       // workgroups per launch (partials)
struct MomAtArgs {
    const void* kx; const void* ky;
    int fp32;
    int64_t n;
    int P, nz;
    const double* zpsi;   // [nz][P + 1]: Psi_h(z_j), then eps0(z_j)
    double v_f;           // m/s
    double* partial;      // [kMomWG][kMomZ][3] sums of v_x, v_y, eps
};

// Kernel launchers (sgpm_kernels.hip).  Return hipError_t as int.  The
// batched launchers take device arrays of descriptors of n_inst instances of
// one shape group and wg0[n_inst + 1], the first workgroup of each instance.
int launch_k1(int fp32, int pmax, int qmax, int paired, const void* args, const uint32_t* wg0,
              int n_inst, int moving, unsigned grid, size_t lds, void* stream, int alt, int nt);
int launch_k2(int fp32, int pmax, int npl, int lanes, const void* args, int n_inst,
              unsigned grid, size_t lds, void* stream);
int launch_k3(const K3Args* args, const uint32_t* wg0, int n_inst, int moving, unsigned grid,
              void* stream);
int launch_set_dyn(Dyn* d, int n, int set_step, uint32_t step, uint32_t rec_base, int set_dt,
                   double dt, void* stream);
int pmax_bucket(int P);
int qmax_bucket(int Q);
int launch_init(const InitArgs& a, void* stream);
int launch_energy_hist(const EnergyHistArgs& a, void* stream);
int launch_moments_at(const MomAtArgs& a, int nwg, void* stream);
double density_at(double eps0, double mu, double kT);   // electrons per m^2
int launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n,
                  void* stream);
size_t k1_lds_bytes(int P, int Q, int fp32, int paired, int hwin_words, int64_t chunk,
                    int alt);
size_t k2_lds_bytes(int P, int Q, int fp32);
size_t k2l_lds_bytes(int P, int Q, int fp32);   // the collider with a lane per candidate
int k3_grid_of(int Q, int nk, int n_win_wg, int nb);

}  // namespace sgpm
