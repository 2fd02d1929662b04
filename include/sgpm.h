/*
 * sgpm.h -- C-ABI of the MI355X (gfx950) implementation of the per-time-step
 * hot path of the stochastic-Galerkin particle method (sG-PM) for the
 * space-homogeneous semiclassical Boltzmann equation of electrons in a
 * graphene nanoribbon with uncertain band gap and field
 * (Medaglia, Nastasi, Romano, Zanella, arXiv:2404.19602).
 *
 * Problem statement (Sec. 4, "Semiclassical BE in the presence of
 * uncertainties"): f(t,k,z) solves df/dt - (e/hbar) E(z).grad_k f = C[f,f]
 * with a Fermi-Dirac initial datum at the band of width W(z); the quantities
 * of interest are expectations over z of the velocity, current and energy
 * moments (Sec. 4.2).  Each particle carries the gPC coefficients of its
 * wave-vector k_i(z) (Sec. 4.1 eq. gPC); one step is the Galerkin drift
 * followed by the nodal collision step of Algorithm 2 with the Pauli factor
 * taken from the previous-step k-histogram (Sec. 3, eq. Pauli).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Units: energies in eV; wave-vectors as kappa = hbar v_F k in eV (the
 *    paper states its grid in these units, L_k hbar v_F = 5 eV); fields in
 *    V/m; times in s; velocities in m/s; current densities in A/m.
 *  - Device memory is owned by the caller: sgpm_workspace_bytes() tells how
 *    much, sgpm_create() receives a device pointer to it.  The library never
 *    allocates device memory.  Host memory for outputs is owned by the caller.
 *  - All device work is enqueued on the HIP stream given at creation
 *    (hipStream_t passed as void*; NULL = the default stream).  Calls that
 *    return host data synchronise that stream.
 *  - Errors: every call returns an sgpm_status.  Arguments are validated
 *    before any device work (SGPM_EINVAL).  A HIP failure returns
 *    SGPM_EDEVICE and poisons the context: later calls return SGPM_ESTATE.
 *    sgpm_last_error() gives a message.  No C++ exception crosses the ABI.
 *  - A context is not thread-safe; use one context per host thread/stream.
 *
 * Layouts
 * -------
 *  - Uncertain variables z are uniform on [-1,1]^dim_z.  Nodes: tensor
 *    Gauss-Legendre with nodes_1d points per dimension, node q = q1 + nodes_1d*q2
 *    for dim_z = 2 (z_1 fastest); weights w_q sum to one.
 *  - Basis: orthonormal Legendre products; for dim_z = 2 the total-degree
 *    basis in graded order (t = 0..M; within t the exponent of z_1 runs from
 *    t down to 0): (0,0),(1,0),(0,1),(2,0),(1,1),(0,2),...  P modes.
 *  - State: structure of arrays, kx[h][i] then ky[h][i] for h < P, i < N
 *    (FP64 in the host-facing calls regardless of the device precision).
 *  - Histogram: uint32 H[q][r][l], r = x index, l = y index of the cell of
 *    [-L_k, L_k]^2 split in nk x nk cells.
 */
#ifndef SGPM_H
#define SGPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sgpm_ctx sgpm_ctx;

typedef enum {
    SGPM_OK = 0,
    SGPM_EINVAL = 1,       /* invalid argument or descriptor                */
    SGPM_ENOMEM = 2,       /* host allocation failed                        */
    SGPM_EWORKSPACE = 3,   /* workspace missing, too small or misaligned    */
    SGPM_EDEVICE = 4,      /* a HIP call failed (context is now poisoned)   */
    SGPM_ESTATE = 5,       /* call not valid in the current state           */
    SGPM_EUNSUPPORTED = 6  /* combination the library does not support     */
} sgpm_status;

typedef enum { SGPM_FP64 = 0, SGPM_FP32 = 1 } sgpm_precision;

/* Per-mechanism order of the rate vector (Sec. 3 eq. lambda). */
enum { SGPM_AC = 0, SGPM_OP_EM = 1, SGPM_OP_AB = 2, SGPM_K_EM = 3, SGPM_K_AB = 4, SGPM_EDGE = 5 };

/* Counters (sgpm_counters), cumulative since sgpm_init_particles/sgpm_set_state. */
enum {
    SGPM_CNT_COLLISIONS = 0,   /* collision iterations (per particle)            */
    SGPM_CNT_EVENTS = 1,       /* non-self events at a node, before Pauli        */
    SGPM_CNT_PAULI_REJ = 2,    /* node events rejected by the Pauli acceptance   */
    SGPM_CNT_EDGE_EXH = 3,     /* edge angle proposals exhausted (kept as self)  */
    SGPM_CNT_CMAX = 4,         /* particles that reached the collision cap       */
    SGPM_CNT_OUT_OF_GRID = 5,  /* node values outside the histogram grid         */
    SGPM_CNT_CANDIDATES = 6,   /* particles the rate bound could not clear       */
    SGPM_N_COUNTERS = 8
};

/* Step kernels, in the order they run within a step (sgpm_kernel_times). */
enum {
    SGPM_KERNEL_STREAM = 0,    /* drift, node evaluation, histogram window, moments,
                                  rate bound and candidate list (all particles)     */
    SGPM_KERNEL_FINALIZE = 1,  /* H^n and its maxima, moment record of t^n          */
    SGPM_KERNEL_COLLIDE = 2,   /* collision loop of the candidates (Algorithm 2)    */
    SGPM_N_KERNELS = 3
};

/* Largest number of instances of one context. */
#define SGPM_MAX_INSTANCES 1024

/* One simulation instance.  Defaults in brackets are the paper's. */
typedef struct {
    int32_t dim_z;          /* number of uncertain inputs: 0, 1 or 2              */
    int32_t degree;         /* gPC total degree M (P = M+1 for dim_z = 1)         */
    int32_t nodes_1d;       /* Gauss-Legendre nodes per uncertain dimension       */
    int32_t precision;      /* sgpm_precision of the particle state and kernels   */
    int64_t n_particles;    /* N >= 1                                             */
    int32_t gap_mode;       /* 0: band gap in eV, gap(z) = gap0 (1 + gap_rel z)     */
                            /* 1: ribbon width in nm, W(z) = gap0 (1 + gap_rel z)   */
    int32_t gap_dim;        /* component of z driving gap/width, -1: deterministic */
    double gap0, gap_rel;
    int32_t field_dim;      /* component of z driving the field, -1: deterministic */
    double field0, field_rel; /* E_x(z) = field0 (1 + field_rel z), V/m           */
    double fermi_eV;        /* Fermi level of the initial datum [0.4]              */
    double temp_K;          /* lattice temperature: Bose factors, acoustic rate    */
                            /* [300]                                                */
    double alpha;           /* self-scattering parameter of eq. gamma_tot [0.1]     */
    int32_t nk;             /* histogram cells per axis [240], 2..4096, Q nk^2 < 2^30 */
    double lk_eV;           /* grid half-width L_k hbar v_F [5]                     */
    int32_t pauli;          /* 1: Pauli acceptance on [1]                           */
    int32_t final_state;    /* 0: energy-conserving phonon final state [0]; 1: the  */
                            /*    paper-literal |k| -/+ omega/v_F                   */
    double rate_scale[6];   /* test knob per mechanism, 1 = physics                 */
    uint64_t seed;          /* Philox key                                           */
    uint32_t instance_id;   /* Philox counter word 3                                */
    int32_t c_max;          /* cap on collisions per particle per step [32], <= 255 */
    int32_t max_steps;      /* capacity of the moment record (steps after init)    */
    int32_t splitting;      /* 0: drift dt, then the collisions (the paper's first- */
                            /*    order splitting) [0]; 1: Strang, drift dt/2,      */
                            /*    collisions, drift dt/2 (higher-order splittings,  */
                            /*    Sec. 3); the Pauli lookup then moves the grid by  */
                            /*    the first half drift                              */
    double init_temp_K;     /* temperature of the Fermi-Dirac initial datum and of  */
                            /* the density n(z) of the current J = -e n V; 0 takes */
                            /* temp_K [0].  A hot start (init_temp_K > temp_K) at  */
                            /* zero field relaxes toward the lattice temperature    */
} sgpm_instance_desc;

/* Fill a descriptor with the paper's defaults (Table 1 and Sec. 5). */
void sgpm_default_desc(sgpm_instance_desc* d);

/* Device workspace needed for n_inst instances (bytes, 256-byte aligned
 * start required).  Returns SGPM_EINVAL for an invalid descriptor. */
sgpm_status sgpm_workspace_bytes(const sgpm_instance_desc* descs, int32_t n_inst, size_t* bytes);

/* Create a context over a caller-owned device workspace of ws_bytes bytes.
 * Builds the FP64 set-up tables on the host (nodes, weights, basis, Galerkin
 * field coefficients, rate constants of the Appendix, Fermi-Dirac CDF
 * tables) and uploads them.  *out receives the context (host memory owned
 * by the library, released by sgpm_destroy).  1 <= n_inst <=
 * SGPM_MAX_INSTANCES.  Instances of the same precision and similar size of
 * basis and node set are stepped by shared launches (one per kernel and
 * step for the whole group); the particles of different instances never
 * interact. */
sgpm_status sgpm_create(const sgpm_instance_desc* descs, int32_t n_inst, void* dev_workspace,
                        size_t ws_bytes, void* hip_stream, sgpm_ctx** out);

/* Fermi-Dirac initial particles at every node, projected onto the gPC modes
 * (Sec. 4 uncertain initial condition); builds H^0 and records the moments
 * at t = 0.  Resets the step counter and the counters.  Asynchronous. */
sgpm_status sgpm_init_particles(sgpm_ctx* ctx);

/* Advance every instance by n_steps steps of length dt_s (Sec. 4.1: Galerkin
 * drift, then the collision step of Algorithm 2 against H^n; H^{n+1} and the
 * moments at t^{n+1} are built by the same pass).  Asynchronous.  By default
 * the steps are replayed from captured HIP graphs of a block of steps
 * (sgpm_set_graph); results do not depend on how they are launched. */
sgpm_status sgpm_step(sgpm_ctx* ctx, double dt_s, int64_t n_steps);

/* LDS bytes of a stream workgroup of instance inst, which size its histogram
 * window (the square of cells around the grid centre counted in LDS; counts
 * outside go through device atomics): 0 = the default (80 KiB for the
 * generic kernel, 150 KiB or the device's limit for the mirror-pair kernel),
 * else 16 KiB to 150 KiB (clamped to the default's maximum).  Results do not
 * depend on it.  Allowed right after init/set_state. */
sgpm_status sgpm_set_stream_lds(sgpm_ctx* ctx, int32_t inst, int32_t bytes);

/* Histogram window of instance inst: its side in cells and the LDS bytes of a
 * stream workgroup (either pointer may be NULL). */
sgpm_status sgpm_window(const sgpm_ctx* ctx, int32_t inst, int32_t* win, int32_t* lds_bytes);

/* Stream kernel of the instances with one uncertain input and 2 to 12 nodes:
 * on > 0 the mirror-pair kernel, which evaluates the nodes z_q and -z_q of
 * the symmetric Gauss-Legendre rule together from the even and odd modes;
 * 0 the generic kernel, one node at a time; on < 0 (the default) the pair
 * kernel for shape groups (instances launched together) of 2^22 particles
 * or more, the generic one below.  Results agree to rounding (the node
 * values are summed in another order).  Resets every instance's chunk to
 * the automatic one; allowed right after init/set_state (the current time
 * is re-recorded). */
sgpm_status sgpm_set_node_pairs(sgpm_ctx* ctx, int32_t on);

/* Collider of the instances with at most 12 nodes and 16 modes: on > 0 a lane per
 * candidate, which loops over the candidate's nodes; 0 a group of lanes per
 * candidate, a node per lane (the form used beyond 12 nodes); on < 0 (the
 * default) the lane form for shape groups of 2^22 particles or more.  The
 * two compute every quantity by the same expressions in the same order:
 * results are identical.  Allowed at any time. */
sgpm_status sgpm_set_collider_lanes(sgpm_ctx* ctx, int32_t on);

/* *paired = 1 if instance inst is stepped by the mirror-pair stream kernel. */
sgpm_status sgpm_node_pairs(const sgpm_ctx* ctx, int32_t inst, int32_t* paired);

/* *lanes = 1 if the candidates of instance inst are collided a lane per
 * candidate, 0 if a group of lanes per candidate. */
sgpm_status sgpm_collider_lanes(const sgpm_ctx* ctx, int32_t inst, int32_t* lanes);

/* Threads per workgroup of the mirror-pair stream kernel: alt = 0 the default
 * form of each instantiation (1024, 768 or 512 threads, by the registers it
 * needs), 1 the other one (512 for a default of 768, else 768); sgpm_autotune
 * tries both and keeps the faster.  The state, histograms and counters are the
 * same in both; the FP64 moment sums group the particles by lane differently
 * (they agree to rounding).  Allowed at any time after sgpm_create. */
sgpm_status sgpm_set_pair_block(sgpm_ctx* ctx, int32_t alt);

/* *threads = threads per workgroup of the stream kernel of instance inst. */
sgpm_status sgpm_stream_threads(const sgpm_ctx* ctx, int32_t inst, int32_t* threads);

/* Cache hints of the mirror-pair stream kernel's state access: mode 1 reads
 * the state and writes its drift with non-temporal hints, 0 with ordinary
 * ones, -1 (the default) non-temporal when the state of some instance exceeds
 * 1 GiB (several times the last-level cache: it is streamed through once per
 * step, and caching it only evicts what the collider could reuse).  The
 * results are identical either way.  Allowed at any time after sgpm_create;
 * EINVAL for another mode. */
sgpm_status sgpm_set_stream_nontemporal(sgpm_ctx* ctx, int32_t mode);

/* *on = 1 if the stream kernels use non-temporal hints now. */
sgpm_status sgpm_stream_nontemporal(const sgpm_ctx* ctx, int32_t* on);

/* Launch mode of sgpm_step: 0 = every kernel launched on the stream; B >= 1
 * = blocks of B steps captured once as a HIP graph (on a private stream) and
 * replayed on the context's stream, remainders from a graph of their own
 * length.  B <= 256; default 16.  Graphs are rebuilt after sgpm_set_chunk. */
sgpm_status sgpm_set_graph(sgpm_ctx* ctx, int32_t steps_per_graph);

/* on != 0: the following sgpm_step calls launch every kernel on the stream
 * with a HIP event after each, for sgpm_kernel_times (slightly slower). */
sgpm_status sgpm_set_profiling(sgpm_ctx* ctx, int32_t on);

/* Per-kernel device time of the last profiled sgpm_step call: avg_ms[k] =
 * mean time between the events around launch k of kind SGPM_KERNEL_*,
 * launches[k] = their number (may be NULL).  Arrays of SGPM_N_KERNELS.
 * Waits for the last event.  Zeros if no profiled call was made. */
sgpm_status sgpm_kernel_times(sgpm_ctx* ctx, double* avg_ms, int64_t* launches);

/* Global step counter (the random streams are keyed by it). */
sgpm_status sgpm_step_count(const sgpm_ctx* ctx, int64_t* steps);

/* Number of recorded times of instance inst (1 right after init/set_state,
 * plus one per step since). */
sgpm_status sgpm_record_length(const sgpm_ctx* ctx, int32_t inst, int64_t* len);

/* Moments for recorded times t_first .. t_first+count-1 (time index 0 is
 * t = 0, index n is after n steps).  per_node[count][Q][4]: V_x, V_y (m/s),
 * mean energy (eV), J_x = -e n(z_q) V_x (A/m).  agg[count][SGPM_N_AGG]:
 * expectations and variances over z by the nodal quadrature (Sec. 4.2) and
 * Monte Carlo standard errors by batch means over particle batches.
 * Either output may be NULL.  Synchronises the stream. */
enum {
    SGPM_AGG_E_VX = 0, SGPM_AGG_VAR_VX, SGPM_AGG_E_JX, SGPM_AGG_VAR_JX, SGPM_AGG_E_EN,
    SGPM_AGG_VAR_EN, SGPM_AGG_SE_E_VX, SGPM_AGG_SE_VAR_VX, SGPM_AGG_SE_E_JX,
    SGPM_AGG_SE_VAR_JX, SGPM_AGG_SE_E_EN, SGPM_AGG_SE_VAR_EN, SGPM_N_AGG
};
sgpm_status sgpm_moments(sgpm_ctx* ctx, int32_t inst, int64_t t_first, int64_t count,
                         double* per_node, double* agg);

/* Reconstructed energy distribution (Sec. 4.1 eq. f_gPC, binned in energy):
 * nodes[Q][nbins] = fraction of particles whose energy at node q lies in bin
 * b, per eV; modes[P][nbins] = sum_q w_q Psi_h(z_q) nodes[q][b].  Bins split
 * [emin, emax) uniformly.  Either output may be NULL.  Synchronises. */
sgpm_status sgpm_reconstruct_f(sgpm_ctx* ctx, int32_t inst, int32_t nbins, double emin_eV,
                               double emax_eV, double* nodes, double* modes);

/* Moments of the particle expansion at points z (Sec. 4.2): every particle's
 * wave-vector evaluated at z, k_i(z) = sum_h k_h Psi_h(z), on the band of
 * that z.  z is [n_z][dim_z] (ignored for dim_z = 0); out is [n_z][4]:
 * V_x, V_y (m/s), mean energy (eV) and J_x = -e n(z) V_x (A/m) with the
 * Fermi-Dirac equilibrium density n(z) of that band.  Sums in FP64 in a
 * fixed order.  The gap must be positive at every z.  Synchronises the
 * stream.  Used for the quantities at z between the nodes: percentile bands
 * over z, the L2(z) error of a truncation order. */
sgpm_status sgpm_moments_at(sgpm_ctx* ctx, int32_t inst, int32_t n_z, const double* z,
                            double* out);

/* The uncertain inputs of instance inst at points z (Sec. 4: the band of
 * width W(z) and the field E(z) of the problem statement): z is
 * [n_z][dim_z] (ignored for dim_z = 0); out is [n_z][4]: band gap 2 eps0(z)
 * (eV), band minimum eps0(z) = hbar v_F pi / W(z) (eV), width W(z) (m) and
 * field E_x(z) (V/m).  A gap that is not positive gives zeros in the first
 * three.  Host only, no device work.  For deterministic runs at sampled z
 * (Monte Carlo sampling of the uncertain inputs). */
sgpm_status sgpm_inputs_at(const sgpm_ctx* ctx, int32_t inst, int32_t n_z, const double* z,
                           double* out);

/* Energy distribution of the particles reconstructed at arbitrary points z
 * (k_i(z) = sum_h k_h Psi_h(z)); z[n_z][dim_z], out[n_z][nbins].  Positive
 * by construction.  Synchronises. */
sgpm_status sgpm_reconstruct_f_at(sgpm_ctx* ctx, int32_t inst, int32_t n_z, const double* z,
                                  int32_t nbins, double emin_eV, double emax_eV, double* out);

/* Pauli violation (Sec. 5, Test 1): for each recorded time, the number of
 * particles above the maximum occupation number, sum over the cells c of
 * max(0, H_q[c] - cap_q), per node q.  cap_q is the largest cell count of
 * node q at record index 0 (the initial datum, or the state given to
 * sgpm_set_state): the occupation of a full cell for this Fermi level and
 * particle count.  out is [count][Q]; synchronises the stream.  The paper's
 * N-bar is the maximum over the times divided by N. */
sgpm_status sgpm_occupancy_excess(sgpm_ctx* ctx, int32_t inst, int64_t t_first, int64_t count,
                                  uint32_t* out);

/* Copy the coefficients in or out (host FP64 arrays kx[P][N] then ky[P][N]
 * in one buffer of 2*P*N doubles).  set_state rebuilds the histogram of the
 * given state, records it as time index 0 and sets the step counter (the
 * random streams depend on it).  Both synchronise. */
sgpm_status sgpm_set_state(sgpm_ctx* ctx, int32_t inst, const double* khat, int64_t step);
sgpm_status sgpm_get_state(sgpm_ctx* ctx, int32_t inst, double* khat);

/* Current histogram H^n (uint32 [Q][nk][nk]) and per-node max (uint32 [Q]).
 * Either may be NULL.  Synchronises. */
sgpm_status sgpm_get_histogram(sgpm_ctx* ctx, int32_t inst, uint32_t* H, uint32_t* Hmax);

/* Counters, uint64 [SGPM_N_COUNTERS].  Synchronises. */
sgpm_status sgpm_counters(sgpm_ctx* ctx, int32_t inst, uint64_t* out);

/* Sizes of instance inst: P modes, Q nodes. */
sgpm_status sgpm_sizes(const sgpm_ctx* ctx, int32_t inst, int32_t* P, int32_t* Q);

/* Host copies of the set-up tables of instance inst (any may be NULL):
 * z[Q][2], w[Q], psi[Q][P], ehat[P], eps0[Q], width_m[Q], field[Q],
 * density_m2[Q]. */
sgpm_status sgpm_tables(const sgpm_ctx* ctx, int32_t inst, double* z, double* w, double* psi,
                        double* ehat, double* eps0, double* width_m, double* field,
                        double* density_m2);

/* Launch shape: particles per workgroup chunk (a multiple of 1024, at most
 * 8192 -- 2^24 with the mirror-pair stream kernel --, at least a quarter of
 * the automatic choice of about N/256, and large enough for at most 4096
 * workgroups) of the step kernels of instance inst;
 * 0 restores the automatic
 * choice.  Particle trajectories, histograms and counters do not depend on
 * it; the FP64 moment sums only through their order.  Allowed right after
 * init/set_state (the current time is re-recorded). */
sgpm_status sgpm_set_chunk(sgpm_ctx* ctx, int32_t inst, int32_t chunk);

/* Autotuner of the launch shape.  From the current state of every instance
 * it runs trial_steps steps of length dt_s (launched kernel by kernel, timed
 * with HIP events on the context's stream) for each candidate shape: every
 * instance's chunk scaled by 1/4, 1/2, 1, 2 or 4 from the automatic one
 * (within the limits of sgpm_set_chunk), times 512, 1024 or 2048 collider
 * workgroups.  A grid other than 1024 must be more than 3 % faster, and so
 * must chunks other than the automatic ones (the two margins multiply).
 * Then, if some instance is stepped by the mirror-pair stream kernel, the
 * other workgroup size of that kernel (sgpm_set_pair_block) at the best
 * shape, kept if it is more than 3 % faster.
 * Between trials and at the end it puts back the particle state, the step
 * counter and the counters, and rebuilds the histogram.
 * Keeps the fastest shape (results do not depend on it; see sgpm_set_chunk)
 * and returns its device time per step in *best_ms_per_step (may be NULL).
 * Needs trial_steps <= max_steps of every instance (1 <= trial_steps <=
 * 1000).  The maximum occupation number (sgpm_occupancy_excess) is kept.
 * The moment record continues when every record has room for the trials
 * after the current time and the chunks are unchanged; otherwise it restarts
 * at the current time.  Synchronises the stream; host copies of the state
 * are made. */
sgpm_status sgpm_autotune(sgpm_ctx* ctx, double dt_s, int32_t trial_steps,
                          double* best_ms_per_step);

/* Current launch shape: chunk and stream workgroups of instance inst, and
 * the collider's workgroups per launch (any pointer may be NULL). */
sgpm_status sgpm_launch_shape(const sgpm_ctx* ctx, int32_t inst, int32_t* chunk,
                              int32_t* stream_workgroups, int32_t* collider_workgroups);

/* Device time (ms) of the last sgpm_step call divided by its step count,
 * measured with HIP events on the context's stream around all of its work
 * (the steps and the closing pass over the final state); 0 if none. */
sgpm_status sgpm_last_step_ms(sgpm_ctx* ctx, double* ms_per_step);

void sgpm_destroy(sgpm_ctx* ctx);
const char* sgpm_last_error(const sgpm_ctx* ctx);
const char* sgpm_status_string(sgpm_status s);

/* Test hook: Philox4x32-10 over n counters on the device.  d_ctr[n][4],
 * d_key[n][2], d_out[n][4] are device pointers; enqueued on hip_stream and
 * synchronised.  Used to check the device generator against the published
 * known answers. */
sgpm_status sgpm_philox_device(const uint32_t* d_ctr, const uint32_t* d_key, uint32_t* d_out,
                               int64_t n, void* hip_stream);

/* Allocation-free energy distribution, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same reconstruction as sgpm_reconstruct_f's
 * nodes output, out[q][b] = fraction of the n particles whose energy at node
 * q lies in bin b, per eV, but from caller device arrays and without a
 * context.  kx, ky: device coefficients [P][n] each (double for SGPM_FP64,
 * float for SGPM_FP32); psi: device [Q][P] basis values Psi_h(z_q); eps0:
 * device [Q] band minima (eV); out: device [Q][nbins] doubles.  Bins split
 * [emin, emax) uniformly.  Asynchronous on hip_stream; no hipMalloc, hipFree
 * or allocating library call.  The bin counts live in a fixed device array
 * of 2^19 counts (4 MiB) per GPU, held until the process ends: Q * nbins
 * above 2^19 returns SGPM_EUNSUPPORTED.  Every call on one GPU shares that
 * array (cleared by the call itself), so calls that overlap on one GPU --
 * on different streams or host threads -- race. */
sgpm_status sgpm_energy_density_noalloc(const void* kx, const void* ky, int32_t precision,
                                        int64_t n, int32_t P, int32_t Q, const double* psi,
                                        const double* eps0, int32_t nbins, double emin_eV,
                                        double emax_eV, double* out, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* SGPM_H */
