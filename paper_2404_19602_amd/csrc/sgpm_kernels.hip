// gfx950 kernels of the sG-PM hot path (arXiv:2404.19602, Algorithm 2).
//
// One time step n of a group of instances is three launches, in this order:
//  K1 stream   -- a lane per particle, a chunk of particles per 1024- (or
//                 512-) thread workgroup.  For every particle: the node values k_i(z_q)
//                 of the state at t^n (eq. gPC), their cells in H^n through
//                 a privatised LDS window (flushed as one slab per
//                 workgroup, overflow cells by global atomics), and FP64
//                 sums of v_x, v_y and the energy per node (Sec. 4.2).  Then
//                 the Galerkin drift (Sec. 4.1) and an upper bound of the
//                 node-maximum collision rate (eq. deltat) that proves most
//                 particles do not collide in this step: those write back
//                 their drifted modes, the others are listed as candidates.
//  K3 finalize -- H^n from the slabs and the overflow grid, its maximum per
//                 node, the occupancy excess, the fixed-order reduction of
//                 the moment sums into the record of t^n, and the clearing
//                 of the next step's counters and stale buffers.
//  K2 collide  -- the candidates, a group of lanes per candidate and one
//                 node per lane: exact node rates, the node maximum, free
//                 flight, mechanism selection (eq. update_gPC), final states,
//                 Pauli acceptance against H^n on the moved grid (eq.
//                 Pauli_gPC) and the projection of eq. update_sG as a group
//                 sum, repeated while the flight ends inside the step; then
//                 the candidate's modes are written back.
// Each kernel reads its own copy of the step counter in device memory and
// advances the copy of the kernel that runs after it (struct Dyn).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <type_traits>
#include <stdint.h>

#include "sgpm_internal.h"

namespace sgpm {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11); counter (c0,c1,c2,c3), key (k0,k1).
struct Words { uint32_t w0, w1, w2, w3; };

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    return Words{c0, c1, c2, c3};
}

// A collider draw.  In FP32 the key passes through an empty asm, so the key
// schedule is recomputed (scalar adds) at each of the several draws per
// collision instead of being kept in scalar registers across the loop, which
// spills them into vector lanes: that takes the FP32 collider from 115 to 85
// VGPRs.  In FP64 the same measured 0.4 us slower per launch, so there the
// schedule is kept.
template <typename T>
__device__ __forceinline__ Words k2_draw(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1) {
    if constexpr (sizeof(T) == 4) __asm__ volatile("" : "+s"(k0), "+s"(k1));
    return philox10(c0, c1, c2, c3, k0, k1);
}

enum : uint32_t { kPurXi = 0, kPurSel = 1, kPurAng = 2, kPurEdge0 = 16, kPurInit = 255 };

// Uniforms strictly inside (0,1): FP64 from the top 52 bits of (hi,lo),
// FP32 from the top 23 bits of hi; every value is exactly representable.
template <typename T> __device__ __forceinline__ T uni(uint32_t hi, uint32_t lo);
template <> __device__ __forceinline__ double uni<double>(uint32_t hi, uint32_t lo) {
    const uint64_t m = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return ((double)m + 0.5) * 0x1p-52;
}
template <> __device__ __forceinline__ float uni<float>(uint32_t hi, uint32_t) {
    return ((float)(hi >> 9) + 0.5f) * 0x1p-23f;
}

template <typename T> struct Num;
template <> struct Num<double> {
    static constexpr double trap = 6.283185307179586476925286766559 / kEdgePts;
    static constexpr double eps = 2.220446049250313e-16;
};
template <> struct Num<float> {
    static constexpr float trap = 6.28318530717958647692f / kEdgePts;
    static constexpr float eps = 1.1920929e-07f;
};

__device__ __forceinline__ double dlog(double x) { return log(x); }
__device__ __forceinline__ float dlog(float x) { return logf(x); }
__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float dexp(float x) { return expf(x); }
__device__ __forceinline__ void dsincospi(double x, double* s, double* c) { sincospi(x, s, c); }
__device__ __forceinline__ void dsincospi(float x, float* s, float* c) { sincospif(x, s, c); }

// cell coordinate floor((x + L) / dk) of the grid [-L, L) split in cells of
// width dk (computed with the product by 1/dk); outside [0, 2^30) or NaN -> -1
template <typename T>
__device__ __forceinline__ int cell_coord(T x, T L, T inv_dk) {
    const T f = floor((x + L) * inv_dk);
    return (f >= (T)0 && f < (T)1073741824) ? (int)f : -1;
}

// 1/sqrt(a): the hardware estimate refined by one Newton step
__device__ __forceinline__ double rsqrt_nr(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    return y * (1.5 - 0.5 * a * y * y);
}
__device__ __forceinline__ float rsqrt_nr(float a) { return __builtin_amdgcn_rsqf(a); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// gfx950 lane swaps on both 32-bit halves of a pair of doubles: swap32 trades
// lanes 32..63 of a for lanes 0..31 of b; swap16 trades the odd 16-lane rows of
// a for the even rows of b.
__device__ __forceinline__ void swap32_f64(double& a, double& b) {
    const uint64_t ua = (uint64_t)__double_as_longlong(a), ub = (uint64_t)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)ua, (uint32_t)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32),
                                                     false, false);
    a = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
    b = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ void swap16_f64(double& a, double& b) {
    const uint64_t ua = (uint64_t)__double_as_longlong(a), ub = (uint64_t)__double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)ua, (uint32_t)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32),
                                                     false, false);
    a = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
    b = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
}

// x read from another lane of the same 16-lane row (DPP control CTRL).  Every
// call is made with the whole wave active and a control whose source lane
// always exists (quad permutations, row mirrors), so no lane keeps its old
// value and none has to be set beforehand.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF,
                                                           false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Wave sums of V per-lane values.  V is padded with zeros to VP, a multiple
// of 4.  Two halving steps (lanes 32 apart, then 16 apart) leave every lane
// with VP/4 partial sums of four lanes each; the 16 lanes of a row then add
// theirs (quad swaps, half-row and row mirrors), so that row r holds the sums
// of values j + (VP/4)(r & 1) + (VP/2)(r >> 1), j < VP/4.  The first lane of
// each row adds those with index below n_out to out[] (each index owned by
// one lane).  No LDS, no index arithmetic.
template <int V>
__device__ __forceinline__ void wave_sums_add(const double (&v)[V], double* out, int n_out,
                                              int lane) {
    constexpr int VP = (V + 3) & ~3, H2 = VP / 2, H4 = VP / 4;
    double u[H2];
#pragma unroll
    for (int j = 0; j < H2; ++j) {
        double a = v[j], b = j + H2 < V ? v[j + H2] : 0.0;
        swap32_f64(a, b);
        u[j] = a + b;
    }
    double w[H4];
#pragma unroll
    for (int j = 0; j < H4; ++j) {
        double a = u[j], b = u[j + H4];
        swap16_f64(a, b);
        w[j] = a + b;
    }
#pragma unroll
    for (int j = 0; j < H4; ++j) {
        double x = w[j];
        x += dpp_f64<0xB1>(x);    // quad_perm [1,0,3,2]
        x += dpp_f64<0x4E>(x);    // quad_perm [2,3,0,1]
        x += dpp_f64<0x141>(x);   // row_half_mirror
        x += dpp_f64<0x140>(x);   // row_mirror
        w[j] = x;
    }
    if ((lane & 15) == 0) {
        const int r = lane >> 4, base = H4 * (r & 1) + H2 * (r >> 1);
#pragma unroll
        for (int j = 0; j < H4; ++j)
            if (base + j < n_out) out[base + j] += w[j];
    }
}

// Cross-lane exchange through LDS inside one wave: a wave's LDS operations
// are performed in order, so only the compiler must keep them in order.
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <typename T>
__device__ __forceinline__ T group_max(T v, int G) {
    for (int m = G >> 1; m >= 1; m >>= 1) {
        const T o = __shfl_xor(v, m, G);
        v = o > v ? o : v;
    }
    return v;
}

// ------------------------------------------------------- rate evaluations
// the five closed-form phonon rates (Appendix) at energy e of a node with
// band minimum e0, order AC, OP-, OP+, K-, K+
template <typename T>
__device__ __forceinline__ void phonon_rates(const Consts<T>& c, T e, T e0, T r[5]) {
    r[0] = (e - e0 >= (T)0) ? c.c_ac * e : (T)0;
    const T eom = e - c.hw_o, eop = e + c.hw_o, ekm = e - c.hw_k, ekp = e + c.hw_k;
    r[1] = (eom - e0 >= (T)0) ? c.c_om * eom : (T)0;
    r[2] = (eop - e0 >= (T)0) ? c.c_op * eop : (T)0;
    r[3] = (ekm - e0 >= (T)0) ? c.c_km * ekm : (T)0;
    r[4] = (ekp - e0 >= (T)0) ? c.c_kp * ekp : (T)0;
}

// edge rate: cedge * eps * int_0^{2pi} exp(-kap (cos t - c)^2) dt by the
// 32-point trapezoid rule, summed with cos(t_j) = cos(t_{32-j})
template <typename T>
__device__ __forceinline__ T edge_rate(const Consts<T>& c, const T* ecos, T cedge, T e0, T kx,
                                       T ky, T e) {
    const T k2 = kx * kx + ky * ky;
    const T kabs = sqrt(k2);
    const T cin = kabs > (T)0 ? kx / kabs : (T)1;
    const T kap = c.edge_kap * k2;
    const T d0 = ecos[0] - cin, d16 = ecos[kEdgePts / 2] - cin;
    T acc = dexp(-kap * d0 * d0) + dexp(-kap * d16 * d16);
    T mid = (T)0;
#pragma unroll
    for (int j = 1; j < kEdgePts / 2; ++j) {
        const T d = ecos[j] - cin;
        mid += dexp(-kap * d * d);
    }
    acc += (T)2 * mid;
    return (e - e0 >= (T)0) ? cedge * e * (acc * Num<T>::trap) : (T)0;
}

// Upper bound of (1 + alpha) max_q sum_nu Gamma^nu(z_q) given an upper bound
// emax of every nodal energy: each rate is non-decreasing in the energy, the
// angular edge integral is at most 2 pi, emission thresholds use the smallest
// band minimum; the margin covers rounding.
template <typename T>
__device__ __forceinline__ T rate_bound(const Consts<T>& c, T emax) {
    T s = c.b_ac * emax + c.b_op * (emax + c.hw_o) + c.b_kp * (emax + c.hw_k) + c.b_edge * emax;
    if (emax >= c.b_thr_o) s += c.b_om * (emax - c.hw_o);
    if (emax >= c.b_thr_k) s += c.b_km * (emax - c.hw_k);
    return c.alpha1 * s * c.b_margin;
}

// Padded basis tables: the rows of psi and w_q psi are stored with PMAX
// entries (zeros past P) so node evaluation and projection unroll without
// per-mode branches.
int pmax_bucket(int P) {
    if (P <= 1) return 1;
    if (P <= 3) return 3;
    if (P <= 6) return 6;
    if (P <= 9) return 9;
    if (P <= 16) return 16;
    return 32;
}

template <typename T, int PMAX>
__device__ __forceinline__ void eval_node(const T* __restrict__ row, const T (&cx)[PMAX],
                                          const T (&cy)[PMAX], T& kx, T& ky) {
    T x = (T)0, y = (T)0;
#pragma unroll
    for (int h = 0; h < PMAX; ++h) { x += cx[h] * row[h]; y += cy[h] * row[h]; }
    kx = x; ky = y;
}

// The modes whose drift is not zero, as bits in a scalar register (the field
// drives only some of them: the mean mode for a deterministic field), so that
// the stores of the drift test a bit rather than read the table every tile.
template <typename T, int PMAX>
__device__ __forceinline__ uint32_t drift_modes(const T* drift, int P) {
    uint32_t m = 0u;
#pragma unroll
    for (int h = 0; h < PMAX; ++h)
        if (h < P && drift[h] != (T)0) m |= 1u << h;
    return __builtin_amdgcn_readfirstlane(m);
}

// The LDS word a stream-kernel lane increments in place of a window cell when
// its node is outside the window or it holds no particle: one of the
// workgroup's counter words that are never read (the first eight are the
// counters), so that the increment needs no branch around it.
constexpr int kWinSink = 15;

// A value that is the same on every lane, moved into scalar registers.  The
// stream kernels keep the cell map's constants there: read from LDS inside
// the node loop, they would be read again after every window increment (the
// compiler must assume that the increment may change them), and the wait for
// that read would also wait for the increment.
__device__ __forceinline__ double uniform_of(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ float uniform_of(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// A cell coordinate relative to a window origin r0 >= 0, before the floor:
// x - r0 for x = (k + L) / dk.  For x >= r0 the difference is exact (x and
// the integer r0 are multiples of x's unit in the last place, and the
// difference is smaller than x), so x - r0 lies in [0, W) exactly when
// floor(x) - r0 does, and truncating it gives floor(x) - r0; for x < r0 it is
// negative, and a NaN stays a NaN.  The floor itself is then not needed.
template <typename T>
__device__ __forceinline__ T win_offset(T x, int r0) {
    return x - (T)r0;
}

// the coefficients of the particles of one tile: base is the tile's first
// particle (the same for the whole workgroup), t this lane's offset in it, so
// every mode is one uniform pointer plus a 32-bit lane offset.  Modes past P
// repeat mode P-1; the padded basis tables are zero there, so they add nothing.
// NT: non-temporal loads, for a state that does not fit in the last-level
// cache and is streamed through it once per step (a compile-time choice: two
// forms of one load in the branches of a run-time test would be merged into
// one by the compiler, dropping the hint)
template <typename T, int PMAX, bool NT = false>
__device__ __forceinline__ void load_tile_coeffs(const T* __restrict__ kxa, const T* __restrict__ kya,
                                                 int64_t n, int P, int64_t base, uint32_t t,
                                                 T (&cx)[PMAX], T (&cy)[PMAX]) {
#pragma unroll
    for (int h = 0; h < PMAX; ++h) {
        const int hh = h < P ? h : P - 1;
        const T* px = kxa + ((size_t)hh * n + base);
        const T* py = kya + ((size_t)hh * n + base);
        if constexpr (NT) {
            cx[h] = __builtin_nontemporal_load(px + t);
            cy[h] = __builtin_nontemporal_load(py + t);
        } else {
            cx[h] = px[t];
            cy[h] = py[t];
        }
    }
}

// a drift store of the stream kernels, with the hint of the state's loads
template <bool NT, typename T>
__device__ __forceinline__ void store_state(T* p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// coefficients of particle i (drift applied), zero past P, branch-free loads
template <typename T, int PMAX>
__device__ __forceinline__ void load_coeffs(const T* __restrict__ kxa, const T* __restrict__ kya,
                                            int64_t n, int P, int64_t i, const T* drift,
                                            T (&cx)[PMAX], T (&cy)[PMAX]) {
#pragma unroll
    for (int h = 0; h < PMAX; ++h) {
        const int hh = h < P ? h : P - 1;
        const T vx = kxa[(size_t)hh * n + i];
        const T vy = kya[(size_t)hh * n + i];
        cx[h] = h < P ? vx - drift[h] : (T)0;     // k_h -= (e/hbar) dt E_h
        cy[h] = h < P ? vy : (T)0;
    }
}

// Descriptor j of a batched launch, read through the constant address space:
// the array is not written while a kernel runs, and pointers loaded from
// constant memory are known to be global, so their accesses compile to global
// (not flat) instructions.
template <typename D>
__device__ __forceinline__ D load_desc(const D* all, int j) {
    typedef const __attribute__((address_space(4))) D CD;
    return __builtin_bit_cast(D, ((CD*)all)[j]);
}

// Instance of a workgroup of a batched launch: the last j with wg0[j] <= b.
// wg0 ascends from wg0[0] = 0, so j is the number of entries j' >= 1 with
// wg0[j'] <= b: every wave counts them with independent loads and ballots
// (no chain of dependent loads as in a bisection).
__device__ __forceinline__ int find_slot(const uint32_t* __restrict__ wg0, int n_inst, uint32_t b) {
    const int lane = threadIdx.x & 63;
    int cnt = 0;
#pragma unroll 4
    for (int j0 = 0; j0 < n_inst; j0 += 64) {
        const int j = j0 + lane;
        const bool le = j >= 1 && j < n_inst && wg0[j] <= b;
        cnt += __popcll(__ballot(le));
    }
    return cnt;
}

// ======================================================= K1: stream kernel
// LDS of the stream kernel.  The fixed part comes first, at offsets known at
// compile time for a node bucket (QA: the bucket's node count; the many-node
// path uses Q), so that every table read is one base register plus an
// immediate offset: consts, psi, eps0sq, shift, psimax, drift, pdrift, the
// per-wave moment sums and the counters.  Then the window and the candidate
// buffer, whose sizes are set at run time.
__host__ __device__ constexpr size_t k1_fixed_bytes(int PM, int QA, size_t s, int waves) {
    return ((((((sizeof(Consts<double>) + 15) & ~(size_t)15) +
               s * ((size_t)QA * PM + 2 * (size_t)QA + 3 * (size_t)PM) + 15) & ~(size_t)15) +
             (size_t)waves * QA * 3 * 8 + 16 * 4) + 15) & ~(size_t)15;
}

constexpr int kK1PSeg = 256;      // candidate list entries per wave of the mirror-pair kernel

size_t k1_lds_bytes(int P, int Q, int fp32, int paired, int hwin_words, int64_t chunk, int alt) {
    const int PM = pmax_bucket(P), qb = qmax_bucket(Q);
    if (paired) {
        const int waves = k1p_block(fp32, PM, qb, alt) / 64;
        return k1_fixed_bytes(PM, qb, fp32 ? 4 : 8, waves) + (size_t)hwin_words * 4 +
               (size_t)waves * kK1PSeg * 4;   // window, candidate lists of the waves
    }
    return k1_fixed_bytes(PM, qb > 0 ? qb : Q, fp32 ? 4 : 8, k1_waves(fp32 != 0, PM, qb)) +
           (size_t)hwin_words * 4 + (size_t)chunk * 4;   // window, candidate buffer
}

template <typename T>
struct K1Lds {
    uint32_t* hwin;
    int* cbuf;
    Consts<T>* c;
    T* psi; T* eps0sq; T* shift; T* psimax;
    T* drift;    // applied before the collisions (dt, or dt/2 with Strang)
    T* pdrift;   // applied after them (0, or dt/2 with Strang)
    double* red;
    uint32_t* cnt;
};

template <typename T>
__device__ __forceinline__ K1Lds<T> k1_lds(unsigned char* smem, int PM, int QA, int hwin_words,
                                           int waves) {
    K1Lds<T> L;
    size_t off = 0;
    L.c = reinterpret_cast<Consts<T>*>(smem);
    off = (sizeof(Consts<double>) + 15) & ~(size_t)15;
    L.psi = reinterpret_cast<T*>(smem + off);
    L.eps0sq = L.psi + QA * PM;
    L.shift = L.eps0sq + QA;
    L.psimax = L.shift + QA;
    L.drift = L.psimax + PM;
    L.pdrift = L.drift + PM;
    off += sizeof(T) * ((size_t)QA * PM + 2 * QA + 3 * PM);
    off = (off + 15) & ~(size_t)15;
    L.red = reinterpret_cast<double*>(smem + off);
    off += (size_t)waves * QA * 3 * 8;
    L.cnt = reinterpret_cast<uint32_t*>(smem + off);
    off = k1_fixed_bytes(PM, QA, sizeof(T), waves);
    L.hwin = reinterpret_cast<uint32_t*>(smem + off);
    L.cbuf = reinterpret_cast<int*>(smem + off + (size_t)hwin_words * 4);
    return L;
}

// LDS window layout: node q counts in the 16-bit half (q & 1) of word
// (q >> 1) W^2 + wr W + wl, (wr, wl) the cell relative to the window's corner,
// so an even and an odd node share a plane of W^2 words and the increment of
// a node known at compile time is a constant.
__device__ __forceinline__ int win_word(int q, int W, int wr, int wl) {
    return __mul24(q >> 1, W * W) + __mul24(wr, W) + wl;
}

// An increment of an LDS word, at workgroup scope.  The scope differs from
// that of the global increments (device scope), so the compiler does not join
// an LDS and a global increment on the two sides of a branch into one flat
// atomic, which counts against both memory counters: the wave's next wait for
// an LDS read would then wait for the global increment to complete.
__device__ __forceinline__ void lds_add(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// An increment of cell (q, r, l) of the overflow grid: the offset in 32 bits
// (Q nk^2 < 2^30) from the uniform base, so the address takes no 64-bit
// register pair.
__device__ __forceinline__ void extra_add(uint32_t* extra, int q, int r, int l, int nk,
                                          uint32_t v = 1u) {
    const uint32_t off = (uint32_t)(q * nk * nk + r * nk + l) << 2;
    atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(extra) + off), v);
}

// one nodal value into H^n: LDS window when inside it, else the overflow grid
template <typename T>
__device__ __forceinline__ void k1_bin(const K1Args<T>& a, const K1Lds<T>& L, const Consts<T>& c,
                                       int q, T kx, T ky) {
    const int r = cell_coord<T>(kx, c.lk, c.inv_dk);
    const int l = cell_coord<T>(ky, c.lk, c.inv_dk);
    if (r < 0 || l < 0 || r >= c.nk || l >= c.nk) {
        lds_add(&L.cnt[SGPM_CNT_OUT_OF_GRID], 1u);
        return;
    }
    const int wr = r - a.win_r0, wl = l - a.win_l0;
    if ((unsigned)wr < (unsigned)a.win && (unsigned)wl < (unsigned)a.win) {
        lds_add(&L.hwin[win_word(q, a.win, wr, wl)], (q & 1) ? 65536u : 1u);
    } else {
        extra_add(a.extra, q, r, l, c.nk);
    }
}

// Is a collision possible in this step?  ub: upper bound of every nodal
// energy after the drift.  No collision iff -log(xi) / G~ >= dt, which holds
// when -log(xi) >= t = gb dt with gb >= G~.  With u = 1 - xi, -log(xi) >=
// u + u^2/2 >= u: the particle is cleared when xi <= 1 - t (with the bound's
// margin) or when u + u^2/2, rounded, exceeds t by more than its rounding.
// The test is conservative only (a particle just inside it is listed); the
// collider decides every candidate with the exact rates, so no logarithm is
// needed here.  For xi >= 1/2, u is exact.
template <typename T>
__device__ __forceinline__ bool k1_candidate(const K1Args<T>& a, const Consts<T>& c, int64_t i, T ub,
                                             uint32_t step, T dt, uint32_t seed_lo, uint32_t seed_hi) {
    const T t = rate_bound<T>(c, ub) * dt;
    const Words wx = philox10((uint32_t)i, step, kPurXi, a.instance, seed_lo, seed_hi);
    const T xi = uni<T>(wx.w0, wx.w1);
    if (xi <= (T)1 - t * c.b_margin) return false;
    const T u = (T)1 - xi;
    return !(u + (T)0.5 * u * u >= t * ((T)1 + (T)4 * Num<T>::eps));
}

// Threads per stream workgroup of an instantiation (k1_waves); 1024 and 512
// both divide the chunk quantum kBlock1.
template <typename T, int PMAX, int QMAX>
struct K1Block {
    static constexpr int value = 64 * k1_waves(sizeof(T) == 4, PMAX, QMAX);
};

template <typename T, int PMAX, int QMAX>
__global__ void __launch_bounds__((K1Block<T, PMAX, QMAX>::value))
k1_stream(const K1Args<T>* __restrict__ all,
                                                     const uint32_t* __restrict__ wg0, int n_inst,
                                                     int moving) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int BLOCK = K1Block<T, PMAX, QMAX>::value, WAVES = BLOCK / 64;
    const int slot = find_slot(wg0, n_inst, blockIdx.x);
    const K1Args<T> a = load_desc(all, slot);
    const uint32_t wg = blockIdx.x - wg0[slot];
    const uint32_t step = a.dyn->step_k1;
    const double vfdt = a.dyn->vfdt;
    // the collider of the previous step is done with its copy of n
    if (moving && wg == 0 && threadIdx.x == 0) a.dyn->step_k2 = step;
    // the finalize kernel of this time accumulates into a cleared slot
    if (wg == 0 && (int)threadIdx.x < a.Q)
        a.excess[(size_t)(step - a.dyn->rec_base) * a.Q + threadIdx.x] = 0u;
    const T dt = (T)a.dyn->dt;
    const int P = a.P, Q = a.Q;
    const K1Lds<T> L = k1_lds<T>(smem, PMAX, QMAX > 0 ? QMAX : Q, a.hwin_words, WAVES);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int w = tid; w < (a.hwin_words >> 2); w += BLOCK)        // whole 16-byte rows
        reinterpret_cast<uint4*>(L.hwin)[w] = make_uint4(0u, 0u, 0u, 0u);
    if (tid == 0) *L.c = *a.tab.consts;
    for (int k = tid; k < Q * PMAX; k += BLOCK) {
        const int q = k / PMAX, h = k - q * PMAX;
        L.psi[k] = h < P ? a.tab.psi[q * P + h] : (T)0;
    }
    const bool strang = a.tab.consts->splitting != 0;
    for (int k = tid; k < PMAX; k += BLOCK) {
        L.psimax[k] = k < P ? a.tab.psimax[k] : (T)0;
        const T full = (moving && k < P) ? (T)(vfdt * a.ehat[k]) : (T)0;
        L.drift[k] = strang ? full * (T)0.5 : full;
        L.pdrift[k] = strang ? full * (T)0.5 : (T)0;
    }
    for (int k = tid; k < WAVES * Q * 3; k += BLOCK) L.red[k] = 0.0;
    if (tid < 16) L.cnt[tid] = 0u;
    __syncthreads();
    // node value of the drift: sum_h drift_h Psi_h(z_q)
    for (int k = tid; k < Q; k += BLOCK) {
        L.eps0sq[k] = a.tab.eps0sq[k];
        T d = (T)0;
        for (int h = 0; h < PMAX; ++h) d += L.drift[h] * L.psi[k * PMAX + h];
        L.shift[k] = d;
    }
    __syncthreads();
    const Consts<T>& c = *L.c;
    const uint32_t dmask = drift_modes<T, PMAX>(L.drift, P);
    const T lk = uniform_of(c.lk), inv_dk = uniform_of(c.inv_dk);

    const int64_t begin = (int64_t)wg * a.chunk;
    const int64_t end = begin + a.chunk < a.n ? begin + a.chunk : a.n;

    double acc[QMAX > 0 ? QMAX : 1][3];
    if constexpr (QMAX > 0) {
#pragma unroll
        for (int q = 0; q < QMAX; ++q) { acc[q][0] = 0.0; acc[q][1] = 0.0; acc[q][2] = 0.0; }
    }

    // the tiles of this workgroup's chunk; FULL: every lane of every tile holds a
    // particle (all chunks but the last), so the per-lane guards fold away
    auto tiles = [&](auto full) {
        constexpr bool FULL = decltype(full)::value;
        for (int64_t base = begin; base < end; base += BLOCK) {
            const int64_t i = base + tid;
            const bool act = FULL || i < end;
            // the node count and the key are re-read (empty asm) on every tile so
            // that the compiler does not keep the per-node tests and the key
            // schedule in scalar registers across the loop, which spills them
            int Qt = Q;
            uint32_t key_lo = a.seed_lo, key_hi = a.seed_hi;
            __asm__ volatile("" : "+s"(Qt), "+s"(key_lo), "+s"(key_hi));
            T cx[PMAX], cy[PMAX];
            load_tile_coeffs<T, PMAX>(a.kx, a.ky, a.n, P, base, act ? (uint32_t)tid : 0u, cx, cy);
            bool cand = false;
            if constexpr (QMAX > 0) {
                // the nodes of one particle
                auto nodes = [&]() -> T {
                    const bool on = act;
                    T e2max = (T)0;
                    uint32_t outmask = 0u;
    #pragma unroll
                    for (int q = 0; q < QMAX; ++q) {
                        if (q < Qt) {
                            T kx, ky;
                            eval_node<T, PMAX>(L.psi + q * PMAX, cx, cy, kx, ky);
                            // read before the histogram increment, which the compiler
                            // must otherwise assume may change them
                            const T e0sq = L.eps0sq[q], sh = L.shift[q];
                            // state at t^n: histogram and moments (Sec. 4.2)
                            const T e2 = kx * kx + ky * ky + e0sq;
                            const T rs = rsqrt_nr(e2);
                            if (on) {
                                if constexpr (sizeof(T) == 8) {
                                    // v_F applied to the lane's sums at the end
                                    acc[q][0] += kx * rs;
                                    acc[q][1] += ky * rs;
                                } else {
                                    // FP32 products summed in FP64: deterministic for
                                    // a fixed launch shape; exact (and then independent
                                    // of the chunking) only while the addends and the
                                    // running sum span at most 53 bits of exponent
                                    acc[q][0] += (double)(c.v_f * kx * rs);
                                    acc[q][1] += (double)(c.v_f * ky * rs);
                                }
                                acc[q][2] += (double)(e2 * rs);
                            }
                            {
                                // the node's cell: inside the LDS window (compared in
                                // floating point, so a NaN fails) one packed increment,
                                // else its bit in outmask for the general path below.
                                // fr, fl: the coordinates less the window's origin
                                // before the floor (see win_offset)
                                const T fr = win_offset<T>((kx + lk) * inv_dk, a.win_r0);
                                const T fl = win_offset<T>((ky + lk) * inv_dk, a.win_l0);
                                const T w = (T)a.win;
                                const bool in = (fr >= (T)0) & (fr < w) & (fl >= (T)0) & (fl < w);
                                // every lane adds (see kWinSink): no branch, so the
                                // wait for a later LDS read need not cover the add
                                lds_add((on && in)
                                              ? &L.hwin[win_word(q, a.win, (int)fr, (int)fl)]
                                              : &L.cnt[kWinSink],
                                          (q & 1) ? 65536u : 1u);
                                outmask |= (on && !in) ? (1u << q) : 0u;
                            }
                            // after the drift, for the rate bound
                            const T dx = kx - sh;
                            const T d2 = dx * dx + ky * ky + e0sq;
                            e2max = fmax(d2, e2max);   // never NaN: a NaN d2 is passed over
                        }
                    }
                    // nodes outside the window (rare): re-evaluated, general path
                    if (__ballot(outmask != 0u)) {
                        for (int q = 0; q < Q; ++q) {
                            if (outmask & (1u << q)) {
                                T kx, ky;
                                eval_node<T, PMAX>(L.psi + q * PMAX, cx, cy, kx, ky);
                                k1_bin<T>(a, L, c, q, kx, ky);
                            }
                        }
                    }
                    return e2max;
                };
                const T e2max = nodes();
                // the nodal energies after the drift, bounded with a relative
                // margin for the rounding of the shifted evaluation
                if (act && moving)
                    cand = k1_candidate<T>(a, c, i, sqrt(e2max) * c.b_margin, step, dt, key_lo, key_hi);
            } else {
                // blocks of four nodes, their twelve sums reduced over the wave together
                for (int q0 = 0; q0 < Q; q0 += 4) {
                    double v[12];
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int q = q0 + b;
                        double vx = 0.0, vy = 0.0, en = 0.0;
                        if (act && q < Q) {
                            T kx, ky;
                            eval_node<T, PMAX>(L.psi + q * PMAX, cx, cy, kx, ky);
                            const T e2 = kx * kx + ky * ky + L.eps0sq[q];
                            const T rs = rsqrt_nr(e2);
                            vx = (double)(c.v_f * kx * rs);
                            vy = (double)(c.v_f * ky * rs);
                            en = (double)(e2 * rs);
                            k1_bin<T>(a, L, c, q, kx, ky);
                        }
                        v[3 * b] = vx; v[3 * b + 1] = vy; v[3 * b + 2] = en;
                    }
                    const int nb = Q - q0 < 4 ? Q - q0 : 4;
                    wave_sums_add<12>(v, L.red + ((size_t)wave * Q + q0) * 3, 3 * nb, lane);
                }
                if (act && moving) {
                    // |k(z_q)| <= sum_h |k_h| max_q |Psi_h(z_q)| per component, after the drift
                    T bx = (T)0, by = (T)0;
    #pragma unroll
                    for (int h = 0; h < PMAX; ++h) {
                        bx += fabs(cx[h] - L.drift[h]) * L.psimax[h];
                        by += fabs(cy[h]) * L.psimax[h];
                    }
                    cand = k1_candidate<T>(a, c, i, sqrt(bx * bx + by * by + c.eps0max_sq), step, dt,
                                           key_lo, key_hi);
                }
            }
            if (act && moving && !cand) {
                // the particle does not collide: its step is the drift alone.  The
                // lane offset is passed through an empty asm statement so that the
                // per-mode store addresses are formed here, not kept for the whole
                // loop in registers (which would spill them).
                uint32_t t = (uint32_t)tid;
                __asm__ volatile("" : "+v"(t));
    #pragma unroll
                for (int h = 0; h < PMAX; ++h)
                    if ((dmask >> h) & 1u)
                        (a.kx + ((size_t)h * a.n + base))[t] = (cx[h] - L.drift[h]) - L.pdrift[h];
            }
            // candidates of this workgroup collected in LDS
            const uint64_t mask = __ballot(cand);
            if (mask) {
                uint32_t base_slot = 0;
                if (lane == 0) base_slot = atomicAdd(&L.cnt[SGPM_CNT_CANDIDATES], (uint32_t)__popcll(mask));
                base_slot = __shfl(base_slot, 0, 64);
                if (cand) {
                    const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
                        (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                    L.cbuf[base_slot + pos] = (int)i;
                }
            }
        }
    };
    if (end - begin == a.chunk) tiles(std::true_type{});
    else tiles(std::false_type{});
    if constexpr (QMAX > 0) {
        double v[3 * QMAX];
        const double vf = sizeof(T) == 8 ? (double)L.c->v_f : 1.0;
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            v[3 * q] = vf * acc[q][0]; v[3 * q + 1] = vf * acc[q][1]; v[3 * q + 2] = acc[q][2];
        }
        wave_sums_add<3 * QMAX>(v, L.red + (size_t)wave * Q * 3, 3 * Q, lane);
    }
    __syncthreads();

    // this workgroup's candidates appended to the global list (one reservation)
    {
        __shared__ uint32_t gbase;
        const uint32_t nc = L.cnt[SGPM_CNT_CANDIDATES];
        if (nc) {
            if (tid == 0) gbase = atomicAdd(a.qc + 2 * (step & 1), nc);
            __syncthreads();
            for (uint32_t k = tid; k < nc; k += BLOCK) a.cand[gbase + k] = L.cbuf[k];
        }
    }

    // the LDS window as this workgroup's dense slab (plain 16-byte stores)
    {
        uint32_t* slab = a.slabs + (size_t)wg * a.hwin_words;
        const int nv = a.hwin_words >> 2;
        for (int w = tid; w < nv; w += BLOCK)
            reinterpret_cast<uint4*>(slab)[w] = reinterpret_cast<const uint4*>(L.hwin)[w];
    }
    // this workgroup's moment sums, waves in order
    for (int k = tid; k < Q * 3; k += BLOCK) {
        double v = 0.0;
        for (int wv = 0; wv < WAVES; ++wv) v += L.red[wv * Q * 3 + k];
        a.partial[(size_t)wg * Q * 3 + k] = v;
    }
    if (tid < 8 && L.cnt[tid]) atomicAdd(&a.counters[tid], (unsigned long long)L.cnt[tid]);
}

// ============================================ K1 with mirror node pairs
// For one uncertain input the Gauss-Legendre nodes are symmetric,
// z_{Q-1-q} = -z_q, and the orthonormal Legendre basis has the parity
// Psi_h(-z) = (-1)^h Psi_h(z), exactly in the tables.  With E and O the sums
// of the even and of the odd modes at z_q, k(z_q) = E + O and
// k(z_{Q-1-q}) = E - O: the two nodes of a pair cost the products of one
// (eq. gPC evaluated at both nodes).  A lane per particle, as in k1_stream,
// but with fewer instructions per node: the pairs, the collision bound from
// the nodal energies before the drift plus the largest nodal drift
// (|k - d| <= |k| + |d|), and candidate lists flushed to the global list by
// each wave as they fill, so that a workgroup's chunk is not limited by its
// LDS.  The workgroup owns a whole compute unit (three or four waves per
// SIMD), and with it nearly all of the LDS for the histogram window.
//
// Counts of the mirror-pair window above thr (a workgroup's counts, between
// two segments of its chunk) moved to the overflow grid, the same cells of
// H^n.  Plane p holds node p in its low and node Q-1-p in its high half (the
// high half of an odd Q's middle plane stays empty).  Not inlined: it runs
// at most once per 65535 particles of a workgroup, and inlined it costs the
// tile loop registers.
__device__ __attribute__((noinline)) void win_spill(uint32_t* hwin, uint32_t* extra, int Q,
                                                    int W, int r0, int l0, int nk, uint32_t thr,
                                                    int tid, int nthreads) {
    const int WW = W * W, words = ((Q + 1) >> 1) * WW;
    for (int k = tid; k < words; k += nthreads) {
        const uint32_t v = hwin[k];
        const uint32_t lo = v & 0xFFFFu, hi = v >> 16;
        if (lo > thr || hi > thr) {
            const int p = k / WW, wr = (k - p * WW) / W, wl = k - p * WW - wr * W;
            uint32_t keep = v;
            if (lo > thr) { extra_add(extra, p, r0 + wr, l0 + wl, nk, lo); keep -= lo; }
            if (hi > thr) { extra_add(extra, Q - 1 - p, r0 + wr, l0 + wl, nk, hi); keep -= hi << 16; }
            hwin[k] = keep;
        }
    }
}

// LDS window of this kernel: pair p in plane p, node p in the low and node
// Q-1-p in the high 16 bits of a word, the middle node of an odd Q in the low
// bits of plane (Q-1)/2.  The finalize kernel decodes it by the instance's
// mirror flag.
// VGPRs of the kernel, estimated: the FP64 moment sums a lane keeps (one node
// of every pair, and the middle node), the coefficients and the temporaries,
// fitted to the compiler's output (at 9 modes and 12 nodes FP64 takes 155, so
// three waves per SIMD; 16 modes take more per mode than the others)
__host__ __device__ constexpr int k1p_regs(int fp32, int pmax, int qmax) {
    return 2 * (3 * (qmax / 2) + 3) + pmax * (fp32 ? 2 : 5) + (fp32 ? 60 : 66) +
           (pmax >= 16 ? (fp32 ? 6 : 14) : 0);
}
// Threads per workgroup of an instantiation: the default, four, three or two
// waves per SIMD by the estimate, and (alt) the other occupancy the autotuner
// may pick, 512 for 768 and 768 for the others (where the default would spill
// or one more wave per SIMD may hide more latency)
__host__ __device__ constexpr int k1p_block_of(int fp32, int pmax, int qmax, int alt) {
    const int r = k1p_regs(fp32, pmax, qmax);
    const int b = r <= 128 ? 1024 : (r <= 168 ? 768 : 512);
    return alt ? (b == 768 ? 512 : 768) : b;
}
int k1p_block(int fp32, int pmax, int qmax, int alt) { return k1p_block_of(fp32, pmax, qmax, alt); }
template <typename T, int PMAX, int QMAX, int ALT>
struct K1PBlock {
    static constexpr int value = k1p_block_of(sizeof(T) == 4, PMAX, QMAX, ALT);
};

// Wave sums of V per-lane values; store(k, s) receives the sum s of v[k] over
// the wave, from one lane per k (the scheme of wave_sums_add).
template <int V, typename F>
__device__ __forceinline__ void wave_sums_map(const double (&v)[V], int lane, F&& store) {
    constexpr int VP = (V + 3) & ~3, H2 = VP / 2, H4 = VP / 4;
    double u[H2];
#pragma unroll
    for (int j = 0; j < H2; ++j) {
        double a = v[j], b = j + H2 < V ? v[j + H2] : 0.0;
        swap32_f64(a, b);
        u[j] = a + b;
    }
    double w[H4];
#pragma unroll
    for (int j = 0; j < H4; ++j) {
        double a = u[j], b = u[j + H4];
        swap16_f64(a, b);
        w[j] = a + b;
    }
#pragma unroll
    for (int j = 0; j < H4; ++j) {
        double x = w[j];
        x += dpp_f64<0xB1>(x);
        x += dpp_f64<0x4E>(x);
        x += dpp_f64<0x141>(x);
        x += dpp_f64<0x140>(x);
        w[j] = x;
    }
    if ((lane & 15) == 0) {
        const int r = lane >> 4, base = H4 * (r & 1) + H2 * (r >> 1);
#pragma unroll
        for (int j = 0; j < H4; ++j)
            if (base + j < V) store(base + j, w[j]);
    }
}

// NT: non-temporal state access (see load_tile_coeffs)
template <typename T, int PMAX, int QMAX, int ALT, int NT>
__global__ void __launch_bounds__((K1PBlock<T, PMAX, QMAX, ALT>::value))
k1_pairs(const K1Args<T>* __restrict__ all, const uint32_t* __restrict__ wg0, int n_inst,
         int moving) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int BLOCK = K1PBlock<T, PMAX, QMAX, ALT>::value, WAVES = BLOCK / 64;
    constexpr int NP = QMAX / 2;            // pair slots
    __shared__ T s_shmax;
    const int slot = find_slot(wg0, n_inst, blockIdx.x);
    const K1Args<T> a = load_desc(all, slot);
    const uint32_t wg = blockIdx.x - wg0[slot];
    const uint32_t step = a.dyn->step_k1;
    const double vfdt = a.dyn->vfdt;
    if (moving && wg == 0 && threadIdx.x == 0) a.dyn->step_k2 = step;
    if (wg == 0 && (int)threadIdx.x < a.Q)
        a.excess[(size_t)(step - a.dyn->rec_base) * a.Q + threadIdx.x] = 0u;
    const T dt = (T)a.dyn->dt;
    const int P = a.P, Q = a.Q;
    const K1Lds<T> L = k1_lds<T>(smem, PMAX, QMAX, a.hwin_words, WAVES);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int w = tid; w < (a.hwin_words >> 2); w += BLOCK)
        reinterpret_cast<uint4*>(L.hwin)[w] = make_uint4(0u, 0u, 0u, 0u);
    if (tid == 0) *L.c = *a.tab.consts;
    for (int k = tid; k < Q * PMAX; k += BLOCK) {
        const int q = k / PMAX, h = k - q * PMAX;
        L.psi[k] = h < P ? a.tab.psi[q * P + h] : (T)0;
    }
    const bool strang = a.tab.consts->splitting != 0;
    for (int k = tid; k < PMAX; k += BLOCK) {
        L.psimax[k] = k < P ? a.tab.psimax[k] : (T)0;
        const T full = (moving && k < P) ? (T)(vfdt * a.ehat[k]) : (T)0;
        L.drift[k] = strang ? full * (T)0.5 : full;
        L.pdrift[k] = strang ? full * (T)0.5 : (T)0;
    }
    for (int k = tid; k < WAVES * Q * 3; k += BLOCK) L.red[k] = 0.0;
    if (tid < 16) L.cnt[tid] = 0u;
    __syncthreads();
    // eps0^2 by pairs: node p at 2p, node Q-1-p at 2p+1, the middle node of an
    // odd Q last, so that a lane reads its node of pair p at 2p plus its parity
    for (int k = tid; k < Q; k += BLOCK) {
        const int half = Q >> 1;
        L.eps0sq[k < half ? 2 * k : (k >= Q - half ? 2 * (Q - 1 - k) + 1 : 2 * half)] =
            a.tab.eps0sq[k];
        T d = (T)0;
        for (int h = 0; h < PMAX; ++h) d += L.drift[h] * L.psi[k * PMAX + h];
        L.shift[k] = d;
    }
    __syncthreads();
    if (tid == 0) {
        T m = (T)0;
        for (int q = 0; q < Q; ++q) m = fmax(m, fabs(L.shift[q]));
        s_shmax = m;
    }
    __syncthreads();
    const Consts<T>& c = *L.c;
    const T shmax = s_shmax;
    const uint32_t dmask = drift_modes<T, PMAX>(L.drift, P);
    const T lk = uniform_of(c.lk), inv_dk = uniform_of(c.inv_dk);
    const int64_t begin = (int64_t)wg * a.chunk;
    const int64_t end = begin + a.chunk < a.n ? begin + a.chunk : a.n;
    const int W = a.win;
    int* seg = L.cbuf + wave * kK1PSeg;      // this wave's candidates
    uint32_t nseg = 0;                       // wave-uniform

    // The moment sums of the pairs are split between the two lanes of each
    // lane pair: the even lane keeps those of node p of every pair for both
    // particles, the odd lane those of node Q-1-p.  That halves the registers
    // they take (with them the kernel fits three waves per SIMD).  Each lane
    // evaluates the node it keeps first and hands the other's terms to its
    // partner.
    const bool odd_lane = (lane & 1) != 0;
    double acc[NP][3], accm[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int p = 0; p < NP; ++p) { acc[p][0] = 0.0; acc[p][1] = 0.0; acc[p][2] = 0.0; }

    // this wave's list into the global one (one reservation)
    auto flush = [&]() {
        uint32_t gb = 0;
        if (lane == 0) gb = atomicAdd(a.qc + 2 * (step & 1), nseg);
        gb = __shfl(gb, 0, 64);
        wave_lds_fence();
        for (uint32_t k = lane; k < nseg; k += 64) a.cand[gb + k] = seg[k];
        wave_lds_fence();
        nseg = 0;
    };

    auto tile = [&](int64_t base, auto full) {
        constexpr bool FULL = decltype(full)::value;
        const int64_t i = base + tid;
        const bool act = FULL || i < end;
        // re-read on every tile (empty asm): see k1_stream
        int Qt = Q;
        uint32_t key_lo = a.seed_lo, key_hi = a.seed_hi;
        __asm__ volatile("" : "+s"(Qt), "+s"(key_lo), "+s"(key_hi));
        const int npairs = Qt >> 1;
        T cx[PMAX], cy[PMAX];
        load_tile_coeffs<T, PMAX, NT != 0>(a.kx, a.ky, a.n, P, base, act ? (uint32_t)tid : 0u,
                                           cx, cy);
        T e2max = (T)0;
        uint32_t outmask = 0u;
        // one nodal value of the state at t^n: window and moment sums
        // t: the node's moment terms (zero for a lane past the end)
        // e0sq: the node's eps0^2 (read before the pair's first increment);
        // j: its half of the window word (0 for node p, 1 for Q-1-p)
        auto node = [&](T e0sq, int plane, int j, T kx, T ky, double (&t)[3], int bit) {
            const T e2 = kx * kx + ky * ky + e0sq;
            const T rs = rsqrt_nr(e2);
            if constexpr (sizeof(T) == 8) {
                t[0] = act ? (double)(kx * rs) : 0.0;    // v_F applied to the sums at the end
                t[1] = act ? (double)(ky * rs) : 0.0;
            } else {
                t[0] = act ? (double)(c.v_f * kx * rs) : 0.0;
                t[1] = act ? (double)(c.v_f * ky * rs) : 0.0;
            }
            t[2] = act ? (double)(e2 * rs) : 0.0;
            const T fr = win_offset<T>((kx + lk) * inv_dk, a.win_r0);
            const T fl = win_offset<T>((ky + lk) * inv_dk, a.win_l0);
            const T w = (T)W;
            const bool in = (fr >= (T)0) & (fr < w) & (fl >= (T)0) & (fl < w);
            // every lane adds (see kWinSink): no branch, so the wait for a
            // later LDS read need not cover the add
            lds_add((act && in) ? &L.hwin[__mul24(plane, W * W) + __mul24((int)fr, W) + (int)fl]
                                  : &L.cnt[kWinSink],
                      j ? 65536u : 1u);
            outmask |= (act && !in) ? (1u << bit) : 0u;
            e2max = fmax(e2, e2max);    // a NaN e2 is passed over
        };
        // the even and odd sums of pair p
        auto eo = [&](int p, T& ex, T& ox, T& ey, T& oy) {
            const T* row = L.psi + p * PMAX;
            ex = (T)0; ox = (T)0; ey = (T)0; oy = (T)0;
#pragma unroll
            for (int h = 0; h < PMAX; h += 2) { ex += cx[h] * row[h]; ey += cy[h] * row[h]; }
#pragma unroll
            for (int h = 1; h < PMAX; h += 2) { ox += cx[h] * row[h]; oy += cy[h] * row[h]; }
        };
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            if (p < npairs) {
                T ex, ox, ey, oy;
                eo(p, ex, ox, ey, oy);
                // node a (kept: p on an even lane, Q-1-p on an odd one) and
                // node b (handed over); sg * ox is exact, so k(a) and k(b) are
                // E + O and E - O rounded as written
                const int ja = odd_lane ? 1 : 0;
                const T sg = odd_lane ? (T)-1 : (T)1;
                double ta[3], tb[3];
                const T e0a = L.eps0sq[2 * p + ja], e0b = L.eps0sq[2 * p + 1 - ja];
                node(e0a, p, ja, ex + sg * ox, ey + sg * oy, ta, 2 * p + ja);
                node(e0b, p, 1 - ja, ex - sg * ox, ey - sg * oy, tb, 2 * p + 1 - ja);
                // the partner's terms of the node this lane keeps (the exchange
                // with every lane active)
#pragma unroll
                for (int m = 0; m < 3; ++m) acc[p][m] += ta[m] + dpp_f64<0xB1>(tb[m]);
            }
            // one pair after the other: overlapping them buys little with three
            // or four waves per SIMD and costs the registers of another wave
            __builtin_amdgcn_sched_barrier(0);
        }
        if (Qt & 1) {
            T ex, ox, ey, oy;
            eo(npairs, ex, ox, ey, oy);
            double t[3];
            node(L.eps0sq[2 * npairs], npairs, 0, ex + ox, ey + oy, t, 2 * NP);
            accm[0] += t[0]; accm[1] += t[1]; accm[2] += t[2];
        }
        // nodes outside the window (rare): the same values again, into the
        // overflow grid or counted outside the grid
        if (__ballot(outmask != 0u)) {
            for (int b = 0; b <= 2 * NP; ++b) {
                if (!(outmask & (1u << b))) continue;
                const int p = b < 2 * NP ? (b >> 1) : npairs;
                const int j = b < 2 * NP ? (b & 1) : 0;
                T ex, ox, ey, oy;
                eo(p, ex, ox, ey, oy);
                const T kx = j ? ex - ox : ex + ox, ky = j ? ey - oy : ey + oy;
                const int q = j ? Qt - 1 - p : p;
                const int r = cell_coord<T>(kx, lk, inv_dk);
                const int l = cell_coord<T>(ky, lk, inv_dk);
                if (r < 0 || l < 0 || r >= c.nk || l >= c.nk)
                    lds_add(&L.cnt[SGPM_CNT_OUT_OF_GRID], 1u);
                else
                    extra_add(a.extra, q, r, l, c.nk);
            }
        }
        // after the drift every nodal wave-vector moves by at most shmax, so
        // sqrt(max e2) + shmax bounds every nodal energy (|k - d| <= |k| + |d|)
        bool cand = false;
        if (act && moving)
            cand = k1_candidate<T>(a, c, i, (sqrt(e2max) + shmax) * c.b_margin, step, dt,
                                   key_lo, key_hi);
        if (act && moving && !cand) {
            uint32_t tt = (uint32_t)tid;
            __asm__ volatile("" : "+v"(tt));
#pragma unroll
            for (int h = 0; h < PMAX; ++h)
                if ((dmask >> h) & 1u)
                    store_state<NT != 0>((a.kx + ((size_t)h * a.n + base)) + tt,
                                         (cx[h] - L.drift[h]) - L.pdrift[h]);
        }
        const uint64_t mask = __ballot(cand);
        if (mask) {
            const uint32_t nnew = (uint32_t)__popcll(mask);
            if (lane == 0) atomicAdd(&L.cnt[SGPM_CNT_CANDIDATES], nnew);
            if (cand) {
                const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
                seg[nseg + pos] = (int)i;
            }
            nseg += nnew;
            if (nseg > (uint32_t)(kK1PSeg - 64)) flush();
        }
    };
    // A 16-bit count of the window holds 65535, and a particle adds at most one
    // to each: a chunk longer than that is taken in segments of SEG particles,
    // and between two segments the counts that the next one could carry past
    // 65535 move to the overflow grid (win_spill).
    constexpr int64_t SEG = (int64_t)(65535 / BLOCK) * BLOCK;
    int64_t base = begin, next = begin + SEG;
    for (; base + BLOCK <= end; base += BLOCK) {
        if (base == next) {
            __syncthreads();
            win_spill(L.hwin, a.extra, Q, W, a.win_r0, a.win_l0, c.nk,
                      65535u - (uint32_t)(end - base < SEG ? end - base : SEG), tid, BLOCK);
            __syncthreads();
            next += SEG;
        }
        tile(base, std::true_type{});
    }
    if (base < end) {
        if (base == next) {
            __syncthreads();
            win_spill(L.hwin, a.extra, Q, W, a.win_r0, a.win_l0, c.nk,
                      65535u - (uint32_t)(end - base), tid, BLOCK);
            __syncthreads();
        }
        tile(base, std::false_type{});
    }
    // the waves' remaining candidates with one reservation for the workgroup
    // (waves ending together would otherwise queue on the list's counter)
    {
        __shared__ uint32_t s_n[WAVES + 1];
        if (lane == 0) s_n[wave] = nseg;
        __syncthreads();
        if (tid == 0) {
            uint32_t tot = 0;
            for (int w = 0; w < WAVES; ++w) { const uint32_t v = s_n[w]; s_n[w] = tot; tot += v; }
            s_n[WAVES] = tot ? atomicAdd(a.qc + 2 * (step & 1), tot) : 0u;
        }
        __syncthreads();
        const uint32_t gb = s_n[WAVES] + s_n[wave];
        for (uint32_t k = lane; k < nseg; k += 64) a.cand[gb + k] = seg[k];
    }
    {
        constexpr int V = 6 * NP + 3;
        double v[V];
        const double vf = sizeof(T) == 8 ? (double)c.v_f : 1.0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const bool mine = odd_lane == (j == 1);
                v[(2 * p + j) * 3] = mine ? vf * acc[p][0] : 0.0;
                v[(2 * p + j) * 3 + 1] = mine ? vf * acc[p][1] : 0.0;
                v[(2 * p + j) * 3 + 2] = mine ? acc[p][2] : 0.0;
            }
        }
        v[6 * NP] = vf * accm[0]; v[6 * NP + 1] = vf * accm[1]; v[6 * NP + 2] = accm[2];
        const int npairs = Q >> 1;
        double* red = L.red + (size_t)wave * Q * 3;
        wave_sums_map<V>(v, lane, [&](int k, double sum) {
            const int m = k % 3, b = k / 3;
            if (b < 2 * NP) {
                const int p = b >> 1;
                if (p < npairs) red[((b & 1) ? Q - 1 - p : p) * 3 + m] = sum;
            } else if (Q & 1) {
                red[npairs * 3 + m] = sum;
            }
        });
    }
    __syncthreads();
    {
        uint32_t* slab = a.slabs + (size_t)wg * a.hwin_words;
        const int nv = a.hwin_words >> 2;
        for (int w = tid; w < nv; w += BLOCK)
            reinterpret_cast<uint4*>(slab)[w] = reinterpret_cast<const uint4*>(L.hwin)[w];
    }
    for (int k = tid; k < Q * 3; k += BLOCK) {
        double v = 0.0;
        for (int wv = 0; wv < WAVES; ++wv) v += L.red[wv * Q * 3 + k];
        a.partial[(size_t)wg * Q * 3 + k] = v;
    }
    if (tid < 8 && L.cnt[tid]) atomicAdd(&a.counters[tid], (unsigned long long)L.cnt[tid]);
}

// ===================================================== K2: collider kernel
// lanes per candidate of the collider: one node per lane, at most a wave
__host__ __device__ __forceinline__ int k2_group_width(int Q) {
    int G = 1;
    while (G < Q && G < 64) G <<= 1;
    return G;
}

size_t k2_lds_bytes(int P, int Q, int fp32) {
    const size_t s = fp32 ? 4 : 8;
    const int PM = pmax_bucket(P);
    const int groups = kBlock / k2_group_width(Q);
    size_t off = sizeof(Consts<double>);
    off = (off + 15) & ~(size_t)15;
    off += s * (2 * (size_t)Q * PM + 4 * (size_t)Q + 32 + 2 * PM);   // psi wpsi eps0 eps0sq cedge vfield ecos drift pdrift
    off = (off + 15) & ~(size_t)15;
    off += s * (size_t)groups * (2 * (size_t)Q + 2 * PM);         // per-group projection scratch
    off = (off + 15) & ~(size_t)15;
    off += 16 * 4;                       // counters
    return off;
}

template <typename T>
struct K2Lds {
    Consts<T>* c;
    T* psi; T* wpsi; T* eps0; T* eps0sq; T* cedge; T* vfield; T* ecos;
    T* drift;            // applied before the collisions (dt, or dt/2 with Strang)
    T* pdrift;           // applied after them (0, or dt/2 with Strang)
    T* scratch;          // [groups][2Q + 2PM]: new node values, then new modes
    uint32_t* cnt;
};

template <typename T>
__device__ __forceinline__ K2Lds<T> k2_lds(unsigned char* smem, int PM, int Q, int groups) {
    K2Lds<T> L;
    size_t off = 0;
    L.c = reinterpret_cast<Consts<T>*>(smem);
    off = sizeof(Consts<double>);
    off = (off + 15) & ~(size_t)15;
    L.psi = reinterpret_cast<T*>(smem + off);
    L.wpsi = L.psi + Q * PM;
    L.eps0 = L.wpsi + Q * PM;
    L.eps0sq = L.eps0 + Q;
    L.cedge = L.eps0sq + Q;
    L.vfield = L.cedge + Q;
    L.ecos = L.vfield + Q;
    L.drift = L.ecos + 32;
    L.pdrift = L.drift + PM;
    off += sizeof(T) * (2 * (size_t)Q * PM + 4 * (size_t)Q + 32 + 2 * PM);
    off = (off + 15) & ~(size_t)15;
    L.scratch = reinterpret_cast<T*>(smem + off);
    off += sizeof(T) * (size_t)groups * (2 * (size_t)Q + 2 * PM);
    off = (off + 15) & ~(size_t)15;
    L.cnt = reinterpret_cast<uint32_t*>(smem + off);
    return L;
}

// Comparisons with a rounded quotient c / g (c >= 0, g > 0, s > 0) decided by
// the product s g against c where that is safe: a product outside c (1 -+ 2 eps)
// (four units of rounding) lies on the same side of c as the exact s g, and the
// rounded quotient lies within one unit of the exact one, so the comparison with
// the rounded quotient comes out the same.  Inside the margin (rare) the
// quotient is formed.  A division costs about a dozen dependent instructions.
template <typename T>
__device__ __forceinline__ bool lt_quot(T s, T c, T g) {   // s < c / g
    const T p = s * g;
    if (p < c * ((T)1 - (T)2 * Num<T>::eps)) return true;
    if (p > c * ((T)1 + (T)2 * Num<T>::eps)) return false;
    return s < c / g;
}
template <typename T>
__device__ __forceinline__ bool quot_lt(T c, T g, T s) {   // c / g < s
    const T p = s * g;
    if (p > c * ((T)1 + (T)2 * Num<T>::eps)) return true;
    if (p < c * ((T)1 - (T)2 * Num<T>::eps)) return false;
    return c / g < s;
}

// Pauli acceptance: is the occupation f = H^n / max H^n of node q at the
// candidate's cell, on the grid moved with this step's drift (lookup at
// k' + v_F E(z_q) dt x^), below eta?  f = 0 for an empty histogram and off
// the grid.
template <typename T>
__device__ __forceinline__ bool pauli_accepts(const uint32_t* __restrict__ h_read,
                                              const uint32_t* __restrict__ hmax_read,
                                              const K2Lds<T>& L, const Consts<T>& c, int q, T px,
                                              T py, T dt, T eta) {
    const uint32_t mx = hmax_read[q];
    if (mx == 0u) return true;
    const T shift = L.vfield[q] * dt;
    const int r = cell_coord<T>(px + shift, c.lk, c.inv_dk);
    const int l = cell_coord<T>(py, c.lk, c.inv_dk);
    if (r < 0 || l < 0 || r >= c.nk || l >= c.nk) return true;
    const uint32_t h = h_read[(size_t)q * c.nk * c.nk + (size_t)r * c.nk + l];
    return quot_lt<T>((T)h, (T)mx, eta);
}


// The candidates of one instance in passes of kBlock / G candidates: this
// workgroup takes the passes first, first + stride, ... below the instance's
// pass count (the list is complete when the kernel starts, so a static share
// needs no work counter); total: the list's length.  A group of G
// lanes serves one candidate, lane g holding nodes g and g + G (NPL = 2 only
// when Q > 64).  Per collision every node's rates are evaluated once: their
// running sums give both Gamma~ (eq. gamma_tot) and the mechanism selection.
template <typename T, int PMAX, int NPL>
__device__ __forceinline__ void k2_instance(const K2Args<T>& a, unsigned char* smem, uint32_t step,
                                            uint32_t total, uint32_t first, uint32_t stride) {
    const int P = a.P, Q = a.Q, G = a.G;
    const K2Lds<T> L = k2_lds<T>(smem, PMAX, Q, kBlock / G);
    const int tid = threadIdx.x;
    const T dt = (T)a.dyn->dt;
    const double vfdt = a.dyn->vfdt;
    const uint32_t* h_read = a.H + (size_t)(step % 3u) * a.hstride;
    const uint32_t* hmax_read = a.Hmax + (size_t)(step % 3u) * a.hmstride;
    const int g = tid % G;                // rank in the group = node handled
    const int grp = tid / G;
    const uint32_t per_pass = kBlock / G;
    // the first pass's candidate and its coefficients (drift not yet applied),
    // fetched while the tables are staged
    const T zero[PMAX] = {};
    const uint32_t cid0 = first * per_pass + grp;
    int64_t i = 0;
    T cx[PMAX] = {}, cy[PMAX] = {};
    if (cid0 < total) {
        i = a.cand[cid0];
        load_coeffs<T, PMAX>(a.kx, a.ky, a.n, P, i, zero, cx, cy);
    }

    if (tid == 0) *L.c = *a.tab.consts;
    for (int k = tid; k < Q * PMAX; k += kBlock) {
        const int q = k / PMAX, h = k - q * PMAX;
        L.psi[k] = h < P ? a.tab.psi[q * P + h] : (T)0;
        L.wpsi[k] = h < P ? a.tab.wpsi[q * P + h] : (T)0;
    }
    for (int k = tid; k < Q; k += kBlock) {
        L.eps0[k] = a.tab.eps0[k]; L.eps0sq[k] = a.tab.eps0sq[k];
        L.cedge[k] = a.tab.cedge[k]; L.vfield[k] = a.tab.vfield[k];
    }
    for (int k = tid; k <= kEdgePts / 2; k += kBlock) L.ecos[k] = a.tab.edge_cos[k];
    const bool strang = a.tab.consts->splitting != 0;
    for (int k = tid; k < PMAX; k += kBlock) {
        const T full = k < P ? (T)(vfdt * a.ehat[k]) : (T)0;
        L.drift[k] = strang ? full * (T)0.5 : full;
        L.pdrift[k] = strang ? full * (T)0.5 : (T)0;
    }
    if (tid < 16) L.cnt[tid] = 0u;
    __syncthreads();
    const Consts<T>& c = *L.c;
    // the grid of H^n moved with the drift applied before the collisions
    const T dt_grid = strang ? dt * (T)0.5 : dt;

    T* nodes = L.scratch + (size_t)grp * (2 * Q + 2 * PMAX);   // [2][Q] new node values
    T* modes = nodes + 2 * Q;                                   // [2][PMAX] new coefficients

#pragma unroll
    for (int h = 0; h < PMAX; ++h) cx[h] -= L.drift[h];   // zero past P on both sides
    for (uint32_t p0 = first * per_pass; p0 < total; p0 += stride * per_pass) {
        const uint32_t cid = p0 + grp;
        if (cid >= total) continue;
        if (cid != cid0) {
            i = a.cand[cid];
            load_coeffs<T, PMAX>(a.kx, a.ky, a.n, P, i, L.drift, cx, cy);
        }
        T tc = (T)0;
        uint32_t coll = 0;
        const uint32_t ctr0 = (uint32_t)i;
        for (;;) {
            // node values and running rate sums AC, OP-, OP+, K-, K+, edge;
            // Gamma~ = (1 + alpha) max over the nodes of the total
            T nkx[NPL], nky[NPL], ne[NPL], cum[NPL][6];
            T smax = (T)0;
#pragma unroll
            for (int j = 0; j < NPL; ++j) {
                const int q = g + j * G;
                if (q < Q) {
                    eval_node<T, PMAX>(L.psi + q * PMAX, cx, cy, nkx[j], nky[j]);
                    ne[j] = sqrt(nkx[j] * nkx[j] + nky[j] * nky[j] + L.eps0sq[q]);
                    T r[5];
                    phonon_rates<T>(c, ne[j], L.eps0[q], r);
                    T run = (T)0;
#pragma unroll
                    for (int m = 0; m < 5; ++m) { run += r[m]; cum[j][m] = run; }
                    // first an upper bound of the edge rate: every trapezoid
                    // term is at most 1, so the integral is at most 2 pi
                    run += (ne[j] - L.eps0[q] >= (T)0)
                               ? L.cedge[q] * ne[j] * ((T)kEdgePts * Num<T>::trap) : (T)0;
                    smax = run > smax ? run : smax;
                }
            }
            smax = group_max<T>(smax, G);
            const Words wx = k2_draw<T>(ctr0, step, (coll << 8) | kPurXi, a.instance, a.seed_lo,
                                      a.seed_hi);
            const T lxi = -dlog(uni<T>(wx.w0, wx.w1));
            // A flight that ends past the step under the bound of Gamma~ ends
            // past it under Gamma~: the bound's sums, maximum, product and the
            // division are each monotone in rounding, and the margin covers a
            // different rounding of the exact sum.  So the decision is the one
            // of the exact rates, and the edge integral (17 exponentials per
            // node) is evaluated only when the flight may end inside the step.
            if (!(tc + lxi / (c.alpha1 * smax * ((T)1 + (T)16 * Num<T>::eps)) < dt)) break;
            smax = (T)0;
#pragma unroll
            for (int j = 0; j < NPL; ++j) {
                const int q = g + j * G;
                if (q < Q) {
                    const T run = cum[j][4] + edge_rate<T>(c, L.ecos, L.cedge[q], L.eps0[q],
                                                           nkx[j], nky[j], ne[j]);
                    cum[j][5] = run;
                    smax = run > smax ? run : smax;
                }
            }
            smax = group_max<T>(smax, G);
            const T Gt = c.alpha1 * smax;
            const T dtc = lxi / Gt;   // eq. dt, node maximum
            if (!(tc + dtc < dt)) break;
            if (g == 0) atomicAdd(&L.cnt[SGPM_CNT_COLLISIONS], 1u);

            const Words ws = k2_draw<T>(ctr0, step, (coll << 8) | kPurSel, a.instance, a.seed_lo,
                                      a.seed_hi);
            const T su = uni<T>(ws.w0, ws.w1), eta = uni<T>(ws.w2, ws.w3);
            const Words wa = k2_draw<T>(ctr0, step, (coll << 8) | kPurAng, a.instance, a.seed_lo,
                                      a.seed_hi);
            const T u1 = uni<T>(wa.w0, wa.w1), u2 = uni<T>(wa.w2, wa.w3);
            // AC angle: twice the polar angle of a uniform point of the unit
            // disk centred at (1,0) (density 1 + cos), by the double angle
            T s_phi, c_phi;
            dsincospi((T)2 * u2, &s_phi, &c_phi);
            const T rr = sqrt(u1);
            const T dx = (T)1 + rr * c_phi, dy = rr * s_phi;
            const T n2 = dx * dx + dy * dy;
            const T cac = (dx * dx - dy * dy) / n2, sac = ((T)2 * dx * dy) / n2;
            T sop, cop;
            dsincospi((T)2 * u1, &sop, &cop);    // OP angle 2 pi u1

            uint32_t nev = 0, nrej = 0, nexh = 0;
#pragma unroll
            for (int j = 0; j < NPL; ++j) {
                const int q = g + j * G;
                if (q >= Q) continue;
                const T kx = nkx[j], ky = nky[j], e = ne[j];
                const T e0 = L.eps0[q];
                // mechanism l: the first with s < G^l_q / Gamma~, else self (7)
                int ell = 7;
#pragma unroll
                for (int m = 5; m >= 0; --m)
                    if (lt_quot<T>(su, cum[j][m], Gt)) ell = m + 1;
                T nx = kx, ny = ky;
                if (ell != 7) {
                    const T kabs = sqrt(kx * kx + ky * ky);
                    const T cin = kabs > (T)0 ? kx / kabs : (T)1;
                    const T sin_ = kabs > (T)0 ? ky / kabs : (T)0;
                    T px = kx, py = ky;
                    bool ok = true;
                    if (ell == 6) {
                        // absolute final angle, density exp(-kap (cos t' - cos t_in)^2)
                        const T kap = c.edge_kap * (kx * kx + ky * ky);
                        ok = false;
                        for (uint32_t jt = 0; jt < (uint32_t)kEdgeTries; ++jt) {
                            const Words we = k2_draw<T>(ctr0, step, (coll << 8) | (kPurEdge0 + jt),
                                                      a.instance, a.seed_lo, a.seed_hi);
                            const T ut = uni<T>(we.w0, we.w1), v = uni<T>(we.w2, we.w3);
                            T st, ct;
                            dsincospi((T)2 * ut, &st, &ct);
                            const T d = ct - cin;
                            if (v < dexp(-kap * d * d)) {
                                px = kabs * ct; py = kabs * st;
                                ok = true;
                                break;
                            }
                        }
                        if (!ok) ++nexh;
                    } else {
                        T ct, st, mag;
                        if (ell == 1) { ct = cac; st = sac; mag = kabs; }
                        else {
                            const bool op = (ell == 2 || ell == 3);
                            const T hw = op ? c.hw_o : c.hw_k;
                            const T de = (ell == 2 || ell == 4) ? -hw : hw;
                            if (op) { ct = cop; st = sop; } else { ct = -cac; st = -sac; }
                            if (c.final_state == 1) {
                                mag = kabs + de;
                            } else {
                                const T e1 = e + de;     // energy-conserving final state
                                mag = sqrt((e1 - e0) * (e1 + e0));
                            }
                        }
                        px = mag * (ct * cin - st * sin_);
                        py = mag * (st * cin + ct * sin_);
                    }
                    if (ok) {
                        ++nev;
                        if (!c.pauli ||
                            pauli_accepts<T>(h_read, hmax_read, L, c, q, px, py, dt_grid, eta)) {
                            nx = px; ny = py;
                        } else {
                            ++nrej;
                        }
                    }
                }
                nodes[q] = nx;
                nodes[Q + q] = ny;
            }
            if (nev) atomicAdd(&L.cnt[SGPM_CNT_EVENTS], nev);
            if (nrej) atomicAdd(&L.cnt[SGPM_CNT_PAULI_REJ], nrej);
            if (nexh) atomicAdd(&L.cnt[SGPM_CNT_EDGE_EXH], nexh);
            // k_h = sum_q w_q Psi_h(z_q) k_q, summed over q in order by lane h,
            // then read back by every lane of the group
            wave_lds_fence();
            for (int h = g; h < P; h += G) {
                T sx = (T)0, sy = (T)0;
                for (int q = 0; q < Q; ++q) {
                    const T w = L.wpsi[q * PMAX + h];
                    sx += w * nodes[q];
                    sy += w * nodes[Q + q];
                }
                modes[h] = sx;
                modes[PMAX + h] = sy;
            }
            wave_lds_fence();
#pragma unroll
            for (int h = 0; h < PMAX; ++h) {
                cx[h] = h < P ? modes[h] : (T)0;
                cy[h] = h < P ? modes[PMAX + h] : (T)0;
            }
            wave_lds_fence();
            tc += dtc;
            ++coll;
            if (coll >= (uint32_t)c.c_max) {
                if (g == 0) atomicAdd(&L.cnt[SGPM_CNT_CMAX], 1u);
                break;
            }
        }
        // the collided modes back into the state: scattered stores of one value
        // per line, non-temporal, so they are not allocated in the caches
        // (which costs a tenth of the lane collider's time at 3e7 particles)
#pragma unroll
        for (int h = 0; h < PMAX; ++h)
            if (h < P && (h % G) == g) {
                __builtin_nontemporal_store(cx[h] - L.pdrift[h], &a.kx[(size_t)h * a.n + i]);
                __builtin_nontemporal_store(cy[h], &a.ky[(size_t)h * a.n + i]);
            }
    }
    // every lane is past its last candidate: the counters are complete
    __syncthreads();
    if (tid < 8 && L.cnt[tid]) atomicAdd(&a.counters[tid], (unsigned long long)L.cnt[tid]);
    __syncthreads();
}

// ------------------------------------------ K2 with a lane per candidate
// For at most 12 nodes a lane takes a whole candidate and loops over its
// nodes, and a wave serves 64 candidates at once.  The draws, logarithm and
// angles of a collision are then computed once per candidate instead of on
// every lane of a node group, no lane idles for want of a node, and many more
// candidates are in flight to hide the latency of their loads.  Every
// quantity is computed by the same expressions as in k2_instance, sums over
// the modes and the projection's sums over the nodes in the same order, and
// the node maxima are exact, so the results are the same bit for bit.  The
// exact rates of an iteration (the 17 exponentials of every node's edge
// integral dominate the kernel) are evaluated as (candidate, node) pairs dealt
// out over the whole wave, a pair per lane, from the candidates' modes staged
// in LDS: the wave evaluates about as many integrals as its candidates need,
// not Q whenever any lane needs them.  The node totals wait in LDS (a column
// per lane) for the pass that takes their maximum and selects the mechanisms.
// The first edge proposal of a collision, shared by all of its nodes, is
// drawn once and kept.
// LDS of the lanes: the node totals [Q][kBlock], the coefficients of the
// candidates whose exact rates are evaluated [kBlock][2 PMAX] and the lanes of
// those candidates [kBlock], in the layout of k2_lds: as many of its per-group
// scratch blocks (2 Q + 2 PMAX values each) as they take
__host__ __device__ constexpr int k2l_groups(int Q, int PM) {
    return (Q + 2 * PM + 1) * kBlock / (2 * Q + 2 * PM) + 1;
}
size_t k2l_lds_bytes(int P, int Q, int fp32) {
    const size_t s = fp32 ? 4 : 8;
    const int PM = pmax_bucket(P);
    size_t off = sizeof(Consts<double>);
    off = (off + 15) & ~(size_t)15;
    off += s * (2 * (size_t)Q * PM + 4 * (size_t)Q + 32 + 2 * PM);
    off = (off + 15) & ~(size_t)15;
    off += s * (size_t)k2l_groups(Q, PM) * (2 * (size_t)Q + 2 * PM);
    off = (off + 15) & ~(size_t)15;
    off += 16 * 4;                                 // counters
    return off;
}

// deal: null to take the passes first, first + stride, ... of kBlock
// candidates; else a counter (zero at the launch) from which each wave takes
// its next 64 candidates as it finishes the last, so that waves whose
// candidates collide more often do not hold up the end of the launch
template <typename T, int PMAX>
__device__ __forceinline__ void k2_lanes_instance(const K2Args<T>& a, unsigned char* smem,
                                                  uint32_t step, uint32_t total, uint32_t first,
                                                  uint32_t stride, uint32_t* deal) {
    const int P = a.P, Q = a.Q;
    // tables as in k2_instance; the per-group scratch holds the edge rates
    const K2Lds<T> L = k2_lds<T>(smem, PMAX, Q, k2l_groups(Q, PMAX));
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    T* tot = L.scratch;                            // [Q][kBlock] node totals of the rates
    T* wcoef = tot + (size_t)Q * kBlock + (size_t)wave * 64 * 2 * PMAX;   // [64][2 PMAX]
    int* wslot = reinterpret_cast<int*>(tot + (size_t)Q * kBlock + (size_t)kBlock * 2 * PMAX) +
                 wave * 64;                        // [64]
    const T dt = (T)a.dyn->dt;
    const double vfdt = a.dyn->vfdt;
    const uint32_t* h_read = a.H + (size_t)(step % 3u) * a.hstride;
    const uint32_t* hmax_read = a.Hmax + (size_t)(step % 3u) * a.hmstride;
    if (tid == 0) *L.c = *a.tab.consts;
    for (int k = tid; k < Q * PMAX; k += kBlock) {
        const int q = k / PMAX, h = k - q * PMAX;
        L.psi[k] = h < P ? a.tab.psi[q * P + h] : (T)0;
        L.wpsi[k] = h < P ? a.tab.wpsi[q * P + h] : (T)0;
    }
    for (int k = tid; k < Q; k += kBlock) {
        L.eps0[k] = a.tab.eps0[k]; L.eps0sq[k] = a.tab.eps0sq[k];
        L.cedge[k] = a.tab.cedge[k]; L.vfield[k] = a.tab.vfield[k];
    }
    for (int k = tid; k <= kEdgePts / 2; k += kBlock) L.ecos[k] = a.tab.edge_cos[k];
    const bool strang = a.tab.consts->splitting != 0;
    for (int k = tid; k < PMAX; k += kBlock) {
        const T full = k < P ? (T)(vfdt * a.ehat[k]) : (T)0;
        L.drift[k] = strang ? full * (T)0.5 : full;
        L.pdrift[k] = strang ? full * (T)0.5 : (T)0;
    }
    if (tid < 16) L.cnt[tid] = 0u;
    __syncthreads();
    const Consts<T>& c = *L.c;
    const T dt_grid = strang ? dt * (T)0.5 : dt;
    uint32_t n_coll = 0, n_ev = 0, n_rej = 0, n_exh = 0, n_cmax = 0;

    auto take = [&]() -> uint32_t {
        uint32_t b = 0;
        if (lane == 0) b = atomicAdd(deal, 64u);
        return __shfl(b, 0, 64);
    };
    for (uint32_t p0 = deal ? take() : first * kBlock + wave * 64; p0 < total;
         p0 = deal ? take() : p0 + stride * kBlock) {
        const uint32_t cid = p0 + lane;
        bool live = cid < total;
        int64_t i = 0;
        T cx[PMAX], cy[PMAX];
#pragma unroll
        for (int h = 0; h < PMAX; ++h) { cx[h] = (T)0; cy[h] = (T)0; }
        if (live) {
            i = a.cand[cid];
            load_coeffs<T, PMAX>(a.kx, a.ky, a.n, P, i, L.drift, cx, cy);
        }
        T tc = (T)0;
        uint32_t coll = 0;
        const uint32_t ctr0 = (uint32_t)i;
        // The first part of a collision iteration of this lane's candidate:
        // node values, phonon rates and a bound of Gamma~ (the edge integral
        // is at most 2 pi), as in k2_instance, and the free flight under the
        // bound.  True if the flight may end inside the step (the exact rates
        // are needed); lxi = -log(xi).
        auto bound_test = [&](T& lxi) -> bool {
            const Words wx = k2_draw<T>(ctr0, step, (coll << 8) | kPurXi, a.instance, a.seed_lo,
                                        a.seed_hi);
            lxi = -dlog(uni<T>(wx.w0, wx.w1));
            // The first iteration's draw is the one the stream kernel tested
            // against its own bound to list this candidate, and nearly every
            // candidate collides then: the exact rates are evaluated at once
            // (the bound only filters; the exact test decides either way).
            if (coll == 0) return true;
            T sb = (T)0;
            for (int q = 0; q < Q; ++q) {
                T kx, ky;
                eval_node<T, PMAX>(L.psi + q * PMAX, cx, cy, kx, ky);
                const T ne = sqrt(kx * kx + ky * ky + L.eps0sq[q]);
                T r[5];
                phonon_rates<T>(c, ne, L.eps0[q], r);
                T run = (T)0;
#pragma unroll
                for (int m = 0; m < 5; ++m) run += r[m];
                run += (ne - L.eps0[q] >= (T)0)
                           ? L.cedge[q] * ne * ((T)kEdgePts * Num<T>::trap) : (T)0;
                sb = run > sb ? run : sb;
            }
            return tc + lxi / (c.alpha1 * sb * ((T)1 + (T)16 * Num<T>::eps)) < dt;
        };
        // The rest of the iteration, after the exact node totals are in tot:
        // the exact free flight and, if it ends inside the step, the collision
        // and projection.  False ends the candidate.
        auto collide = [&](T lxi) -> bool {
            T smax = (T)0;
            for (int q = 0; q < Q; ++q) {
                const T run = tot[q * kBlock + tid];
                smax = run > smax ? run : smax;
            }
            const T Gt = c.alpha1 * smax;
            const T dtc = lxi / Gt;   // eq. dt, node maximum
            if (!(tc + dtc < dt)) return false;
            ++n_coll;
            const Words ws = k2_draw<T>(ctr0, step, (coll << 8) | kPurSel, a.instance, a.seed_lo,
                                        a.seed_hi);
            const T su = uni<T>(ws.w0, ws.w1), eta = uni<T>(ws.w2, ws.w3);
            const Words wa = k2_draw<T>(ctr0, step, (coll << 8) | kPurAng, a.instance, a.seed_lo,
                                        a.seed_hi);
            const T u1 = uni<T>(wa.w0, wa.w1), u2 = uni<T>(wa.w2, wa.w3);
            T s_phi, c_phi;
            dsincospi((T)2 * u2, &s_phi, &c_phi);
            const T rr = sqrt(u1);
            const T dx = (T)1 + rr * c_phi, dy = rr * s_phi;
            const T n2 = dx * dx + dy * dy;
            const T cac = (dx * dx - dy * dy) / n2, sac = ((T)2 * dx * dy) / n2;
            T sop, cop;
            dsincospi((T)2 * u1, &sop, &cop);    // OP angle 2 pi u1
            bool have0 = false;                   // the first edge proposal, drawn once
            T st0 = (T)0, ct0 = (T)0, v0 = (T)0;
            T ax[PMAX], ay[PMAX];
#pragma unroll
            for (int h = 0; h < PMAX; ++h) { ax[h] = (T)0; ay[h] = (T)0; }
            for (int q = 0; q < Q; ++q) {
                T kx, ky;
                eval_node<T, PMAX>(L.psi + q * PMAX, cx, cy, kx, ky);
                const T e = sqrt(kx * kx + ky * ky + L.eps0sq[q]);
                const T e0 = L.eps0[q];
                T r[5], cum[6];
                phonon_rates<T>(c, e, e0, r);
                T run = (T)0;
#pragma unroll
                for (int m = 0; m < 5; ++m) { run += r[m]; cum[m] = run; }
                cum[5] = tot[q * kBlock + tid];   // cum[4] + the edge rate, as summed above
                int ell = 7;
#pragma unroll
                for (int m = 5; m >= 0; --m)
                    if (lt_quot<T>(su, cum[m], Gt)) ell = m + 1;
                T nx = kx, ny = ky;
                if (ell != 7) {
                    const T kabs = sqrt(kx * kx + ky * ky);
                    const T cin = kabs > (T)0 ? kx / kabs : (T)1;
                    const T sin_ = kabs > (T)0 ? ky / kabs : (T)0;
                    T px = kx, py = ky;
                    bool ok = true;
                    if (ell == 6) {
                        const T kap = c.edge_kap * (kx * kx + ky * ky);
                        if (!have0) {
                            const Words we = k2_draw<T>(ctr0, step, (coll << 8) | kPurEdge0,
                                                        a.instance, a.seed_lo, a.seed_hi);
                            const T ut = uni<T>(we.w0, we.w1);
                            v0 = uni<T>(we.w2, we.w3);
                            dsincospi((T)2 * ut, &st0, &ct0);
                            have0 = true;
                        }
                        const T d0 = ct0 - cin;
                        ok = v0 < dexp(-kap * d0 * d0);
                        if (ok) { px = kabs * ct0; py = kabs * st0; }
                        for (uint32_t jt = 1; !ok && jt < (uint32_t)kEdgeTries; ++jt) {
                            const Words we = k2_draw<T>(ctr0, step, (coll << 8) | (kPurEdge0 + jt),
                                                        a.instance, a.seed_lo, a.seed_hi);
                            const T ut = uni<T>(we.w0, we.w1), v = uni<T>(we.w2, we.w3);
                            T st, ct;
                            dsincospi((T)2 * ut, &st, &ct);
                            const T d = ct - cin;
                            if (v < dexp(-kap * d * d)) {
                                px = kabs * ct; py = kabs * st;
                                ok = true;
                            }
                        }
                        if (!ok) ++n_exh;
                    } else {
                        T ct, st, mag;
                        if (ell == 1) { ct = cac; st = sac; mag = kabs; }
                        else {
                            const bool op = (ell == 2 || ell == 3);
                            const T hw = op ? c.hw_o : c.hw_k;
                            const T de = (ell == 2 || ell == 4) ? -hw : hw;
                            if (op) { ct = cop; st = sop; } else { ct = -cac; st = -sac; }
                            if (c.final_state == 1) {
                                mag = kabs + de;
                            } else {
                                const T e1 = e + de;     // energy-conserving final state
                                mag = sqrt((e1 - e0) * (e1 + e0));
                            }
                        }
                        px = mag * (ct * cin - st * sin_);
                        py = mag * (st * cin + ct * sin_);
                    }
                    if (ok) {
                        ++n_ev;
                        if (!c.pauli ||
                            pauli_accepts<T>(h_read, hmax_read, L, c, q, px, py, dt_grid, eta)) {
                            nx = px; ny = py;
                        } else {
                            ++n_rej;
                        }
                    }
                }
                // k_h = sum_q w_q Psi_h(z_q) k_q, summed over the nodes in order
#pragma unroll
                for (int h = 0; h < PMAX; ++h) {
                    ax[h] += L.wpsi[q * PMAX + h] * nx;
                    ay[h] += L.wpsi[q * PMAX + h] * ny;
                }
            }
#pragma unroll
            for (int h = 0; h < PMAX; ++h) {
                cx[h] = h < P ? ax[h] : (T)0;
                cy[h] = h < P ? ay[h] : (T)0;
            }
            tc += dtc;
            ++coll;
            if (coll >= (uint32_t)c.c_max) { ++n_cmax; return false; }
            return true;
        };
        while (__ballot(live)) {
            T lxi = (T)0;
            bool exact = false;
            if (live) {
                exact = bound_test(lxi);
                live = exact;
            }
            // exact rates, the edge integral of every node: the (candidate,
            // node) pairs of the lanes that need them are dealt out over the
            // whole wave, a pair per lane, so the wave evaluates about as many
            // integrals as are needed rather than Q whenever one lane needs any
            const uint64_t need = __ballot(exact);
            if (!need) continue;
            if (exact) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
                wslot[rank] = lane;
#pragma unroll
                for (int h = 0; h < PMAX; ++h) {
                    wcoef[lane * 2 * PMAX + h] = cx[h];
                    wcoef[lane * 2 * PMAX + PMAX + h] = cy[h];
                }
            }
            wave_lds_fence();
            const uint32_t items = (uint32_t)__popcll(need) * (uint32_t)Q;
            for (uint32_t t = (uint32_t)lane; t < items; t += 64) {
                const uint32_t o = t / (uint32_t)Q;
                const int q = (int)(t - o * (uint32_t)Q);
                const int own = wslot[o];
                const T* oc = wcoef + own * 2 * PMAX;
                const T* row = L.psi + q * PMAX;
                // the node value as eval_node forms it from the owner's modes
                T kx = (T)0, ky = (T)0;
#pragma unroll
                for (int h = 0; h < PMAX; ++h) { kx += oc[h] * row[h]; ky += oc[PMAX + h] * row[h]; }
                const T ne = sqrt(kx * kx + ky * ky + L.eps0sq[q]);
                T r[5];
                phonon_rates<T>(c, ne, L.eps0[q], r);
                T run = (T)0;
#pragma unroll
                for (int m = 0; m < 5; ++m) run += r[m];
                const T e = edge_rate<T>(c, L.ecos, L.cedge[q], L.eps0[q], kx, ky, ne);
                tot[q * kBlock + wave * 64 + own] = run + e;
            }
            wave_lds_fence();
            if (exact) live = collide(lxi);
        }
        if (cid < total) {
#pragma unroll
            for (int h = 0; h < PMAX; ++h)
                if (h < P) {
                    // non-temporal: see k2_instance
                    __builtin_nontemporal_store(cx[h] - L.pdrift[h], &a.kx[(size_t)h * a.n + i]);
                    __builtin_nontemporal_store(cy[h], &a.ky[(size_t)h * a.n + i]);
                }
        }
    }
    if (n_coll) atomicAdd(&L.cnt[SGPM_CNT_COLLISIONS], n_coll);
    if (n_ev) atomicAdd(&L.cnt[SGPM_CNT_EVENTS], n_ev);
    if (n_rej) atomicAdd(&L.cnt[SGPM_CNT_PAULI_REJ], n_rej);
    if (n_exh) atomicAdd(&L.cnt[SGPM_CNT_EDGE_EXH], n_exh);
    if (n_cmax) atomicAdd(&L.cnt[SGPM_CNT_CMAX], n_cmax);
    __syncthreads();
    if (tid < 8 && L.cnt[tid]) atomicAdd(&a.counters[tid], (unsigned long long)L.cnt[tid]);
    __syncthreads();
}

// Collider grid of a group.  The passes of all instances, concatenated in
// instance order, are dealt out round-robin.  Workgroup 0 advances the
// finalize kernel's copy of the step of every instance (that kernel is done).
template <typename T, int PMAX, int NPL, bool LANES>
__device__ __forceinline__ void k2_run(const K2Args<T>& a, unsigned char* smem, uint32_t step,
                                       uint32_t total, uint32_t first, uint32_t stride) {
    if constexpr (LANES) k2_lanes_instance<T, PMAX>(a, smem, step, total, first, stride, nullptr);
    else k2_instance<T, PMAX, NPL>(a, smem, step, total, first, stride);
}

template <typename T, int PMAX, int NPL, bool LANES = false>
__device__ __forceinline__ void k2_body(const K2Args<T>* __restrict__ all, int n_inst) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int kPer = (SGPM_MAX_INSTANCES + kBlock - 1) / kBlock;   // instances per thread
    __shared__ uint32_t s_base[SGPM_MAX_INSTANCES + 1];   // first global pass of instance j
    __shared__ uint32_t s_scan[kBlock];
    __shared__ uint32_t s_list[SGPM_MAX_INSTANCES];   // instances holding a pass of this workgroup
    __shared__ uint32_t s_nlist;
    typedef const __attribute__((address_space(4))) K2Args<T> CA;
    const uint32_t grid = gridDim.x;
    const int tid = threadIdx.x;
    if (n_inst == 1) {
        // one instance: its passes b, b + grid, ... are this workgroup's
        const K2Args<T> a = load_desc(all, 0);
        const uint32_t step = a.dyn->step_k2;
        const uint32_t total = a.qc[2 * (step & 1u)];
        if (blockIdx.x == 0 && tid == 0) a.dyn->step_k3 = step + 1u;   // the finalize kernel is done
        const uint32_t per_pass = (uint32_t)(kBlock / a.G);
        if constexpr (LANES) {
            // the waves take their candidates from the spare word of the
            // step's counters, cleared by the last finalize kernel
            if (blockIdx.x < (total + per_pass - 1) / per_pass)
                k2_lanes_instance<T, PMAX>(a, smem, step, total, 0, grid,
                                           a.qc + 2 * (step & 1u) + 1);
        } else if (blockIdx.x < (total + per_pass - 1) / per_pass) {
            k2_run<T, PMAX, NPL, LANES>(a, smem, step, total, blockIdx.x, grid);
        }
        return;
    }
    // every instance's step, list length and pass count, read in parallel
    uint32_t loc[kPer];
    uint32_t sum = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int j = tid * kPer + u;
        uint32_t passes = 0;
        if (j < n_inst) {
            Dyn* dyn = ((CA*)all)[j].dyn;
            const uint32_t step = dyn->step_k2;
            const uint32_t total = ((CA*)all)[j].qc[2 * (step & 1u)];
            const uint32_t per_pass = (uint32_t)(kBlock / ((CA*)all)[j].G);
            passes = (total + per_pass - 1) / per_pass;
            if (blockIdx.x == 0) dyn->step_k3 = step + 1u;   // the finalize kernel is done
        }
        loc[u] = passes;
        sum += passes;
    }
    // exclusive prefix sums of the pass counts (instances concatenated in order)
    s_scan[tid] = sum;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        const uint32_t v = tid >= off ? s_scan[tid - off] : 0u;
        __syncthreads();
        s_scan[tid] += v;
        __syncthreads();
    }
    uint32_t run = s_scan[tid] - sum;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int j = tid * kPer + u;
        if (j < n_inst) s_base[j] = run;
        run += loc[u];
    }
    if (tid == 0) {
        s_base[n_inst] = s_scan[kBlock - 1];
        s_nlist = 0u;
    }
    __syncthreads();
    // The global passes b, b + grid, ... of the concatenation belong to this
    // workgroup (b = blockIdx.x), so a group of many small lists spreads like
    // one long list.  Its first pass in instance j is r = (b - base_j) mod grid;
    // the instances where that pass exists are listed in parallel (in any order:
    // the instances share nothing but this workgroup's LDS, restaged for each).
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int j = tid * kPer + u;
        if (j < n_inst) {
            const uint32_t base = s_base[j], passes = s_base[j + 1] - base;
            const uint32_t r = (blockIdx.x + grid - base % grid) % grid;
            if (r < passes) s_list[atomicAdd(&s_nlist, 1u)] = (uint32_t)j;
        }
    }
    __syncthreads();
    const uint32_t nlist = s_nlist;
    for (uint32_t t = 0; t < nlist; ++t) {
        const int j = (int)s_list[t];
        const uint32_t r = (blockIdx.x + grid - s_base[j] % grid) % grid;
        const K2Args<T> a = load_desc(all, j);
        // the step and list length read again (neither changes while the
        // collider runs), which keeps the static LDS small
        const uint32_t step = a.dyn->step_k2;
        k2_run<T, PMAX, NPL, LANES>(a, smem, step, a.qc[2 * (step & 1u)], r, grid);
    }
}

// Compiled for three waves per SIMD (at most 168 VGPRs, so three workgroups
// share a compute unit, which the throughput of the collisions depends on)
// where that costs at most a few spilled registers: FP32, and FP64 up to six
// modes with one node per lane.  The others keep their registers (wide).
template <typename T, int PMAX, int NPL>
struct K2Narrow {
    static constexpr bool value = sizeof(T) == 4 || (PMAX <= 6 && NPL == 1);
};

template <typename T, int PMAX, int NPL>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
k2_collide(const K2Args<T>* __restrict__ all, int n_inst) {
    k2_body<T, PMAX, NPL>(all, n_inst);
}

template <typename T, int PMAX, int NPL>
__global__ void __launch_bounds__(kBlock) k2_collide_wide(const K2Args<T>* __restrict__ all,
                                                          int n_inst) {
    k2_body<T, PMAX, NPL>(all, n_inst);
}

// a lane per candidate (at most 12 nodes).  Held to two waves per SIMD: the
// FP64 forms otherwise take a few registers past 256 and run one wave per SIMD,
// a third slower; three waves would spill hundreds of bytes per lane.
template <typename T, int PMAX>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
k2_lanes(const K2Args<T>* __restrict__ all, int n_inst) {
    k2_body<T, PMAX, 1, true>(all, n_inst);
}

// ===================================================== K3: finalize kernel
// Node counted in half hi of window plane p, or -1 if that half is unused:
// two consecutive nodes per plane, or (mirror) node p low and Q-1-p high.
__device__ __forceinline__ int win_node(int mirror, int Q, int p, int hi) {
    if (mirror) {
        if (hi) return p < (Q >> 1) ? Q - 1 - p : -1;
        return p < ((Q + 1) >> 1) ? p : -1;
    }
    const int q = 2 * p + hi;
    return q < Q ? q : -1;
}

// Workgroups [0, n_win_wg): kK3Words window words each (two cells per word),
// every slab summed, plus the overflow count, into H^n.  Workgroups after
// that: kK3Rest cells of the rest of the grid (overflow count only).  Every
// workgroup zeroes the overflow cells it read and contributes its maximum;
// workgroup (q + Q b) also reduces moment batch b of node q.
__global__ void __launch_bounds__(kBlock) k3_finalize(const K3Args* __restrict__ all,
                                                      const uint32_t* __restrict__ wg0, int n_inst,
                                                      int moving) {
    const int slot = find_slot(wg0, n_inst, blockIdx.x);
    const K3Args a = load_desc(all, slot);
    const int wg = (int)(blockIdx.x - wg0[slot]);
    const uint32_t step = a.dyn->step_k3;
    // the stream kernel of this step is done with its copy of n
    if (moving && wg == 0 && threadIdx.x == 0) a.dyn->step_k1 = step + 1u;
    const int nwg = a.nwg, nb = a.nb;
    const double* partial = a.partial;
    // one record slot per time, kNumBatches batches wide whatever the launch
    // shape, so a change of shape never moves the slots of other times
    double* record = a.record + (size_t)(step - a.dyn->rec_base) * kNumBatches * a.Q * 3;
    uint32_t* h_out = a.H + (size_t)(step % 3u) * a.hstride;
    uint32_t* hmax_out = a.Hmax + (size_t)(step % 3u) * a.hmstride;
    const int tid = threadIdx.x;
    const int cells = a.nk * a.nk;
    const int wcells = a.win * a.win;
    const int wwords = (a.Q + 1) / 2 * wcells;   // window words in use (planes of wcells)
    __shared__ uint32_t part[kK3Lanes][kK3Words][2];
    __shared__ uint32_t smax[kMaxQ];
    __shared__ uint32_t scap[kMaxQ], sex[kMaxQ];
    for (int k = tid; k < a.Q; k += kBlock) { smax[k] = 0u; scap[k] = a.cap[k]; sex[k] = 0u; }
    __syncthreads();
    if (nwg <= kK3Direct && wg < a.n_win_wg) {
        // few slabs: a thread sums its four words of every slab itself, then
        // settles its eight cells, their overflow counts loaded together
        const int word0 = (wg * kBlock + tid) * 4;
        if (word0 < a.hwin_words) {
            uint32_t lo[4] = {0u, 0u, 0u, 0u}, hi[4] = {0u, 0u, 0u, 0u};
            const uint32_t* src = a.slabs + word0;
#pragma unroll 4
            for (int sl = 0; sl < nwg; ++sl) {
                const uint4 v = *reinterpret_cast<const uint4*>(src + (size_t)sl * a.hwin_words);
                lo[0] += v.x & 0xFFFFu; hi[0] += v.x >> 16;
                lo[1] += v.y & 0xFFFFu; hi[1] += v.y >> 16;
                lo[2] += v.z & 0xFFFFu; hi[2] += v.z >> 16;
                lo[3] += v.w & 0xFFFFu; hi[3] += v.w >> 16;
            }
            size_t gc[8];
            int qc[8];
            uint32_t ex[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                // half k & 1 of word k >> 1 of the thread's four: node 2 p + (k & 1)
                // of plane p (the window layout of win_word)
                const int word = word0 + (k >> 1);
                const int p = word / wcells, rem = word - p * wcells;
                const int q = win_node(a.mirror, a.Q, p, k & 1);
                const bool ok = word < wwords && q >= 0;
                const int r = a.win_r0 + rem / a.win, l = a.win_l0 + rem % a.win;
                qc[k] = ok ? q : -1;
                gc[k] = ok ? (size_t)q * cells + (size_t)r * a.nk + l : 0;
                ex[k] = ok ? a.extra[gc[k]] : 0u;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (qc[k] < 0) continue;
                const uint32_t sum = ((k & 1) ? hi[k >> 1] : lo[k >> 1]) + ex[k];
                a.extra[gc[k]] = 0u;
                h_out[gc[k]] = sum;
                if (sum) atomicMax(&smax[qc[k]], sum);
                if (sum > scap[qc[k]]) atomicAdd(&sex[qc[k]], sum - scap[qc[k]]);
            }
        }
    }
    // many slabs: window blocks wg * fold, ..., wg * fold + fold - 1, the slabs
    // split over kK3Lanes lanes and summed through LDS
    for (int blk = 0; nwg > kK3Direct && wg < a.n_win_wg && blk < a.fold; ++blk) {
        const int wb = wg * a.fold + blk;
        // 16 columns of four words, kK3Lanes slab lanes; 16-byte loads
        const int col = tid % (kK3Words / 4);
        const int lane = tid / (kK3Words / 4);
        const int word0 = wb * kK3Words + 4 * col;
        // the overflow count of the cell this thread settles below, loaded
        // together with the slabs (each cell is settled by one thread only)
        size_t g_set = 0;
        int q_set = -1;
        uint32_t ex_set = 0u;
        if (tid < 2 * kK3Words) {
            // half tid & 1 of the block's word tid >> 1 (the window layout of win_word)
            const int word = wb * kK3Words + (tid >> 1);
            const int p = word / wcells, rem = word - p * wcells;
            const int q = win_node(a.mirror, a.Q, p, tid & 1);
            if (word < wwords && q >= 0) {
                q_set = q;
                const int r = a.win_r0 + rem / a.win, l = a.win_l0 + rem % a.win;
                g_set = (size_t)q_set * cells + (size_t)r * a.nk + l;
                ex_set = a.extra[g_set];
            }
        }
        uint32_t lo[4] = {0u, 0u, 0u, 0u}, hi[4] = {0u, 0u, 0u, 0u};
        if (word0 < a.hwin_words) {
            const uint32_t* src = a.slabs + word0;
#pragma unroll 4
            for (int s = lane; s < nwg; s += kK3Lanes) {
                const uint4 v = *reinterpret_cast<const uint4*>(src + (size_t)s * a.hwin_words);
                lo[0] += v.x & 0xFFFFu; hi[0] += v.x >> 16;
                lo[1] += v.y & 0xFFFFu; hi[1] += v.y >> 16;
                lo[2] += v.z & 0xFFFFu; hi[2] += v.z >> 16;
                lo[3] += v.w & 0xFFFFu; hi[3] += v.w >> 16;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) { part[lane][4 * col + j][0] = lo[j]; part[lane][4 * col + j][1] = hi[j]; }
        __syncthreads();
        if (q_set >= 0) {
            const int wl = tid >> 1, half = tid & 1;
            uint32_t sum = ex_set;
#pragma unroll
            for (int k = 0; k < kK3Lanes; ++k) sum += part[k][wl][half];
            a.extra[g_set] = 0u;
            h_out[g_set] = sum;
            if (sum) atomicMax(&smax[q_set], sum);
            if (sum > scap[q_set]) atomicAdd(&sex[q_set], sum - scap[q_set]);
        }
        __syncthreads();   // part[] is rewritten by the next block
    }
    if (wg >= a.n_win_wg) {
        // kK3Rest cells outside the window, kK3Rest / kBlock per thread, their
        // overflow counts loaded together
        constexpr int kPer = kK3Rest / kBlock;
        const int64_t c0 = (int64_t)(wg - a.n_win_wg) * kK3Rest;
        const int64_t total = (int64_t)a.Q * cells;
        int qc[kPer];
        uint32_t v[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int64_t g = c0 + tid + (int64_t)u * kBlock;
            const int q = g < total ? (int)(g / cells) : 0;
            const int rem = (int)(g - (int64_t)q * cells);
            const int r = rem / a.nk, l = rem - r * a.nk;
            const int wr = r - a.win_r0, wl = l - a.win_l0;
            const bool inwin = (unsigned)wr < (unsigned)a.win && (unsigned)wl < (unsigned)a.win;
            qc[u] = (g < total && !inwin) ? q : -1;
            v[u] = qc[u] >= 0 ? a.extra[g] : 0u;
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            if (qc[u] < 0) continue;
            const int64_t g = c0 + tid + (int64_t)u * kBlock;
            a.extra[g] = 0u;
            h_out[g] = v[u];
            if (v[u]) atomicMax(&smax[qc[u]], v[u]);
            if (v[u] > scap[qc[u]]) atomicAdd(&sex[qc[u]], v[u] - scap[qc[u]]);
        }
    }
    __syncthreads();
    for (int k = tid; k < a.Q; k += kBlock)
        if (smax[k]) atomicMax(&hmax_out[k], smax[k]);
    // particles above the maximum occupation number at this time (Pauli violation)
    for (int k = tid; k < a.Q; k += kBlock)
        if (sex[k]) atomicAdd(&a.excess[(size_t)(step - a.dyn->rec_base) * a.Q + k], sex[k]);
    if (wg == 0) {
        // stale maximum slot of step n + 1 and the counters of that step
        uint32_t* hmax_clr = a.Hmax + (size_t)((step + 1u) % 3u) * a.hmstride;
        for (int k = tid; k < a.Q; k += kBlock) hmax_clr[k] = 0u;
        if (tid < 2) a.qc[2 * ((step + 1u) & 1u) + tid] = 0u;
    }
    // moment record: batch b of node q collects the stream workgroups w = b (mod NB),
    // one wave, lane j taking w = b + j nb, b + (j + 64) nb, ...; then a fixed tree
    if (wg < a.Q * nb && tid < 64) {
        const int q = wg % a.Q, b = wg / a.Q;
        double v0 = 0.0, v1 = 0.0, v2 = 0.0;
        for (int w = b + tid * nb; w < nwg; w += 64 * nb) {
            const double* pw = partial + ((size_t)w * a.Q + q) * 3;
            v0 += pw[0]; v1 += pw[1]; v2 += pw[2];
        }
        v0 = wave_sum(v0); v1 = wave_sum(v1); v2 = wave_sum(v2);
        if (tid == 0) {
            double* r = record + ((size_t)b * a.Q + q) * 3;
            r[0] = v0; r[1] = v1; r[2] = v2;
        }
    }
}

// ------------------------------------------------------------ launchers
int qmax_bucket(int Q) {
    if (Q <= 1) return 1;
    if (Q <= 8) return 8;
    if (Q <= 12) return 12;
    return 0;
}

template <typename T, int PMAX, int QMAX>
static int launch_k1_t(const void* args, const uint32_t* wg0, int n_inst, int moving, unsigned grid,
                       size_t lds, void* stream) {
    hipLaunchKernelGGL((k1_stream<T, PMAX, QMAX>), dim3(grid), dim3(K1Block<T, PMAX, QMAX>::value), lds,
                       (hipStream_t)stream, static_cast<const K1Args<T>*>(args), wg0, n_inst,
                       moving);
    return (int)hipGetLastError();
}

template <typename T, int PMAX>
static int launch_k1_q(int qmax, const void* args, const uint32_t* wg0, int n_inst, int moving,
                       unsigned grid, size_t lds, void* stream) {
    switch (qmax) {
    case 1: return launch_k1_t<T, PMAX, 1>(args, wg0, n_inst, moving, grid, lds, stream);
    case 8: return launch_k1_t<T, PMAX, 8>(args, wg0, n_inst, moving, grid, lds, stream);
    case 12: return launch_k1_t<T, PMAX, 12>(args, wg0, n_inst, moving, grid, lds, stream);
    default: return launch_k1_t<T, PMAX, 0>(args, wg0, n_inst, moving, grid, lds, stream);
    }
}

template <typename T>
static int launch_k1_any(int pmax, int qmax, const void* args, const uint32_t* wg0, int n_inst,
                         int moving, unsigned grid, size_t lds, void* stream) {
    switch (pmax) {
    case 1: return launch_k1_q<T, 1>(qmax, args, wg0, n_inst, moving, grid, lds, stream);
    case 3: return launch_k1_q<T, 3>(qmax, args, wg0, n_inst, moving, grid, lds, stream);
    case 6: return launch_k1_q<T, 6>(qmax, args, wg0, n_inst, moving, grid, lds, stream);
    case 9: return launch_k1_q<T, 9>(qmax, args, wg0, n_inst, moving, grid, lds, stream);
    case 16: return launch_k1_q<T, 16>(qmax, args, wg0, n_inst, moving, grid, lds, stream);
    default: return launch_k1_q<T, 32>(qmax, args, wg0, n_inst, moving, grid, lds, stream);
    }
}

template <typename T, int PMAX, int QMAX, int ALT, int NT>
static void launch_k1p_f(const void* args, const uint32_t* wg0, int n_inst, int moving,
                         unsigned grid, size_t lds, void* stream) {
    hipLaunchKernelGGL((k1_pairs<T, PMAX, QMAX, ALT, NT>), dim3(grid),
                       dim3(K1PBlock<T, PMAX, QMAX, ALT>::value), lds, (hipStream_t)stream,
                       static_cast<const K1Args<T>*>(args), wg0, n_inst, moving);
}

template <typename T, int PMAX, int QMAX>
static int launch_k1p_t(const void* args, const uint32_t* wg0, int n_inst, int moving,
                        unsigned grid, size_t lds, void* stream, int alt, int nt) {
    if (alt) {
        if (nt) launch_k1p_f<T, PMAX, QMAX, 1, 1>(args, wg0, n_inst, moving, grid, lds, stream);
        else launch_k1p_f<T, PMAX, QMAX, 1, 0>(args, wg0, n_inst, moving, grid, lds, stream);
    } else {
        if (nt) launch_k1p_f<T, PMAX, QMAX, 0, 1>(args, wg0, n_inst, moving, grid, lds, stream);
        else launch_k1p_f<T, PMAX, QMAX, 0, 0>(args, wg0, n_inst, moving, grid, lds, stream);
    }
    return (int)hipGetLastError();
}

template <typename T>
static int launch_k1p_any(int pmax, int qmax, const void* args, const uint32_t* wg0, int n_inst,
                          int moving, unsigned grid, size_t lds, void* stream, int alt,
                          int nt) {
    const bool q12 = qmax == 12;
    switch (pmax) {
    case 3: return q12 ? launch_k1p_t<T, 3, 12>(args, wg0, n_inst, moving, grid, lds, stream, alt, nt)
                       : launch_k1p_t<T, 3, 8>(args, wg0, n_inst, moving, grid, lds, stream, alt, nt);
    case 6: return q12 ? launch_k1p_t<T, 6, 12>(args, wg0, n_inst, moving, grid, lds, stream, alt, nt)
                       : launch_k1p_t<T, 6, 8>(args, wg0, n_inst, moving, grid, lds, stream, alt, nt);
    case 9: return q12 ? launch_k1p_t<T, 9, 12>(args, wg0, n_inst, moving, grid, lds, stream, alt, nt)
                       : launch_k1p_t<T, 9, 8>(args, wg0, n_inst, moving, grid, lds, stream, alt, nt);
    default: return q12 ? launch_k1p_t<T, 16, 12>(args, wg0, n_inst, moving, grid, lds, stream, alt, nt)
                        : launch_k1p_t<T, 16, 8>(args, wg0, n_inst, moving, grid, lds, stream, alt, nt);
    }
}

int launch_k1(int fp32, int pmax, int qmax, int paired, const void* args, const uint32_t* wg0,
              int n_inst, int moving, unsigned grid, size_t lds, void* stream, int alt, int nt) {
    if (paired) {
        if (!k1p_buckets(pmax, qmax)) return (int)hipErrorInvalidValue;
        if (fp32)
            return launch_k1p_any<float>(pmax, qmax, args, wg0, n_inst, moving, grid, lds, stream,
                                         alt, nt);
        return launch_k1p_any<double>(pmax, qmax, args, wg0, n_inst, moving, grid, lds, stream,
                                      alt, nt);
    }
    if (fp32) return launch_k1_any<float>(pmax, qmax, args, wg0, n_inst, moving, grid, lds, stream);
    return launch_k1_any<double>(pmax, qmax, args, wg0, n_inst, moving, grid, lds, stream);
}

template <typename T, int PMAX, int NPL>
static void launch_k2_p(const K2Args<T>* a, int n_inst, dim3 g, size_t lds, hipStream_t s) {
    if constexpr (K2Narrow<T, PMAX, NPL>::value)
        hipLaunchKernelGGL((k2_collide<T, PMAX, NPL>), g, dim3(kBlock), lds, s, a, n_inst);
    else
        hipLaunchKernelGGL((k2_collide_wide<T, PMAX, NPL>), g, dim3(kBlock), lds, s, a, n_inst);
}

template <typename T, int NPL>
static int launch_k2_n(int pmax, const K2Args<T>* a, int n_inst, unsigned grid, size_t lds,
                       hipStream_t s) {
    const dim3 g(grid);
    switch (pmax) {
    case 1: launch_k2_p<T, 1, NPL>(a, n_inst, g, lds, s); break;
    case 3: launch_k2_p<T, 3, NPL>(a, n_inst, g, lds, s); break;
    case 6: launch_k2_p<T, 6, NPL>(a, n_inst, g, lds, s); break;
    case 9: launch_k2_p<T, 9, NPL>(a, n_inst, g, lds, s); break;
    case 16: launch_k2_p<T, 16, NPL>(a, n_inst, g, lds, s); break;
    default: launch_k2_p<T, 32, NPL>(a, n_inst, g, lds, s); break;
    }
    return (int)hipGetLastError();
}

template <typename T>
static int launch_k2l(int pmax, const K2Args<T>* a, int n_inst, unsigned grid, size_t lds,
                      hipStream_t s) {
    const dim3 g(grid), b(kBlock);
    switch (pmax) {
    case 1: hipLaunchKernelGGL((k2_lanes<T, 1>), g, b, lds, s, a, n_inst); break;
    case 3: hipLaunchKernelGGL((k2_lanes<T, 3>), g, b, lds, s, a, n_inst); break;
    case 6: hipLaunchKernelGGL((k2_lanes<T, 6>), g, b, lds, s, a, n_inst); break;
    case 9: hipLaunchKernelGGL((k2_lanes<T, 9>), g, b, lds, s, a, n_inst); break;
    case 16: hipLaunchKernelGGL((k2_lanes<T, 16>), g, b, lds, s, a, n_inst); break;
    default: hipLaunchKernelGGL((k2_lanes<T, 32>), g, b, lds, s, a, n_inst); break;
    }
    return (int)hipGetLastError();
}

// npl: nodes per lane, 2 when some instance of the group has more than 64
// nodes; lanes: a lane per candidate (every instance has at most 12 nodes)
int launch_k2(int fp32, int pmax, int npl, int lanes, const void* args, int n_inst,
              unsigned grid, size_t lds, void* stream) {
    const hipStream_t s = (hipStream_t)stream;
    if (lanes) {
        if (fp32) return launch_k2l<float>(pmax, static_cast<const K2Args<float>*>(args), n_inst,
                                           grid, lds, s);
        return launch_k2l<double>(pmax, static_cast<const K2Args<double>*>(args), n_inst, grid,
                                  lds, s);
    }
    if (fp32) {
        const K2Args<float>* a = static_cast<const K2Args<float>*>(args);
        return npl > 1 ? launch_k2_n<float, 2>(pmax, a, n_inst, grid, lds, s)
                       : launch_k2_n<float, 1>(pmax, a, n_inst, grid, lds, s);
    }
    const K2Args<double>* a = static_cast<const K2Args<double>*>(args);
    return npl > 1 ? launch_k2_n<double, 2>(pmax, a, n_inst, grid, lds, s)
                   : launch_k2_n<double, 1>(pmax, a, n_inst, grid, lds, s);
}

// finalize workgroups of one instance: the window part, the rest of the
// grid, and at least one per (node, batch) of the moment record
int k3_grid_of(int Q, int nk, int n_win_wg, int nb) {
    const int64_t rest = ((int64_t)Q * nk * nk + kK3Rest - 1) / kK3Rest;
    int64_t grid = (int64_t)n_win_wg + rest;
    if (grid < (int64_t)Q * nb) grid = (int64_t)Q * nb;
    return (int)grid;
}

int launch_k3(const K3Args* args, const uint32_t* wg0, int n_inst, int moving, unsigned grid,
              void* stream) {
    hipLaunchKernelGGL(k3_finalize, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, args, wg0,
                       n_inst, moving);
    return (int)hipGetLastError();
}

// Step state of n instances: the step counters (set_step) and the time step
// (set_dt), written by one small kernel so the writes are ordered on the stream.
__global__ void set_dyn_kernel(Dyn* d, int n, int set_step, uint32_t step, uint32_t rec_base,
                               int set_dt, double dt) {
    const int k = (int)threadIdx.x;
    if (k >= n) return;
    if (set_step) {
        d[k].step_k1 = step; d[k].step_k3 = step; d[k].step_k2 = step - 1u;
        d[k].rec_base = rec_base;
    }
    if (set_dt) { d[k].dt = dt; d[k].vfdt = d[k].v_f * dt; }
}

int launch_set_dyn(Dyn* d, int n, int set_step, uint32_t step, uint32_t rec_base, int set_dt,
                   double dt, void* stream) {
    if (n <= 0) return 0;
    for (int k0 = 0; k0 < n; k0 += 1024) {
        const int m = n - k0 < 1024 ? n - k0 : 1024;
        hipLaunchKernelGGL(set_dyn_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, d + k0, m,
                           set_step, step, rec_base, set_dt, dt);
    }
    return (int)hipGetLastError();
}

// -------------------------------------------------------- initial datum
__device__ double fd_w(double e, double mu, double kT) { return e / (1.0 + exp((e - mu) / kT)); }

__device__ double fd_panel(const InitArgs& a, double lo, double hi) {
    const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
    double s = 0.0;
    for (int k = 0; k < 10; ++k) s += a.gl[10 + k] * fd_w(c + h * a.gl[k], a.mu, a.kT);
    return s * h;
}

// Energy with F_q(eps) = u, u = (m + 1/2) 2^-52, by safeguarded Newton
// inside the table panel that brackets the target; the upper half works
// with the complementary tail so both tails keep full relative precision.
__device__ double fd_inverse(const InitArgs& a, int q, uint64_t m) {
    const int np = a.cdf_np;
    const double* lo = a.cdf_lo + (size_t)q * (np + 1);
    const double* hi = a.cdf_hi + (size_t)q * (np + 1);
    const double e0 = a.eps0[q];
    const double Z = lo[np];
    const bool upper = m >= (1ull << 51);
    const double target = upper ? ((double)((1ull << 52) - 1ull - m) + 0.5) * 0x1p-52 * Z
                                : ((double)m + 0.5) * 0x1p-52 * Z;
    int j0 = 0, j1 = np - 1;
    while (j0 < j1) {
        const int mid = (j0 + j1 + 1) >> 1;
        const bool right = upper ? (hi[mid] > target) : (lo[mid] <= target);
        if (right) j0 = mid; else j1 = mid - 1;
    }
    const int j = j0;
    const double xa = e0 + j * a.cdf_h, xb = e0 + (j + 1) * a.cdf_h;
    double ba = xa, bb = xb;      // bracket
    double fracv = upper ? (hi[j] - target) / (hi[j] - hi[j + 1])
                         : (target - lo[j]) / (lo[j + 1] - lo[j]);
    fracv = fmin(fmax(fracv, 0.0), 1.0);
    double e = xa + fracv * (xb - xa);
    for (int it = 0; it < 60; ++it) {
        const double F = upper ? target - (fd_panel(a, e, xb) + hi[j + 1])
                               : (lo[j] + fd_panel(a, xa, e)) - target;   // increasing in e
        if (F > 0.0) bb = e; else ba = e;
        const double g = fd_w(e, a.mu, a.kT);
        double en = (g > 0.0) ? e - F / g : 0.5 * (ba + bb);
        if (!(en > ba && en < bb)) en = 0.5 * (ba + bb);
        if (en == e || !(bb > ba)) break;
        if (fabs(en - e) <= 2e-16 * e) { e = en; break; }
        e = en;
    }
    return e;
}

__global__ void __launch_bounds__(kBlock) init_kernel(const InitArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n) return;
    const Words w = philox10((uint32_t)i, 0xFFFFFFFFu, kPurInit, a.instance, a.seed_lo, a.seed_hi);
    const uint64_t m = ((uint64_t)w.w0 << 20) | (uint64_t)(w.w1 >> 12);
    const double uth = uni<double>(w.w2, w.w3);
    double sth, cth;
    sincospi(2.0 * uth, &sth, &cth);
    double ax[kMaxP], ay[kMaxP];
    for (int h = 0; h < a.P; ++h) { ax[h] = 0.0; ay[h] = 0.0; }
    for (int q = 0; q < a.Q; ++q) {
        const double e = fd_inverse(a, q, m);
        const double e0 = a.eps0[q];
        const double kabs = sqrt((e - e0) * (e + e0));
        const double nx = kabs * cth, ny = kabs * sth;
        for (int h = 0; h < a.P; ++h) {
            ax[h] += a.wpsi[q * a.P + h] * nx;
            ay[h] += a.wpsi[q * a.P + h] * ny;
        }
    }
    for (int h = 0; h < a.P; ++h) {
        if (a.kx64) { a.kx64[(size_t)h * a.n + i] = ax[h]; a.ky64[(size_t)h * a.n + i] = ay[h]; }
        else { a.kx32[(size_t)h * a.n + i] = (float)ax[h]; a.ky32[(size_t)h * a.n + i] = (float)ay[h]; }
    }
}

int launch_init(const InitArgs& a, void* stream) {
    const int64_t blocks = (a.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(init_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

// ---------------------------------------------- energy distribution
template <typename T>
__device__ void energy_hist_t(const EnergyHistArgs& a, int64_t i) {
    const T* kx = reinterpret_cast<const T*>(a.kx);
    const T* ky = reinterpret_cast<const T*>(a.ky);
    for (int q = 0; q < a.Q; ++q) {
        double x = 0.0, y = 0.0;
        for (int h = 0; h < a.P; ++h) {
            x += (double)kx[(size_t)h * a.n + i] * a.psi[q * a.P + h];
            y += (double)ky[(size_t)h * a.n + i] * a.psi[q * a.P + h];
        }
        const double e = sqrt(x * x + y * y + a.eps0[q] * a.eps0[q]);
        const double fb = floor((e - a.emin) / a.width);
        if (fb >= 0.0 && fb < (double)a.nbins) atomicAdd(&a.bins[(size_t)q * a.nbins + (int)fb], 1ull);
    }
}

__global__ void __launch_bounds__(kBlock) energy_hist_kernel(const EnergyHistArgs a) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n) return;
    if (a.fp32) energy_hist_t<float>(a, i); else energy_hist_t<double>(a, i);
}

int launch_energy_hist(const EnergyHistArgs& a, void* stream) {
    const int64_t blocks = (a.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(energy_hist_kernel, dim3((unsigned)blocks), dim3(kBlock), 0,
                       (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

// ---------------------------------- energy distribution without allocation
// For callers that cannot allocate device memory: the bin counts live in a
// file-scope device array (one copy per GPU, held until the process ends)
// instead of a caller-provided workspace.  Host code never passes the
// array's name to a kernel: it takes the array's device address per device
// with hipGetSymbolAddress once and passes that.
constexpr int kNoAllocCounts = 1 << 19;     // Q * nbins limit: 4 MiB of counts
static __device__ __align__(256) unsigned long long scratch[kNoAllocCounts];

__global__ void __launch_bounds__(kBlock) fill_u64_kernel(unsigned long long* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void __launch_bounds__(kBlock) counts_to_density_kernel(const unsigned long long* c,
                                                                   double* out, int64_t n,
                                                                   double scale) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = (double)c[i] / scale;
}

// ------------------------------------------------- moments at given z
// Each particle's expansion evaluated at up to kMomZ points z (Sec. 4.2: the
// particle reconstruction at arbitrary z): sums of v_x, v_y and eps per point
// in FP64, one partial per workgroup, reduced in fixed order.
template <typename T>
__device__ __forceinline__ void moments_at_t(const MomAtArgs& a, const double* zt, double (&acc)[kMomZ][3]) {
    const T* kx = static_cast<const T*>(a.kx);
    const T* ky = static_cast<const T*>(a.ky);
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < a.n;
         i += (int64_t)gridDim.x * kBlock) {
        // modes outer, points inner: k(z_j) = sum_h k_h Psi_h(z_j)
        double x[kMomZ], y[kMomZ];
#pragma unroll
        for (int j = 0; j < kMomZ; ++j) { x[j] = 0.0; y[j] = 0.0; }
        for (int h = 0; h < a.P; ++h) {
            const double cx = (double)kx[(size_t)h * a.n + i];
            const double cy = (double)ky[(size_t)h * a.n + i];
#pragma unroll
            for (int j = 0; j < kMomZ; ++j) {
                const double p = zt[j * (a.P + 1) + h];
                x[j] += cx * p;
                y[j] += cy * p;
            }
        }
#pragma unroll
        for (int j = 0; j < kMomZ; ++j) {
            if (j < a.nz) {
                const double e0 = zt[j * (a.P + 1) + a.P];
                const double e = sqrt(x[j] * x[j] + y[j] * y[j] + e0 * e0);
                acc[j][0] += a.v_f * x[j] / e;
                acc[j][1] += a.v_f * y[j] / e;
                acc[j][2] += e;
            }
        }
    }
}

__global__ void __launch_bounds__(kBlock) moments_at_kernel(const MomAtArgs a) {
    __shared__ double zt[kMomZ * (kMaxP + 1)];
    __shared__ double red[kWaves][kMomZ][3];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = tid; k < kMomZ * (a.P + 1); k += kBlock)
        zt[k] = k < a.nz * (a.P + 1) ? a.zpsi[k] : 0.0;
    __syncthreads();
    double acc[kMomZ][3];
#pragma unroll
    for (int j = 0; j < kMomZ; ++j) { acc[j][0] = 0.0; acc[j][1] = 0.0; acc[j][2] = 0.0; }
    if (a.fp32) moments_at_t<float>(a, zt, acc); else moments_at_t<double>(a, zt, acc);
#pragma unroll
    for (int j = 0; j < kMomZ; ++j)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const double v = wave_sum(acc[j][m]);
            if (lane == 0) red[wave][j][m] = v;
        }
    __syncthreads();
    if (tid < kMomZ * 3) {
        const int j = tid / 3, m = tid - 3 * (tid / 3);
        double v = 0.0;
        for (int w = 0; w < kWaves; ++w) v += red[w][j][m];
        a.partial[((size_t)blockIdx.x * kMomZ + j) * 3 + m] = v;
    }
}

int launch_moments_at(const MomAtArgs& a, int nwg, void* stream) {
    hipLaunchKernelGGL(moments_at_kernel, dim3((unsigned)nwg), dim3(kBlock), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

// ------------------------------------------------------ Philox test hook
__global__ void philox_kernel(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Words w = philox10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3],
                             key[2 * i], key[2 * i + 1]);
    out[4 * i] = w.w0; out[4 * i + 1] = w.w1; out[4 * i + 2] = w.w2; out[4 * i + 3] = w.w3;
}

int launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n, void* stream) {
    if (n <= 0) return 0;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(philox_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       ctr, key, out, n);
    return (int)hipGetLastError();
}

}  // namespace sgpm

namespace {

// device address of the scratch array on each device, taken once per device
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[64] = {};

}  // namespace

extern "C" sgpm_status sgpm_energy_density_noalloc(const void* kx, const void* ky,
                                                   int32_t precision, int64_t n, int32_t P,
                                                   int32_t Q, const double* psi,
                                                   const double* eps0, int32_t nbins,
                                                   double emin_eV, double emax_eV, double* out,
                                                   void* hip_stream) {
    using namespace sgpm;
    if (!kx || !ky || !psi || !eps0 || !out) return SGPM_EINVAL;
    if (precision != SGPM_FP64 && precision != SGPM_FP32) return SGPM_EINVAL;
    if (n < 1 || n > (int64_t)2000000000 || P < 1 || P > kMaxP || Q < 1 || Q > kMaxQ)
        return SGPM_EINVAL;
    if (nbins < 1 || !(emax_eV > emin_eV) || !std::isfinite(emin_eV) || !std::isfinite(emax_eV))
        return SGPM_EINVAL;
    if ((int64_t)Q * nbins > kNoAllocCounts) return SGPM_EUNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SGPM_EDEVICE;
    unsigned long long* counts = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
                return SGPM_EDEVICE;
            g_scratch_ptr[dev] = static_cast<unsigned long long*>(p);
        }
        counts = g_scratch_ptr[dev];
    }
    const hipStream_t st = (hipStream_t)hip_stream;
    const int64_t m = (int64_t)Q * nbins;
    const unsigned blocks = (unsigned)((m + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks), dim3(kBlock), 0, st, counts, m);
    if (hipGetLastError() != hipSuccess) return SGPM_EDEVICE;
    EnergyHistArgs a;
    a.kx = kx; a.ky = ky; a.fp32 = precision == SGPM_FP32 ? 1 : 0; a.n = n; a.P = P; a.Q = Q;
    a.psi = psi; a.eps0 = eps0; a.nbins = nbins; a.emin = emin_eV;
    a.width = (emax_eV - emin_eV) / nbins;
    a.bins = counts;
    if (launch_energy_hist(a, hip_stream) != 0) return SGPM_EDEVICE;
    hipLaunchKernelGGL(counts_to_density_kernel, dim3(blocks), dim3(kBlock), 0, st, counts, out, m,
                       (double)n * a.width);
    if (hipGetLastError() != hipSuccess) return SGPM_EDEVICE;
    return SGPM_OK;
}
