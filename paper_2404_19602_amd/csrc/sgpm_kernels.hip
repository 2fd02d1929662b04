// gfx950 kernels of the sG-PM hot path (arXiv:2404.19602, Algorithm 2).
//
// One time step of one instance is three launches:
//  K1 stream   -- lane per particle over a chunk per workgroup: Galerkin drift
//                 (Sec. 4.1), an upper bound of the node-maximum collision
//                 rate from the coefficients (eq. deltat) that proves most
//                 particles do not collide in this step; for those, the node
//                 values k_i(z_q) (eq. gPC), their cells in H^{n+1} through a
//                 privatised LDS window, and FP64 sums of v_x, v_y and the
//                 energy per node (Sec. 4.2).  The others are listed, in a
//                 fixed order, as collision candidates.
//  K2 collide  -- the candidates of one K1 workgroup, a group of lanes per
//                 candidate and one node per lane: exact node rates, the
//                 node maximum, free flight, mechanism selection (eq.
//                 update_gPC), final states, Pauli acceptance against H^n on
//                 the moved grid (eq. Pauli_gPC) and the projection of eq.
//                 update_sG as a group sum; then their H^{n+1} cells and sums.
//  K3 finalize -- one workgroup per node: the maximum of H^{n+1}, clearing of
//                 the stale buffer for the next step, and the fixed-order
//                 reduction of the moment sums into the record.
#include <hip/hip_runtime.h>
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
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    return Words{c0, c1, c2, c3};
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

// floor((x + L)/dk) as the rounded quotient gives it: the product by 1/dk is
// replaced by the true division only within a few ulps of an integer.
// Outside [0, 2^30) (and NaN) -> -1.
template <typename T>
__device__ __forceinline__ int cell_coord(T x, T L, T dk, T inv_dk) {
    const T s = x + L;
    T qt = s * inv_dk;
    const T r = rint(qt);
    if (fabs(qt - r) <= (T)8 * Num<T>::eps * fabs(qt) + (T)1e-30) qt = s / dk;
    const T f = floor(qt);
    return (f >= (T)0 && f < (T)1073741824) ? (int)f : -1;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T group_max(T v, int G) {
    for (int m = G >> 1; m >= 1; m >>= 1) {
        const T o = __shfl_xor(v, m, G);
        v = o > v ? o : v;
    }
    return v;
}

// sum over the lanes of the group, the same value (the group's first lane's
// result) delivered to every lane
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
    for (int m = G >> 1; m >= 1; m >>= 1) v += __shfl_xor(v, m, G);
    return __shfl(v, 0, G);
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

// ======================================================= K1: stream kernel
size_t k1_lds_bytes(int P, int Q, int fp32, int hwin_words) {
    const size_t s = fp32 ? 4 : 8;
    size_t off = (size_t)hwin_words * 4;
    off = (off + 15) & ~(size_t)15;
    off += sizeof(Consts<double>);                       // consts (either precision fits)
    off = (off + 15) & ~(size_t)15;
    off += s * ((size_t)Q * P + Q + 2 * P);             // psi, eps0sq, psimax, drift
    off = (off + 15) & ~(size_t)15;
    off += (size_t)kWaves1 * Q * 3 * 8;                  // per-wave moment sums
    off += 16 * 4;                                       // counters
    return off;
}

template <typename T>
struct K1Lds {
    uint32_t* hwin;
    Consts<T>* c;
    T* psi; T* eps0sq; T* psimax; T* drift;
    double* red;
    uint32_t* cnt;
};

template <typename T>
__device__ __forceinline__ K1Lds<T> k1_lds(unsigned char* smem, int P, int Q, int hwin_words) {
    K1Lds<T> L;
    size_t off = (size_t)hwin_words * 4;
    off = (off + 15) & ~(size_t)15;
    L.hwin = reinterpret_cast<uint32_t*>(smem);
    L.c = reinterpret_cast<Consts<T>*>(smem + off);
    off += sizeof(Consts<double>);
    off = (off + 15) & ~(size_t)15;
    L.psi = reinterpret_cast<T*>(smem + off);
    L.eps0sq = L.psi + Q * P;
    L.psimax = L.eps0sq + Q;
    L.drift = L.psimax + P;
    off += sizeof(T) * ((size_t)Q * P + Q + 2 * P);
    off = (off + 15) & ~(size_t)15;
    L.red = reinterpret_cast<double*>(smem + off);
    off += (size_t)kWaves1 * Q * 3 * 8;
    L.cnt = reinterpret_cast<uint32_t*>(smem + off);
    return L;
}

// one nodal value into H^{n+1}: LDS window when inside it, else global
template <typename T>
__device__ __forceinline__ void k1_bin(const K1Args<T>& a, const K1Lds<T>& L, const Consts<T>& c,
                                       int q, T kx, T ky) {
    const int r = cell_coord<T>(kx, c.lk, c.dk, c.inv_dk);
    const int l = cell_coord<T>(ky, c.lk, c.dk, c.inv_dk);
    if (r < 0 || l < 0 || r >= c.nk || l >= c.nk) {
        atomicAdd(&L.cnt[SGPM_CNT_OUT_OF_GRID], 1u);
        return;
    }
    const int wr = r - a.win_r0, wl = l - a.win_l0;
    if ((unsigned)wr < (unsigned)a.win && (unsigned)wl < (unsigned)a.win) {
        const int idx = (q * a.win + wr) * a.win + wl;
        atomicAdd(&L.hwin[idx >> 1], (idx & 1) ? 65536u : 1u);
    } else {
        atomicAdd(&a.h_acc[(size_t)q * c.nk * c.nk + (size_t)r * c.nk + l], 1u);
    }
}

template <typename T, int PMAX, int QMAX>
__global__ void __launch_bounds__(kBlock1) k1_stream(const K1Args<T> a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int P = a.P, Q = a.Q;
    const K1Lds<T> L = k1_lds<T>(smem, P, Q, a.hwin_words);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int w = tid; w < a.hwin_words; w += kBlock1) L.hwin[w] = 0u;
    if (tid == 0) *L.c = *a.tab.consts;
    for (int k = tid; k < Q * P; k += kBlock1) L.psi[k] = a.tab.psi[k];
    for (int k = tid; k < Q; k += kBlock1) L.eps0sq[k] = a.tab.eps0sq[k];
    for (int k = tid; k < P; k += kBlock1) {
        L.psimax[k] = a.tab.psimax[k];
        L.drift[k] = a.do_drift ? (T)(a.vfdt * a.ehat[k]) : (T)0;
    }
    for (int k = tid; k < kWaves1 * Q * 3; k += kBlock1) L.red[k] = 0.0;
    if (tid < 16) L.cnt[tid] = 0u;
    __syncthreads();
    const Consts<T>& c = *L.c;

    const int64_t begin = (int64_t)blockIdx.x * a.chunk;
    const int64_t end = begin + a.chunk < a.n ? begin + a.chunk : a.n;
    int* my_cand = a.cand_idx + ((size_t)blockIdx.x * kWaves1 + wave) * a.cap_w;
    int ncand = 0;     // uniform per wave

    double acc[QMAX > 0 ? QMAX : 1][3];
    if constexpr (QMAX > 0) {
#pragma unroll
        for (int q = 0; q < QMAX; ++q) { acc[q][0] = 0.0; acc[q][1] = 0.0; acc[q][2] = 0.0; }
    }

    for (int64_t base = begin; base < end; base += kBlock1) {
        const int64_t i = base + tid;
        const bool act = i < end;
        const int64_t ii = act ? i : begin;
        T cx[PMAX], cy[PMAX];
#pragma unroll
        for (int h = 0; h < PMAX; ++h) {
            if (h < P) {
                cx[h] = a.kx[(size_t)h * a.n + ii] - L.drift[h];   // k_h -= (e/hbar) dt E_h
                cy[h] = a.ky[(size_t)h * a.n + ii];
            } else {
                cx[h] = (T)0; cy[h] = (T)0;
            }
        }
        bool cand = false;
        if (act && a.do_collide) {
            // |k(z_q)| <= sum_h |k_h| max_q |Psi_h(z_q)| per component
            T bx = (T)0, by = (T)0;
#pragma unroll
            for (int h = 0; h < PMAX; ++h)
                if (h < P) { bx += fabs(cx[h]) * L.psimax[h]; by += fabs(cy[h]) * L.psimax[h]; }
            const T emax = sqrt(bx * bx + by * by + c.eps0max_sq);
            const T gb = rate_bound<T>(c, emax);
            const Words wx = philox10((uint32_t)i, a.step, kPurXi, a.instance, a.seed_lo, a.seed_hi);
            const T xlog = -dlog(uni<T>(wx.w0, wx.w1));
            cand = !(xlog >= gb * a.dt);    // no collision iff -log(xi)/G~ >= dt
        }
        const bool fin = act && !cand;
        if (fin && a.do_drift) {
#pragma unroll
            for (int h = 0; h < PMAX; ++h)
                if (h < P && L.drift[h] != (T)0) a.kx[(size_t)h * a.n + i] = cx[h];
        }
        // candidates of this wave, in lane order
        const uint64_t mask = __ballot(cand);
        if (cand) {
            const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            my_cand[ncand + pos] = (int)(i - begin);
        }
        ncand += __popcll(mask);

        // nodes of the particles that are final now
        if constexpr (QMAX > 0) {
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
                if (q < Q && fin) {
                    const T* ps = L.psi + q * P;
                    T kx = (T)0, ky = (T)0;
#pragma unroll
                    for (int h = 0; h < PMAX; ++h)
                        if (h < P) { kx += cx[h] * ps[h]; ky += cy[h] * ps[h]; }
                    const T e = sqrt(kx * kx + ky * ky + L.eps0sq[q]);
                    const T inv = (T)1 / e;
                    acc[q][0] += (double)(c.v_f * kx * inv);
                    acc[q][1] += (double)(c.v_f * ky * inv);
                    acc[q][2] += (double)e;
                    k1_bin<T>(a, L, c, q, kx, ky);
                }
            }
        } else {
            for (int q = 0; q < Q; ++q) {
                double vx = 0.0, vy = 0.0, en = 0.0;
                if (fin) {
                    const T* ps = L.psi + q * P;
                    T kx = (T)0, ky = (T)0;
#pragma unroll
                    for (int h = 0; h < PMAX; ++h)
                        if (h < P) { kx += cx[h] * ps[h]; ky += cy[h] * ps[h]; }
                    const T e = sqrt(kx * kx + ky * ky + L.eps0sq[q]);
                    const T inv = (T)1 / e;
                    vx = (double)(c.v_f * kx * inv);
                    vy = (double)(c.v_f * ky * inv);
                    en = (double)e;
                    k1_bin<T>(a, L, c, q, kx, ky);
                }
                vx = wave_sum(vx); vy = wave_sum(vy); en = wave_sum(en);
                if (lane == 0) {
                    double* m = L.red + ((size_t)wave * Q + q) * 3;
                    m[0] += vx; m[1] += vy; m[2] += en;
                }
            }
        }
    }
    if constexpr (QMAX > 0) {
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            if (q < Q) {
                const double vx = wave_sum(acc[q][0]), vy = wave_sum(acc[q][1]),
                             en = wave_sum(acc[q][2]);
                if (lane == 0) {
                    double* m = L.red + ((size_t)wave * Q + q) * 3;
                    m[0] = vx; m[1] = vy; m[2] = en;
                }
            }
        }
    }
    if (lane == 0) {
        a.cand_cnt[(size_t)blockIdx.x * kWaves1 + wave] = ncand;
        if (ncand) atomicAdd(&L.cnt[SGPM_CNT_CANDIDATES], (uint32_t)ncand);
    }
    __syncthreads();

    // flush the LDS window: nonzero cells to global atomics
    {
        const int wcells = a.win * a.win;
        for (int w = tid; w < a.hwin_words; w += kBlock1) {
            const uint32_t v = L.hwin[w];
            if (v == 0u) continue;
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const uint32_t cnt = half ? (v >> 16) : (v & 0xFFFFu);
                if (cnt == 0u) continue;
                const int idx = 2 * w + half;
                const int q = idx / wcells, rem = idx - q * wcells;
                const int r = a.win_r0 + rem / a.win, l = a.win_l0 + rem % a.win;
                atomicAdd(&a.h_acc[(size_t)q * c.nk * c.nk + (size_t)r * c.nk + l], cnt);
            }
        }
    }
    // this workgroup's moment sums, waves in order
    for (int k = tid; k < Q * 3; k += kBlock1) {
        double v = 0.0;
        for (int wv = 0; wv < kWaves1; ++wv) v += L.red[wv * Q * 3 + k];
        a.partial[(size_t)blockIdx.x * Q * 3 + k] = v;
    }
    if (tid < 8 && L.cnt[tid]) atomicAdd(&a.counters[tid], (unsigned long long)L.cnt[tid]);
}

// ===================================================== K2: collider kernel
size_t k2_lds_bytes(int P, int Q, int fp32) {
    const size_t s = fp32 ? 4 : 8;
    size_t off = sizeof(Consts<double>);
    off = (off + 15) & ~(size_t)15;
    off += s * (2 * (size_t)Q * P + 4 * (size_t)Q + 32 + P);   // psi wpsi eps0 eps0sq cedge vfield ecos drift
    off = (off + 15) & ~(size_t)15;
    off += (size_t)2 * kBlock * 3 * 8;   // final sums of a pass, [groups][Q][3]
    off += (size_t)Q * 3 * 8;            // running sums
    off += 16 * 4 + (kWaves1 + 1) * 4;   // counters, candidate offsets
    return off;
}

template <typename T>
struct K2Lds {
    Consts<T>* c;
    T* psi; T* wpsi; T* eps0; T* eps0sq; T* cedge; T* vfield; T* ecos; T* drift;
    double* pass;   // [groups per pass][Q][3]
    double* run;    // [Q][3]
    uint32_t* cnt;
    int* off;       // [kWaves1 + 1]
};

template <typename T>
__device__ __forceinline__ K2Lds<T> k2_lds(unsigned char* smem, int P, int Q) {
    K2Lds<T> L;
    size_t off = 0;
    L.c = reinterpret_cast<Consts<T>*>(smem);
    off = sizeof(Consts<double>);
    off = (off + 15) & ~(size_t)15;
    L.psi = reinterpret_cast<T*>(smem + off);
    L.wpsi = L.psi + Q * P;
    L.eps0 = L.wpsi + Q * P;
    L.eps0sq = L.eps0 + Q;
    L.cedge = L.eps0sq + Q;
    L.vfield = L.cedge + Q;
    L.ecos = L.vfield + Q;
    L.drift = L.ecos + 32;
    off += sizeof(T) * (2 * (size_t)Q * P + 4 * (size_t)Q + 32 + P);
    off = (off + 15) & ~(size_t)15;
    L.pass = reinterpret_cast<double*>(smem + off);
    off += (size_t)2 * kBlock * 3 * 8;
    L.run = reinterpret_cast<double*>(smem + off);
    off += (size_t)Q * 3 * 8;
    L.cnt = reinterpret_cast<uint32_t*>(smem + off);
    off += 16 * 4;
    L.off = reinterpret_cast<int*>(smem + off);
    return L;
}

// Pauli occupation f = H^n / max H^n of node q at the candidate's cell on the
// grid moved with this step's drift (lookup at k' + v_F E(z_q) dt x^)
template <typename T>
__device__ __forceinline__ T pauli_f(const K2Args<T>& a, const K2Lds<T>& L, const Consts<T>& c,
                                     int q, T px, T py) {
    const uint32_t mx = a.hmax_read[q];
    if (mx == 0u) return (T)0;
    const T shift = L.vfield[q] * a.dt;
    const int r = cell_coord<T>(px + shift, c.lk, c.dk, c.inv_dk);
    const int l = cell_coord<T>(py, c.lk, c.dk, c.inv_dk);
    if (r < 0 || l < 0 || r >= c.nk || l >= c.nk) return (T)0;
    const uint32_t h = a.h_read[(size_t)q * c.nk * c.nk + (size_t)r * c.nk + l];
    return (T)h / (T)mx;
}

template <typename T, int PMAX>
__global__ void __launch_bounds__(kBlock) k2_collide(const K2Args<T> a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int P = a.P, Q = a.Q, G = a.G;
    const K2Lds<T> L = k2_lds<T>(smem, P, Q);
    const int tid = threadIdx.x;
    const int wg = blockIdx.x;

    if (tid == 0) {
        int s = 0;
        for (int w = 0; w < kWaves1; ++w) {
            L.off[w] = s;
            s += a.cand_cnt[(size_t)wg * kWaves1 + w];
        }
        L.off[kWaves1] = s;
    }
    __syncthreads();
    const int M = L.off[kWaves1];
    if (M == 0) return;

    if (tid == 0) *L.c = *a.tab.consts;
    for (int k = tid; k < Q * P; k += kBlock) { L.psi[k] = a.tab.psi[k]; L.wpsi[k] = a.tab.wpsi[k]; }
    for (int k = tid; k < Q; k += kBlock) {
        L.eps0[k] = a.tab.eps0[k]; L.eps0sq[k] = a.tab.eps0sq[k];
        L.cedge[k] = a.tab.cedge[k]; L.vfield[k] = a.tab.vfield[k];
    }
    for (int k = tid; k <= kEdgePts / 2; k += kBlock) L.ecos[k] = a.tab.edge_cos[k];
    for (int k = tid; k < P; k += kBlock) L.drift[k] = (T)(a.vfdt * a.ehat[k]);
    for (int k = tid; k < Q * 3; k += kBlock) L.run[k] = 0.0;
    if (tid < 16) L.cnt[tid] = 0u;
    __syncthreads();
    const Consts<T>& c = *L.c;

    const int g = tid % G;                // rank in the group = node handled
    const int grp = tid / G;
    const int per_pass = kBlock / G;
    const int64_t begin = (int64_t)wg * a.chunk;

    for (int p0 = 0; p0 < M; p0 += per_pass) {
        const int cid = p0 + grp;
        const bool has = cid < M;
        int64_t i = begin;
        if (has) {
            int w = 0;
            while (cid >= L.off[w + 1]) ++w;
            i = begin + a.cand_idx[((size_t)wg * kWaves1 + w) * a.cap_w + (cid - L.off[w])];
        }
        T cx[PMAX], cy[PMAX];
#pragma unroll
        for (int h = 0; h < PMAX; ++h) {
            if (h < P) {
                cx[h] = a.kx[(size_t)h * a.n + i] - L.drift[h];
                cy[h] = a.ky[(size_t)h * a.n + i];
            } else {
                cx[h] = (T)0; cy[h] = (T)0;
            }
        }
        if (has) {
            T tc = (T)0;
            uint32_t coll = 0;
            const uint32_t ctr0 = (uint32_t)i;
            for (;;) {
                // Gamma~ = (1 + alpha) max over the nodes of sum_nu Gamma^nu
                T smax = (T)0;
                for (int q = g; q < Q; q += G) {
                    const T* ps = L.psi + q * P;
                    T kx = (T)0, ky = (T)0;
#pragma unroll
                    for (int h = 0; h < PMAX; ++h)
                        if (h < P) { kx += cx[h] * ps[h]; ky += cy[h] * ps[h]; }
                    const T e = sqrt(kx * kx + ky * ky + L.eps0sq[q]);
                    T r[5];
                    phonon_rates<T>(c, e, L.eps0[q], r);
                    T sum = (T)0;
#pragma unroll
                    for (int m = 0; m < 5; ++m) sum += r[m];
                    sum += edge_rate<T>(c, L.ecos, L.cedge[q], L.eps0[q], kx, ky, e);
                    smax = sum > smax ? sum : smax;
                }
                smax = group_max<T>(smax, G);
                const T Gt = c.alpha1 * smax;
                const Words wx = philox10(ctr0, a.step, (coll << 8) | kPurXi, a.instance, a.seed_lo,
                                          a.seed_hi);
                const T dtc = -dlog(uni<T>(wx.w0, wx.w1)) / Gt;   // eq. dt, node maximum
                if (!(tc + dtc < a.dt)) break;
                if (g == 0) atomicAdd(&L.cnt[SGPM_CNT_COLLISIONS], 1u);

                const Words ws = philox10(ctr0, a.step, (coll << 8) | kPurSel, a.instance, a.seed_lo,
                                          a.seed_hi);
                const T su = uni<T>(ws.w0, ws.w1), eta = uni<T>(ws.w2, ws.w3);
                const Words wa = philox10(ctr0, a.step, (coll << 8) | kPurAng, a.instance, a.seed_lo,
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

                T px_new[PMAX], py_new[PMAX];
#pragma unroll
                for (int h = 0; h < PMAX; ++h) { px_new[h] = (T)0; py_new[h] = (T)0; }
                uint32_t nev = 0, nrej = 0, nexh = 0;
                for (int q = g; q < Q; q += G) {
                    const T* ps = L.psi + q * P;
                    T kx = (T)0, ky = (T)0;
#pragma unroll
                    for (int h = 0; h < PMAX; ++h)
                        if (h < P) { kx += cx[h] * ps[h]; ky += cy[h] * ps[h]; }
                    const T e0 = L.eps0[q];
                    const T e = sqrt(kx * kx + ky * ky + L.eps0sq[q]);
                    T r[5];
                    phonon_rates<T>(c, e, e0, r);
                    int ell = 7;
                    T cum = (T)0;
#pragma unroll
                    for (int m = 0; m < 5; ++m) {
                        cum += r[m];
                        if (ell == 7 && su < cum / Gt) ell = m + 1;
                    }
                    if (ell == 7) {
                        cum += edge_rate<T>(c, L.ecos, L.cedge[q], e0, kx, ky, e);
                        if (su < cum / Gt) ell = 6;
                    }
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
                            for (uint32_t j = 0; j < (uint32_t)kEdgeTries; ++j) {
                                const Words we = philox10(ctr0, a.step, (coll << 8) | (kPurEdge0 + j),
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
                            const T f = c.pauli ? pauli_f<T>(a, L, c, q, px, py) : (T)0;
                            if (f < eta) { nx = px; ny = py; } else { ++nrej; }
                        }
                    }
                    const T* wp = L.wpsi + q * P;
#pragma unroll
                    for (int h = 0; h < PMAX; ++h)
                        if (h < P) { px_new[h] += wp[h] * nx; py_new[h] += wp[h] * ny; }
                }
                if (nev) atomicAdd(&L.cnt[SGPM_CNT_EVENTS], nev);
                if (nrej) atomicAdd(&L.cnt[SGPM_CNT_PAULI_REJ], nrej);
                if (nexh) atomicAdd(&L.cnt[SGPM_CNT_EDGE_EXH], nexh);
                // k_h = sum_q w_q Psi_h(z_q) k_q  (group sum over the nodes)
#pragma unroll
                for (int h = 0; h < PMAX; ++h) {
                    if (h < P) {
                        cx[h] = group_sum<T>(px_new[h], G);
                        cy[h] = group_sum<T>(py_new[h], G);
                    }
                }
                tc += dtc;
                ++coll;
                if (coll >= (uint32_t)c.c_max) {
                    if (g == 0) atomicAdd(&L.cnt[SGPM_CNT_CMAX], 1u);
                    break;
                }
            }
#pragma unroll
            for (int h = 0; h < PMAX; ++h)
                if (h < P && (h % G) == g) {
                    a.kx[(size_t)h * a.n + i] = cx[h];
                    a.ky[(size_t)h * a.n + i] = cy[h];
                }
        }
        // final node values: H^{n+1} cells and the pass's sums per (candidate, node)
        for (int q = g; q < Q; q += G) {
            double vx = 0.0, vy = 0.0, en = 0.0;
            if (has) {
                const T* ps = L.psi + q * P;
                T kx = (T)0, ky = (T)0;
#pragma unroll
                for (int h = 0; h < PMAX; ++h)
                    if (h < P) { kx += cx[h] * ps[h]; ky += cy[h] * ps[h]; }
                const T e = sqrt(kx * kx + ky * ky + L.eps0sq[q]);
                const T inv = (T)1 / e;
                const int r = cell_coord<T>(kx, c.lk, c.dk, c.inv_dk);
                const int l = cell_coord<T>(ky, c.lk, c.dk, c.inv_dk);
                if (r < 0 || l < 0 || r >= c.nk || l >= c.nk)
                    atomicAdd(&L.cnt[SGPM_CNT_OUT_OF_GRID], 1u);
                else
                    atomicAdd(&a.h_acc[(size_t)q * c.nk * c.nk + (size_t)r * c.nk + l], 1u);
                vx = (double)(c.v_f * kx * inv);
                vy = (double)(c.v_f * ky * inv);
                en = (double)e;
            }
            double* dst = L.pass + ((size_t)grp * Q + q) * 3;
            dst[0] = vx; dst[1] = vy; dst[2] = en;
        }
        __syncthreads();
        // running sums per node, candidates in list order
        for (int k = tid; k < Q * 3; k += kBlock) {
            const int q = k / 3, o = k % 3;
            double s = L.run[k];
            for (int gg = 0; gg < per_pass && p0 + gg < M; ++gg) s += L.pass[((size_t)gg * Q + q) * 3 + o];
            L.run[k] = s;
        }
        __syncthreads();
    }
    // add the candidates' sums to the stream workgroup's partial sums
    for (int k = tid; k < Q * 3; k += kBlock) a.partial[(size_t)wg * Q * 3 + k] += L.run[k];
    if (tid < 8 && L.cnt[tid]) atomicAdd(&a.counters[tid], (unsigned long long)L.cnt[tid]);
}

// ===================================================== K3: finalize kernel
__global__ void __launch_bounds__(kBlock) k3_finalize(const K3Args a) {
    const int q = blockIdx.x, tid = threadIdx.x;
    const size_t cells = (size_t)a.nk * a.nk;
    const uint32_t* h = a.h_acc + (size_t)q * cells;
    uint32_t* z = a.h_clr + (size_t)q * cells;
    uint32_t m = 0;
    for (size_t k = tid; k < cells; k += kBlock) {
        const uint32_t v = h[k];
        m = v > m ? v : m;
        z[k] = 0u;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const uint32_t o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    __shared__ uint32_t wm[kWaves];
    if ((tid & 63) == 0) wm[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        uint32_t mm = 0;
        for (int w = 0; w < kWaves; ++w) mm = wm[w] > mm ? wm[w] : mm;
        a.hmax_out[q] = mm;
    }
    // moment record: batch b collects the workgroups w = b (mod NB), in order
    for (int k = tid; k < a.nb * 3; k += kBlock) {
        const int b = k / 3, o = k % 3;
        double s = 0.0;
        for (int w = b; w < a.nwg; w += a.nb) s += a.partial[((size_t)w * a.Q + q) * 3 + o];
        a.record[((size_t)b * a.Q + q) * 3 + o] = s;
    }
}

// ------------------------------------------------------------ launchers
template <typename T, int PMAX, int QMAX>
static int launch_k1_t(const K1Args<T>& a, int nwg, void* stream) {
    const size_t lds = k1_lds_bytes(a.P, a.Q, sizeof(T) == 4, a.hwin_words);
    hipLaunchKernelGGL((k1_stream<T, PMAX, QMAX>), dim3(nwg), dim3(kBlock1), lds,
                       (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

template <typename T, int PMAX>
static int launch_k1_q(const K1Args<T>& a, int nwg, void* stream) {
    if (a.Q <= 1) return launch_k1_t<T, PMAX, 1>(a, nwg, stream);
    if (a.Q <= 8) return launch_k1_t<T, PMAX, 8>(a, nwg, stream);
    if (a.Q <= 16) return launch_k1_t<T, PMAX, 16>(a, nwg, stream);
    return launch_k1_t<T, PMAX, 0>(a, nwg, stream);
}

template <typename T>
static int launch_k1_any(const K1Args<T>& a, int nwg, void* stream) {
    if (a.P <= 1) return launch_k1_q<T, 1>(a, nwg, stream);
    if (a.P <= 8) return launch_k1_q<T, 8>(a, nwg, stream);
    if (a.P <= 16) return launch_k1_q<T, 16>(a, nwg, stream);
    return launch_k1_q<T, 32>(a, nwg, stream);
}

int launch_k1_f64(const K1Args<double>& a, int nwg, void* s) { return launch_k1_any<double>(a, nwg, s); }
int launch_k1_f32(const K1Args<float>& a, int nwg, void* s) { return launch_k1_any<float>(a, nwg, s); }

template <typename T>
static int launch_k2_any(const K2Args<T>& a, int nwg, void* stream) {
    const size_t lds = k2_lds_bytes(a.P, a.Q, sizeof(T) == 4);
    const dim3 grid(nwg), blk(kBlock);
    const hipStream_t s = (hipStream_t)stream;
    if (a.P <= 1) hipLaunchKernelGGL((k2_collide<T, 1>), grid, blk, lds, s, a);
    else if (a.P <= 8) hipLaunchKernelGGL((k2_collide<T, 8>), grid, blk, lds, s, a);
    else if (a.P <= 16) hipLaunchKernelGGL((k2_collide<T, 16>), grid, blk, lds, s, a);
    else hipLaunchKernelGGL((k2_collide<T, 32>), grid, blk, lds, s, a);
    return (int)hipGetLastError();
}

int launch_k2_f64(const K2Args<double>& a, int nwg, void* s) { return launch_k2_any<double>(a, nwg, s); }
int launch_k2_f32(const K2Args<float>& a, int nwg, void* s) { return launch_k2_any<float>(a, nwg, s); }

int launch_k3(const K3Args& a, void* stream) {
    hipLaunchKernelGGL(k3_finalize, dim3(a.Q), dim3(kBlock), 0, (hipStream_t)stream, a);
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
