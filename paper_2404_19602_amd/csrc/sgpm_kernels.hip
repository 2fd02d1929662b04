// gfx950 kernels of the sG-PM hot path (arXiv:2404.19602, Algorithm 2).
//
// One launch of step_kernel advances one instance by one time step:
//   - Galerkin drift of the coefficients (Sec. 4.1, electric forcing),
//   - evaluation of k_i(z_q) at the Gauss nodes (eq. gPC),
//   - collision decision: a rigorous upper bound of the node-maximum rate
//     clears most particles without the exact rates (eq. deltat); the rest
//     are compacted into an LDS queue and run the exact collision loop
//     (mechanism selection eq. update_gPC, final states, Pauli acceptance
//     eq. Pauli_gPC against H^n on the moved grid, projection eq. update_sG),
//   - the histogram H^{n+1} of every node (eq. f_gPC) through a privatised
//     LDS window flushed with global atomics, the per-node maximum through
//     atomicMax of the values the atomics return,
//   - FP64 per-node sums of v_x, v_y and the energy (Sec. 4.2), reduced in a
//     fixed order by the last workgroup into the moment record,
//   - clearing of the stale histogram buffer for the next step.
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

template <typename T> struct Consts;
template <> struct Consts<double> {
    static constexpr double two_pi = 6.283185307179586476925286766559;
    static constexpr double trap = 6.283185307179586476925286766559 / kEdgePts;
};
template <> struct Consts<float> {
    static constexpr float two_pi = 6.28318530717958647692f;
    static constexpr float trap = 6.28318530717958647692f / kEdgePts;
};

__device__ __forceinline__ double dlog(double x) { return log(x); }
__device__ __forceinline__ float dlog(float x) { return logf(x); }
__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float dexp(float x) { return expf(x); }
__device__ __forceinline__ void dsincospi(double x, double* s, double* c) { sincospi(x, s, c); }
__device__ __forceinline__ void dsincospi(float x, float* s, float* c) { sincospif(x, s, c); }

// Cell index floor((x + L)/dk) exactly as the quotient is rounded: the cheap
// product by 1/dk is corrected by a true division only when it lies within
// a few ulps of an integer.
template <typename T>
__device__ __forceinline__ int cell_coord(T x, T L, T dk, T inv_dk) {
    const T s = x + L;
    T qt = s * inv_dk;
    const T r = rint(qt);
    if (fabs(qt - r) <= (T)8 * (T)(sizeof(T) == 8 ? 2.220446049250313e-16 : 1.1920929e-07) * fabs(qt) +
                             (T)1e-30)
        qt = s / dk;
    const T f = floor(qt);
    // outside the grid (including NaN) maps to -1
    return (f >= (T)0 && f < (T)1e9) ? (int)f : -1;
}

// ------------------------------------------------------------ wave sums
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------- rates
// The five closed-form phonon rates (Appendix) at energy e of node q, in the
// order AC, OP-, OP+, K-, K+.
template <typename T>
__device__ __forceinline__ void phonon_rates(const StepArgs<T>& a, T e, T e0, T r[5]) {
    r[0] = (e - e0 >= (T)0) ? a.c_ac * e : (T)0;
    const T eom = e - a.hw_o, eop = e + a.hw_o, ekm = e - a.hw_k, ekp = e + a.hw_k;
    r[1] = (eom - e0 >= (T)0) ? a.c_om * eom : (T)0;
    r[2] = (eop - e0 >= (T)0) ? a.c_op * eop : (T)0;
    r[3] = (ekm - e0 >= (T)0) ? a.c_km * ekm : (T)0;
    r[4] = (ekp - e0 >= (T)0) ? a.c_kp * ekp : (T)0;
}

// Edge rate: cedge_q * eps * int_0^{2pi} exp(-kap (cos t - c)^2) dt by the
// 32-point trapezoid rule, summed with the symmetry cos(t_j) = cos(t_{32-j}).
template <typename T>
__device__ __forceinline__ T edge_rate(const StepArgs<T>& a, int q, T kx, T ky, T e) {
    const T k2 = kx * kx + ky * ky;
    const T kabs = sqrt(k2);
    const T c = kabs > (T)0 ? kx / kabs : (T)1;
    const T kap = a.edge_kap * k2;
    const T* cs = a.tab.edge_cos;
    T d0 = cs[0] - c, d16 = cs[kEdgePts / 2] - c;
    T acc = dexp(-kap * d0 * d0) + dexp(-kap * d16 * d16);
    T mid = (T)0;
#pragma unroll
    for (int j = 1; j < kEdgePts / 2; ++j) {
        const T d = cs[j] - c;
        mid += dexp(-kap * d * d);
    }
    acc += (T)2 * mid;
    const T e0 = a.tab.eps0[q];
    return (e - e0 >= (T)0) ? a.tab.cedge[q] * e * (acc * Consts<T>::trap) : (T)0;
}

// Upper bound of max_q sum_nu Gamma^nu given the largest nodal energy: every
// rate is non-decreasing in the energy, the angular edge integral is at most
// 2 pi, and emission thresholds use the smallest band minimum.
template <typename T>
__device__ __forceinline__ T rate_bound(const StepArgs<T>& a, T emax) {
    T s = a.b_ac * emax + a.b_op * (emax + a.hw_o) + a.b_kp * (emax + a.hw_k) + a.b_edge * emax;
    if (emax >= a.b_thr_o) s += a.b_om * (emax - a.hw_o);
    if (emax >= a.b_thr_k) s += a.b_km * (emax - a.hw_k);
    return a.alpha1 * s * a.b_margin;
}

// --------------------------------------------------------- LDS layout
struct Lds {
    uint32_t* hwin;     // packed 16-bit counters of the histogram window
    int* queue;         // candidate particles (offset within the chunk)
    double* macc;       // [waves][Q][3] moment sums
    uint32_t* wgmax;    // [Q]
    uint32_t* cnt;      // [8] counters + [8] queue length
};

__host__ __device__ inline size_t lds_offsets(int Q, int hwin_words, size_t* o_queue,
                                              size_t* o_macc, size_t* o_wgmax, size_t* o_cnt) {
    size_t off = (size_t)hwin_words * 4;
    off = (off + 15) & ~(size_t)15;
    *o_queue = off;
    off += (size_t)kQueueCap * 4;
    off = (off + 15) & ~(size_t)15;
    *o_macc = off;
    off += (size_t)kWaves * Q * 3 * 8;
    *o_wgmax = off;
    off += (size_t)Q * 4;
    off = (off + 15) & ~(size_t)15;
    *o_cnt = off;
    off += 16 * 4;
    return off;
}

size_t step_lds_bytes(int Q, int hwin_words) {
    size_t a, b, c, d;
    return lds_offsets(Q, hwin_words, &a, &b, &c, &d);
}

// Bin one nodal value into the histogram of node q, and account the moments.
template <typename T>
__device__ __forceinline__ void bin_value(const StepArgs<T>& a, const Lds& s, int q, T kx, T ky) {
    const int r = cell_coord<T>(kx, a.lk, a.dk, a.inv_dk);
    const int l = cell_coord<T>(ky, a.lk, a.dk, a.inv_dk);
    if (r < 0 || l < 0 || r >= a.nk || l >= a.nk) {
        atomicAdd(&s.cnt[SGPM_CNT_OUT_OF_GRID], 1u);
        return;
    }
    const int wr = r - a.win_r0, wl = l - a.win_l0;
    if (wr >= 0 && wr < a.win && wl >= 0 && wl < a.win) {
        const int idx = (q * a.win + wr) * a.win + wl;
        atomicAdd(&s.hwin[idx >> 1], (idx & 1) ? 65536u : 1u);
    } else {
        const uint32_t old = atomicAdd(&a.h_acc[(size_t)q * a.nk * a.nk + (size_t)r * a.nk + l], 1u);
        atomicMax(&s.wgmax[q], old + 1u);
    }
}

// Evaluate the nodes of one particle's coefficients and add its nodal
// values to the histogram and to the per-wave moment sums.  Must be called
// by every lane of the wave (active = false contributes nothing).
template <typename T, int PMAX>
__device__ __forceinline__ void finalize_particle(const StepArgs<T>& a, const Lds& s,
                                                  const T (&cx)[PMAX], const T (&cy)[PMAX],
                                                  bool active) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = 0; q < a.Q; ++q) {
        const T* ps = a.tab.psi + q * a.P;
        T kx = (T)0, ky = (T)0;
#pragma unroll
        for (int h = 0; h < PMAX; ++h)
            if (h < a.P) { kx += cx[h] * ps[h]; ky += cy[h] * ps[h]; }
        double vx = 0.0, vy = 0.0, en = 0.0;
        if (active) {
            const T e = sqrt(kx * kx + ky * ky + a.tab.eps0sq[q]);
            vx = (double)(a.v_f * kx / e);
            vy = (double)(a.v_f * ky / e);
            en = (double)e;
            bin_value<T>(a, s, q, kx, ky);
        }
        vx = wave_sum(vx); vy = wave_sum(vy); en = wave_sum(en);
        if (lane == 0) {
            double* m = s.macc + ((size_t)wave * a.Q + q) * 3;
            m[0] += vx; m[1] += vy; m[2] += en;
        }
    }
}

template <typename T, int PMAX>
__device__ __forceinline__ void load_drift(const StepArgs<T>& a, int64_t i, T (&cx)[PMAX],
                                           T (&cy)[PMAX]) {
#pragma unroll
    for (int h = 0; h < PMAX; ++h) {
        if (h < a.P) {
            cx[h] = a.kx[(size_t)h * a.n + i];
            cy[h] = a.ky[(size_t)h * a.n + i];
            if (a.do_drift) cx[h] -= a.drift[h];   // k_h^{n+1} = k_h^n - (e/hbar) dt E_h
        } else {
            cx[h] = (T)0; cy[h] = (T)0;
        }
    }
}

// Pauli occupation f = H^n / max H^n at the candidate's cell on the grid
// moved with this step's drift (lookup at k' + v_F E(z_q) dt x^).
template <typename T>
__device__ __forceinline__ T pauli_f(const StepArgs<T>& a, int q, T px, T py) {
    const uint32_t mx = a.hmax_read[q];
    if (mx == 0u) return (T)0;
    const T shift = a.tab.vfield[q] * a.dt;
    const int r = cell_coord<T>(px + shift, a.lk, a.dk, a.inv_dk);
    const int l = cell_coord<T>(py, a.lk, a.dk, a.inv_dk);
    if (r < 0 || l < 0 || r >= a.nk || l >= a.nk) return (T)0;
    const uint32_t h = a.h_read[(size_t)q * a.nk * a.nk + (size_t)r * a.nk + l];
    return (T)h / (T)mx;
}

// Exact collision loop of one particle (Algorithm 2 inner while-loop); the
// coefficients (already drifted) are updated in place.
template <typename T, int PMAX>
__device__ void collide(const StepArgs<T>& a, const Lds& s, int64_t i, T (&cx)[PMAX],
                        T (&cy)[PMAX]) {
    T tc = (T)0;
    uint32_t c = 0;
    const uint32_t ctr0 = (uint32_t)i;
    for (;;) {
        // Gamma~ = (1 + alpha) max_q sum_nu Gamma^nu(z_q)
        T smax = (T)0;
        for (int q = 0; q < a.Q; ++q) {
            const T* ps = a.tab.psi + q * a.P;
            T kx = (T)0, ky = (T)0;
#pragma unroll
            for (int h = 0; h < PMAX; ++h)
                if (h < a.P) { kx += cx[h] * ps[h]; ky += cy[h] * ps[h]; }
            const T e = sqrt(kx * kx + ky * ky + a.tab.eps0sq[q]);
            T r[5];
            phonon_rates<T>(a, e, a.tab.eps0[q], r);
            T sum = (T)0;
#pragma unroll
            for (int m = 0; m < 5; ++m) sum += r[m];
            sum += edge_rate<T>(a, q, kx, ky, e);
            smax = sum > smax ? sum : smax;
        }
        const T G = a.alpha1 * smax;
        const Words wx = philox10(ctr0, a.step, (c << 8) | kPurXi, a.instance, a.seed_lo, a.seed_hi);
        const T xi = uni<T>(wx.w0, wx.w1);
        const T dtc = -dlog(xi) / G;            // free flight, eq. dt with the node maximum
        if (!(tc + dtc < a.dt)) break;
        atomicAdd(&s.cnt[SGPM_CNT_COLLISIONS], 1u);

        const Words ws = philox10(ctr0, a.step, (c << 8) | kPurSel, a.instance, a.seed_lo, a.seed_hi);
        const T su = uni<T>(ws.w0, ws.w1), eta = uni<T>(ws.w2, ws.w3);
        const Words wa = philox10(ctr0, a.step, (c << 8) | kPurAng, a.instance, a.seed_lo, a.seed_hi);
        const T u1 = uni<T>(wa.w0, wa.w1), u2 = uni<T>(wa.w2, wa.w3);
        // AC angle: twice the polar angle of a uniform point of the unit disk
        // centred at (1,0) (density 1 + cos); cos/sin by the double angle.
        T s_phi, c_phi;
        dsincospi((T)2 * u2, &s_phi, &c_phi);
        const T rr = sqrt(u1);
        const T dx = (T)1 + rr * c_phi, dy = rr * s_phi;
        const T n2 = dx * dx + dy * dy;
        const T cac = (dx * dx - dy * dy) / n2, sac = ((T)2 * dx * dy) / n2;
        T sop, cop;
        dsincospi((T)2 * u1, &sop, &cop);       // OP angle 2 pi u1

        T ax[PMAX], ay[PMAX];
#pragma unroll
        for (int h = 0; h < PMAX; ++h) { ax[h] = (T)0; ay[h] = (T)0; }
        uint32_t nev = 0, nrej = 0, nexh = 0;
        for (int q = 0; q < a.Q; ++q) {
            const T* ps = a.tab.psi + q * a.P;
            T kx = (T)0, ky = (T)0;
#pragma unroll
            for (int h = 0; h < PMAX; ++h)
                if (h < a.P) { kx += cx[h] * ps[h]; ky += cy[h] * ps[h]; }
            const T e0 = a.tab.eps0[q];
            const T e = sqrt(kx * kx + ky * ky + a.tab.eps0sq[q]);
            T r[5];
            phonon_rates<T>(a, e, e0, r);
            int ell = 7;
            T cum = (T)0;
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                cum += r[m];
                if (ell == 7 && su < cum / G) ell = m + 1;
            }
            if (ell == 7) {
                cum += edge_rate<T>(a, q, kx, ky, e);
                if (su < cum / G) ell = 6;
            }
            T nx = kx, ny = ky;
            if (ell != 7) {
                const T kabs = sqrt(kx * kx + ky * ky);
                const T cin = kabs > (T)0 ? kx / kabs : (T)1;
                const T sin_ = kabs > (T)0 ? ky / kabs : (T)0;
                T px, py;
                bool ok = true;
                if (ell == 6) {
                    // absolute final angle, density exp(-kap (cos t' - cos t_in)^2)
                    const T kap = a.edge_kap * (kx * kx + ky * ky);
                    ok = false;
                    for (uint32_t j = 0; j < (uint32_t)kEdgeTries; ++j) {
                        const Words we = philox10(ctr0, a.step, (c << 8) | (kPurEdge0 + j),
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
                        const T hw = op ? a.hw_o : a.hw_k;
                        const T de = (ell == 2 || ell == 4) ? -hw : hw;
                        if (op) { ct = cop; st = sop; } else { ct = -cac; st = -sac; }
                        if (a.final_state == 1) {
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
                    const T f = a.pauli ? pauli_f<T>(a, q, px, py) : (T)0;
                    if (f < eta) { nx = px; ny = py; } else { ++nrej; }
                }
            }
            const T* wp = a.tab.wpsi + q * a.P;
#pragma unroll
            for (int h = 0; h < PMAX; ++h)
                if (h < a.P) { ax[h] += wp[h] * nx; ay[h] += wp[h] * ny; }
        }
        if (nev) atomicAdd(&s.cnt[SGPM_CNT_EVENTS], nev);
        if (nrej) atomicAdd(&s.cnt[SGPM_CNT_PAULI_REJ], nrej);
        if (nexh) atomicAdd(&s.cnt[SGPM_CNT_EDGE_EXH], nexh);
#pragma unroll
        for (int h = 0; h < PMAX; ++h) { cx[h] = ax[h]; cy[h] = ay[h]; }
        tc += dtc;
        ++c;
        if (c >= (uint32_t)a.c_max) { atomicAdd(&s.cnt[SGPM_CNT_CMAX], 1u); break; }
    }
}

// Run the exact collision loop on the first m queued candidates, one per lane.
template <typename T, int PMAX>
__device__ void process_queue(const StepArgs<T>& a, const Lds& s, int64_t begin, int m) {
    const int tid = threadIdx.x;
    const bool has = tid < m;
    const int64_t i = has ? begin + s.queue[tid] : begin;
    T cx[PMAX], cy[PMAX];
    load_drift<T, PMAX>(a, i, cx, cy);
    if (has) {
        collide<T, PMAX>(a, s, i, cx, cy);
#pragma unroll
        for (int h = 0; h < PMAX; ++h)
            if (h < a.P) { a.kx[(size_t)h * a.n + i] = cx[h]; a.ky[(size_t)h * a.n + i] = cy[h]; }
    }
    finalize_particle<T, PMAX>(a, s, cx, cy, has);
}

template <typename T, int PMAX>
__global__ void __launch_bounds__(kBlock) step_kernel(const StepArgs<T> a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    size_t oq, om, ow, oc;
    lds_offsets(a.Q, a.hwin_words, &oq, &om, &ow, &oc);
    Lds s;
    s.hwin = reinterpret_cast<uint32_t*>(smem);
    s.queue = reinterpret_cast<int*>(smem + oq);
    s.macc = reinterpret_cast<double*>(smem + om);
    s.wgmax = reinterpret_cast<uint32_t*>(smem + ow);
    s.cnt = reinterpret_cast<uint32_t*>(smem + oc);
    uint32_t* qlen = s.cnt + 8;
    const int tid = threadIdx.x;

    for (int w = tid; w < a.hwin_words; w += kBlock) s.hwin[w] = 0u;
    for (int w = tid; w < kWaves * a.Q * 3; w += kBlock) s.macc[w] = 0.0;
    for (int w = tid; w < a.Q; w += kBlock) s.wgmax[w] = 0u;
    if (tid < 16) s.cnt[tid] = 0u;

    // clear the stale histogram buffer (it accumulates the next step)
    {
        uint4* hc = reinterpret_cast<uint4*>(a.h_clr);
        const uint4 z = make_uint4(0u, 0u, 0u, 0u);
        for (int64_t k = (int64_t)blockIdx.x * kBlock + tid; k < a.clear_vec4;
             k += (int64_t)gridDim.x * kBlock)
            hc[k] = z;
        if (blockIdx.x == 0)
            for (int w = tid; w < a.Q; w += kBlock) a.hmax_clr[w] = 0u;
    }
    __syncthreads();

    const int64_t begin = (int64_t)blockIdx.x * a.chunk;
    const int64_t end = begin + a.chunk < a.n ? begin + a.chunk : a.n;
    const T vdt_margin = a.dt;

    for (int64_t base = begin; base < end; base += kBlock) {
        const int64_t i = base + tid;
        const bool act = i < end;
        T cx[PMAX], cy[PMAX];
        load_drift<T, PMAX>(a, act ? i : begin, cx, cy);
        bool cand = false;
        if (act && a.do_collide) {
            // largest nodal energy -> rigorous rate bound -> can this particle
            // collide in this step at all?  (no collision iff -log xi / G >= dt)
            T e2max = (T)0;
            for (int q = 0; q < a.Q; ++q) {
                const T* ps = a.tab.psi + q * a.P;
                T kx = (T)0, ky = (T)0;
#pragma unroll
                for (int h = 0; h < PMAX; ++h)
                    if (h < a.P) { kx += cx[h] * ps[h]; ky += cy[h] * ps[h]; }
                const T e2 = kx * kx + ky * ky + a.tab.eps0sq[q];
                e2max = e2 > e2max ? e2 : e2max;
            }
            const T gb = rate_bound<T>(a, sqrt(e2max));
            const Words wx = philox10((uint32_t)i, a.step, kPurXi, a.instance, a.seed_lo, a.seed_hi);
            const T xlog = -dlog(uni<T>(wx.w0, wx.w1));
            cand = !(xlog >= gb * vdt_margin);
        }
        if (act && !cand && a.do_drift) {
#pragma unroll
            for (int h = 0; h < PMAX; ++h)
                if (h < a.P && ((a.drift_mask >> h) & 1u)) a.kx[(size_t)h * a.n + i] = cx[h];
        }
        finalize_particle<T, PMAX>(a, s, cx, cy, act && !cand);
        if (cand) {
            const uint32_t slot = atomicAdd(qlen, 1u);
            s.queue[slot] = (int)(i - begin);
            atomicAdd(&s.cnt[SGPM_CNT_CANDIDATES], 1u);
        }
        __syncthreads();
        const int pending = (int)*qlen;
        if (pending >= kBlock) {
            process_queue<T, PMAX>(a, s, begin, kBlock);
            const int rest = pending - kBlock;
            int moved = 0;
            if (tid < rest) moved = s.queue[kBlock + tid];
            __syncthreads();
            if (tid < rest) s.queue[tid] = moved;
            if (tid == 0) *qlen = (uint32_t)rest;
        }
        __syncthreads();
    }
    {
        const int pending = (int)*qlen;
        if (pending > 0) process_queue<T, PMAX>(a, s, begin, pending);
    }
    __syncthreads();

    // flush the LDS window: nonzero cells to global atomics, track the max
    {
        const int wcells = a.win * a.win;
        for (int w = tid; w < a.hwin_words; w += kBlock) {
            const uint32_t v = s.hwin[w];
            if (v == 0u) continue;
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const uint32_t cnt = half ? (v >> 16) : (v & 0xFFFFu);
                if (cnt == 0u) continue;
                const int idx = 2 * w + half;
                const int q = idx / wcells, rem = idx - q * wcells;
                const int r = a.win_r0 + rem / a.win, l = a.win_l0 + rem % a.win;
                const uint32_t old =
                    atomicAdd(&a.h_acc[(size_t)q * a.nk * a.nk + (size_t)r * a.nk + l], cnt);
                atomicMax(&s.wgmax[q], old + cnt);
            }
        }
    }
    __syncthreads();
    for (int q = tid; q < a.Q; q += kBlock)
        if (s.wgmax[q]) atomicMax(&a.hmax_acc[q], s.wgmax[q]);
    if (tid < 8 && s.cnt[tid]) atomicAdd(&a.counters[tid], (unsigned long long)s.cnt[tid]);

    // per-workgroup moment partials, then the last workgroup reduces them in
    // a fixed order into the batches of the record
    for (int k = tid; k < a.Q * 3; k += kBlock) {
        double v = 0.0;
        for (int wv = 0; wv < kWaves; ++wv) v += s.macc[wv * a.Q * 3 + k];
        a.partial[(size_t)blockIdx.x * a.Q * 3 + k] = v;
    }
    __threadfence();
    __syncthreads();
    __shared__ int is_last;
    if (tid == 0) is_last = (atomicAdd(a.done, 1u) == (uint32_t)(gridDim.x - 1));
    __syncthreads();
    if (is_last) {
        __threadfence();
        const int per = a.Q * 3;
        for (int k = tid; k < a.nb * per; k += kBlock) {
            const int b = k / per, rem = k - b * per;
            double v = 0.0;
            for (int w = b; w < (int)gridDim.x; w += a.nb)
                v += __hip_atomic_load(&a.partial[(size_t)w * per + rem], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            a.record[k] = v;
        }
        if (tid == 0) *a.done = 0u;
    }
}

template <typename T, int PMAX>
static int launch_step_t(const StepArgs<T>& a, void* stream) {
    const size_t lds = step_lds_bytes(a.Q, a.hwin_words);
    hipLaunchKernelGGL((step_kernel<T, PMAX>), dim3(a.nwg), dim3(kBlock), lds,
                       (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_step_f64(const StepArgs<double>& a, int pmax, void* stream) {
    if (pmax <= 1) return launch_step_t<double, 1>(a, stream);
    if (pmax <= 4) return launch_step_t<double, 4>(a, stream);
    if (pmax <= 8) return launch_step_t<double, 8>(a, stream);
    if (pmax <= 16) return launch_step_t<double, 16>(a, stream);
    return launch_step_t<double, 32>(a, stream);
}

int launch_step_f32(const StepArgs<float>& a, int pmax, void* stream) {
    if (pmax <= 1) return launch_step_t<float, 1>(a, stream);
    if (pmax <= 4) return launch_step_t<float, 4>(a, stream);
    if (pmax <= 8) return launch_step_t<float, 8>(a, stream);
    if (pmax <= 16) return launch_step_t<float, 16>(a, stream);
    return launch_step_t<float, 32>(a, stream);
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
    // panel j with lo[j] <= target < lo[j+1]  (or hi[j+1] <= target < hi[j])
    int j0 = 0, j1 = np - 1;
    while (j0 < j1) {
        const int mid = (j0 + j1 + 1) >> 1;
        const bool right = upper ? (hi[mid] > target) : (lo[mid] <= target);
        if (right) j0 = mid; else j1 = mid - 1;
    }
    const int j = j0;
    double xa = e0 + j * a.cdf_h, xb = e0 + (j + 1) * a.cdf_h;
    double ba = xa, bb = xb;      // bracket
    double fracv = upper ? (hi[j] - target) / (hi[j] - hi[j + 1]) : (target - lo[j]) / (lo[j + 1] - lo[j]);
    fracv = fmin(fmax(fracv, 0.0), 1.0);
    double e = xa + fracv * (xb - xa);
    for (int it = 0; it < 60; ++it) {
        const double F = upper ? target - (fd_panel(a, e, xb) + hi[j + 1])
                               : (lo[j] + fd_panel(a, xa, e)) - target;   // increasing in e
        if (F > 0.0) bb = e; else ba = e;
        const double g = fd_w(e, a.mu, a.kT);
        double en = (g > 0.0) ? e - F / g : 0.5 * (ba + bb);
        if (!(en > ba && en < bb)) en = 0.5 * (ba + bb);
        if (en == e || bb - ba <= 0.0) break;
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
