// Device functions shared by the plain (one kernel per stage) and the fused
// (one kernel per epoch) forms of the step.  T is the storage and arithmetic
// type of HH gates, synaptic conductance and calcium: double for the FP64
// form, float for the mixed form; voltage, cable system, h, z, p are
// always double.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "sim.hpp"

namespace pa {

// --------------------------------------------------------------- Threefry
// Counter-based generator Threefry-4x64 with 12 rounds (Salmon et al. 2011,
// "Parallel random numbers: as easy as 1, 2, 3"): per round, words (0,1) and
// (2,3) are mixed by add / rotate / xor with the Threefish-256 rotation
// amounts of that round (period 8), then words 1 and 3 trade places; every
// fourth round injects the next key-schedule word set, whose fifth word is
// the xor of the key words and the parity constant 0x1BD11BDAA9FC1A22, plus
// the injection count in the last word.
__device__ __forceinline__ uint64_t rotl(uint64_t x, uint32_t r) {
    return (x << r) | (x >> (64u - r));
}

__device__ inline void threefry4x64_12(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                       uint64_t k0, uint64_t k1, uint64_t k2, uint64_t k3,
                                       uint64_t out[4]) {
    constexpr uint32_t RA[8] = {14, 52, 23, 5, 25, 46, 58, 32};
    constexpr uint32_t RB[8] = {16, 57, 40, 37, 33, 12, 22, 32};
    const uint64_t k4 = 0x1BD11BDAA9FC1A22ull ^ k0 ^ k1 ^ k2 ^ k3;
    const uint64_t ks[5] = {k0, k1, k2, k3, k4};
    uint64_t w[4] = {c0 + k0, c1 + k1, c2 + k2, c3 + k3};
#pragma unroll
    for (uint32_t inj = 1; inj <= 3; ++inj) {
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t r = (inj - 1) * 4 + j;
            // even rounds mix (w0,w1),(w2,w3); odd rounds (w0,w3),(w2,w1):
            // the same as mixing fixed pairs and swapping words 1 and 3
            uint64_t &a1 = (j & 1) ? w[3] : w[1];
            uint64_t &a3 = (j & 1) ? w[1] : w[3];
            w[0] += a1;
            a1 = rotl(a1, RA[r & 7]) ^ w[0];
            w[2] += a3;
            a3 = rotl(a3, RB[r & 7]) ^ w[2];
        }
        w[0] += ks[inj % 5];
        w[1] += ks[(inj + 1) % 5];
        w[2] += ks[(inj + 2) % 5];
        w[3] += ks[(inj + 3) % 5] + inj;
    }
    out[0] = w[0]; out[1] = w[1]; out[2] = w[2]; out[3] = w[3];
}

constexpr uint64_t NOISE_TAG = 0x5354432d6e6f6973ull;  // "STC-nois"

// Standard normal of synapse `sid` at step n: counter n/4, key (seed, sid,
// tag, 0); Box-Muller on words (0,1) for n mod 4 in {0,1} and (2,3) for
// {2,3}; cosine branch on even n, sine on odd.
__device__ inline double std_normal(uint64_t seed, uint64_t sid, uint64_t n) {
    uint64_t x[4];
    threefry4x64_12(n >> 2, 0, 0, 0, seed, sid, NOISE_TAG, 0, x);
    const uint32_t lane = (uint32_t)(n & 3);
    const uint64_t xa = (lane & 2) ? x[2] : x[0];
    const uint64_t xb = (lane & 2) ? x[3] : x[1];
    const double ua = ((double)(xa >> 11) + 0.5) * 0x1.0p-53;
    const double ub = ((double)(xb >> 11) + 0.5) * 0x1.0p-53;
    const double r = sqrt(-2.0 * log(ua));
    const double ang = 6.283185307179586 * ub;
    return (lane & 1) ? r * sin(ang) : r * cos(ang);
}

// --------------------------------------------------------------- HH rates
__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float dexp(float x) { return expf(x); }
__device__ __forceinline__ double dexpm1(double x) { return expm1(x); }
__device__ __forceinline__ float dexpm1(float x) { return expm1f(x); }

template <class T>
__device__ __forceinline__ T exprelr(T x) {
    return (x == T(0)) ? T(1) : x / dexpm1(x);
}

// Hodgkin-Huxley (1952) rates in 1/ms, rest at -65 mV, q10 factor 1.
template <class T>
__device__ __forceinline__ void hh_rates(T v, T r[6]) {
    r[0] = exprelr<T>(-(v + T(40)) / T(10));
    r[1] = T(4) * dexp(-(v + T(65)) / T(18));
    r[2] = T(0.07) * dexp(-(v + T(65)) / T(20));
    r[3] = T(1) / (dexp(-(v + T(35)) / T(10)) + T(1));
    r[4] = T(0.1) * exprelr<T>(-(v + T(55)) / T(10));
    r[5] = T(0.125) * dexp(-(v + T(65)) / T(80));
}

// Exact exponential integration of the three gates at the new voltage.
template <class T>
__device__ inline void gate_update(const DevNet &d, uint32_t k, double vnew) {
    T *gm = (T *)d.gm, *gh = (T *)d.gh, *gn = (T *)d.gn;
    const T v = (T)vnew;
    const T dt = (T)d.dt;
    T r[6];
    hh_rates<T>(v, r);
    T *x[3] = {gm + k, gh + k, gn + k};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const T a = r[2 * j], b = r[2 * j + 1];
        const T xinf = a / (a + b);
        *x[j] = xinf + (*x[j] - xinf) * dexp(-dt * (a + b));
    }
}

// --------------------------------------------------------------- flags
__device__ inline void raise_flag(const DevNet &d, uint32_t flag, uint32_t cell) {
    uint32_t old = atomicOr(&d.ctr->flags, flag);
    if (old == 0) d.ctr->bad_cell = cell;
}

// --------------------------------------------------------------- events
// Appends event e for delivery at step s to the ring of `cell`; steps before
// `min_step` are in the past (epoch already running) and raise FLAG_LATE.
__device__ inline void push_event(const DevNet &d, uint32_t cell, uint64_t s, const Event &e,
                                  uint64_t min_step) {
    if (s < min_step) {
        raise_flag(d, FLAG_LATE, cell);
        return;
    }
    if (s >= min_step + d.R - d.K) {
        raise_flag(d, FLAG_OVERFLOW, cell);
        return;
    }
    const uint32_t slot = (uint32_t)(s % d.R);
    const uint64_t ring = (uint64_t)cell * d.R + slot;
    const uint32_t pos = atomicAdd(&d.ev_n[ring], 1u);
    if (pos < d.Q) d.ev[ring * d.Q + pos] = e;
    else raise_flag(d, FLAG_OVERFLOW, cell);
}

__device__ __forceinline__ bool ev_before(const Event &a, const Event &b) {
    if (a.t != b.t) return a.t < b.t;
    if (a.src != b.src) return a.src < b.src;
    if (a.conn != b.conn) return a.conn < b.conn;
    return a.port < b.port;
}

// Applies one event to its synapse.
template <class T>
__device__ __forceinline__ void apply_event(const DevNet &d, const Event &e, uint64_t n) {
    const uint32_t s = e.syn;
    if (e.port == 1) {
        T *g = (T *)d.g;
        if (d.syn_kind[s] == 1) {
            const double h0 = d.stc.h0;
            g[s] = g[s] + (T)(e.w * ((d.h[s] + h0 * d.z[s]) / h0));
        } else {
            g[s] = g[s] + (T)e.w;
        }
    } else {
        T *c = (T *)d.c;
        c[s] = c[s] + (T)d.stc.c_pre;
    }
    d.ev_cnt[2 * s + e.port - 1] += 1ull;
    d.ev_sum[2 * s + e.port - 1] += (unsigned long long)n;
}

// Delivers the events of step n of one cell in (t_e, src, conn, port)
// order, then the post-synaptic hook of a spike in the previous step.
template <class T>
__device__ inline void deliver_cell(const DevNet &d, uint32_t cell, uint64_t n) {
    const uint64_t ring = (uint64_t)cell * d.R + (uint32_t)(n % d.R);
    uint32_t cnt = d.ev_n[ring];
    if (cnt) {
        if (cnt > d.Q) cnt = d.Q;  // overflow was flagged at insertion
        Event *ev = d.ev + ring * d.Q;
        // insertion sort in place; slots hold few events
        for (uint32_t i = 1; i < cnt; ++i) {
            Event x = ev[i];
            uint32_t j = i;
            while (j > 0 && ev_before(x, ev[j - 1])) {
                ev[j] = ev[j - 1];
                --j;
            }
            ev[j] = x;
        }
        for (uint32_t i = 0; i < cnt; ++i) apply_event<T>(d, ev[i], n);
        d.ev_n[ring] = 0;
        atomicAdd((unsigned long long *)&d.ctr->events, (unsigned long long)cnt);
    }
    if (d.post[cell]) {
        T *c = (T *)d.c;
        const T cp = (T)d.stc.c_post;
        for (uint32_t s = d.syn_off[cell]; s < d.syn_off[cell + 1]; ++s)
            if (d.syn_kind[s] == 1) c[s] = c[s] + cp;
        d.post[cell] = 0;
    }
}

// --------------------------------------------------------------- currents
// Membrane current (nA, outward positive) and dI/dV (uS) of CV i at V^n:
// HH, synapses in (CV, id) order, then clamps active at t_n.
template <class T>
__device__ inline void cv_current(const DevNet &d, uint32_t i, double v, double tn, double &Iout,
                                  double &Gout) {
    double I = 0.0, G = 0.0;
    const int32_t k = d.hh_of[i];
    if (k >= 0) {
        const double *P = d.hh_par + 6 * (size_t)k;
        const double m = (double)((const T *)d.gm)[k];
        const double hh = (double)((const T *)d.gh)[k];
        const double nn = (double)((const T *)d.gn)[k];
        const double gna = P[0] * m * m * m * hh;
        const double gk = P[1] * nn * nn * nn * nn;
        const double idens = gna * (v - P[3]) + gk * (v - P[4]) + P[2] * (v - P[5]);
        const double sc = d.hh_scale[k];
        I = sc * idens;
        G = sc * (gna + gk + P[2]);
    }
    const T *g = (const T *)d.g;
    for (uint32_t q = d.cv_syn_off[i]; q < d.cv_syn_off[i + 1]; ++q) {
        const double gs = (double)g[q];
        I += gs * (v - d.syn_erev[q]);
        G += gs;
    }
    for (uint32_t q = d.cv_cl_off[i]; q < d.cv_cl_off[i + 1]; ++q) {
        if (d.cl_t0[q] <= tn && tn < d.cl_t0[q] + d.cl_dur[q]) I -= d.cl_amp[q];
    }
    Iout = I;
    Gout = G;
}

// --------------------------------------------------------------- synapses
// Conductance decay, then for tagging-and-capture synapses one step of
// Eqs. 17-20 from step-start h, z, c and the cell's step-start p.
template <class T>
__device__ inline void syn_update(const DevNet &d, uint32_t s, uint64_t n, double p) {
    T *g = (T *)d.g;
    if constexpr (sizeof(T) == 8) g[s] = g[s] * (T)d.syn_decay[s];
    else g[s] = g[s] * d.syn_decay_f[s];
    if (d.syn_kind[s] != 1) return;
    T *cp = (T *)d.c;
    const Stc &P = d.stc;
    const T c = cp[s];
    const double h = d.h[s], z = d.z[s], h0 = P.h0;
    const double thp = (c - (T)P.theta_p > T(0)) ? 1.0 : 0.0;
    const double thd = (c - (T)P.theta_d > T(0)) ? 1.0 : 0.0;
    const double ah = d.dt / P.tau_h;
    const double drift = 0.1 * (h0 - h) + P.gamma_p * (10.0 - h) * thp - P.gamma_d * h * thd;
    double hn = h + ah * drift;
    if (thp + thd > 0.0)
        hn += P.sigma_pl * sqrt((thp + thd) * ah) * std_normal(d.seed, d.syn_sid[s], n);
    const double tagp = ((h - h0) - P.theta_tag > 0.0) ? 1.0 : 0.0;
    const double tagd = ((h0 - h) - P.theta_tag > 0.0) ? 1.0 : 0.0;
    const double az = d.dt / P.tau_z;
    const double zn = z + az * p * P.f_int * ((1.0 - z) * tagp - (z + 0.5) * tagd);
    d.h[s] = hn;
    d.z[s] = zn;
    if constexpr (sizeof(T) == 8) cp[s] = c * (T)d.r_c;
    else cp[s] = c * d.r_c_f;
}

// --------------------------------------------------------------- cells
__device__ inline void prp_update(const DevNet &d, uint32_t cell) {
    const double ap = d.dt / d.stc.tau_p;
    const double trig = (d.S[cell] - d.stc.theta_pro > 0.0) ? 1.0 : 0.0;
    const double p = d.p[cell];
    d.p[cell] = p + ap * (-p + d.stc.p_max * trig);
}

// Threshold crossing V^n < theta <= V^{n+1}: records the spike with the
// linearly interpolated time and arms the post-synaptic hook.
__device__ inline void detect(const DevNet &d, uint32_t cell, uint64_t n, double v0, double v1) {
    if (!(v0 < d.theta && v1 >= d.theta)) return;
    const double tn = (double)n * d.dt;
    const double ts = tn + d.dt * ((d.theta - v0) / (v1 - v0));
    const uint32_t pos = atomicAdd(&d.ctr->ep_n, 1u);
    d.ep_gid[pos] = cell;
    d.ep_step[pos] = (uint32_t)n;
    d.ep_t[pos] = ts;
    d.post[cell] = 1;
}

}  // namespace pa
