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
// 64-bit left rotation by a constant r in (0, 64) as two 32-bit funnel
// shifts of the halves (v_alignbit), instead of two 64-bit shifts and ors.
__device__ __forceinline__ uint64_t rotl(uint64_t x, uint32_t r) {
    const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    uint32_t nhi, nlo;
    if (r == 32) {
        nhi = lo;
        nlo = hi;
    } else if (r < 32) {
        nhi = __builtin_amdgcn_alignbit(hi, lo, 32u - r);
        nlo = __builtin_amdgcn_alignbit(lo, hi, 32u - r);
    } else {
        nhi = __builtin_amdgcn_alignbit(lo, hi, 64u - r);
        nlo = __builtin_amdgcn_alignbit(hi, lo, 64u - r);
    }
    return ((uint64_t)nhi << 32) | nlo;
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

// The early-phase noise increment sigma sqrt((Theta_p + Theta_d) dt / tau_h) N
// of synapse s at step n; out of line, as it is needed only while calcium
// is above a threshold.
static __device__ __attribute__((noinline)) double noise_increment(uint64_t seed, uint64_t sid, uint64_t n, double sigma,
                                                           double th, double ah) {
    return sigma * sqrt(th * ah) * std_normal(seed, sid, n);
}

// The mixed form's normal: the same Threefry words, lane choice and
// Box-Muller branch, with the uniforms' top 24 bits and the logarithm,
// square root and sine or cosine in FP32 (the hardware's approximations);
// it differs from the FP64 normal by FP32 rounding, far below the noise's
// own scale in the FP64 early-phase weight.
__device__ __forceinline__ float std_normal_f32(uint64_t seed, uint64_t sid, uint64_t n) {
    uint64_t x[4];
    threefry4x64_12(n >> 2, 0, 0, 0, seed, sid, NOISE_TAG, 0, x);
    const uint32_t lane = (uint32_t)(n & 3);
    const uint64_t xa = (lane & 2) ? x[2] : x[0];
    const uint64_t xb = (lane & 2) ? x[3] : x[1];
    const float ua = ((float)(uint32_t)(xa >> 40) + 0.5f) * 0x1.0p-24f;
    const float ub = ((float)(uint32_t)(xb >> 40) + 0.5f) * 0x1.0p-24f;
    const float r = __fsqrt_rn(-2.0f * __logf(ua));
    const float ang = 6.28318530717958648f * ub;
    return (lane & 1) ? r * __sinf(ang) : r * __cosf(ang);
}

// The mixed form's increment sigma sqrt((Theta_p + Theta_d) dt / tau_h) N
// with the factor, like the normal, in FP32.
__device__ __forceinline__ double noise_f32(uint64_t seed, uint64_t sid, uint64_t n, double sigma, double th,
                                            double ah) {
    const float k = (float)sigma * __fsqrt_rn((float)(th * ah));
    return (double)(k * std_normal_f32(seed, sid, n));
}

static __device__ __attribute__((noinline)) double noise_increment_f32(uint64_t seed, uint64_t sid, uint64_t n,
                                                               double sigma, double th, double ah) {
    return noise_f32(seed, sid, n, sigma, th, ah);
}

// noise_increment_f32 of two synapses (ids sid1, sid2, threshold sums th1,
// th2) in one call, the two generators' arithmetic interleaved.
struct NoisePair {
    double a, b;
};
static __device__ __attribute__((noinline)) NoisePair noise_increment2_f32(uint64_t seed, uint64_t sid1,
                                                                         uint64_t sid2, uint64_t n, double sigma,
                                                                         double th1, double th2, double ah) {
    return {noise_f32(seed, sid1, n, sigma, th1, ah), noise_f32(seed, sid2, n, sigma, th2, ah)};
}

constexpr uint64_t POIS_TAG = 0x706f6973736f6e21ull;

// Inter-arrival time (ms) number j of Poisson source k at rate (Hz):
// -ln(u) / rate, u from the first word of Threefry(counter j, key
// (seed, k, tag, 0)).
__device__ inline double poisson_isi(uint64_t seed, uint64_t k, uint64_t j, double rate_hz) {
    uint64_t x[4];
    threefry4x64_12(j, 0, 0, 0, seed, k, POIS_TAG, 0, x);
    const double u = ((double)(x[0] >> 11) + 0.5) * 0x1.0p-53;
    return -log(u) * (1000.0 / rate_hz);
}

// --------------------------------------------------------------- HH rates
__device__ __forceinline__ double dexp(double x) { return exp(x); }
__device__ __forceinline__ float dexp(float x) { return expf(x); }
__device__ __forceinline__ double dexpm1(double x) { return expm1(x); }
__device__ __forceinline__ float dexpm1(float x) { return expm1f(x); }

// Hodgkin-Huxley (1952) rates in 1/ms, rest at -65 mV, q10 factor 1:
// opening and closing rate (alpha, beta) of gate j (0 = m, 1 = h, 2 = n),
//   alpha_m = exprelr(x1), alpha_h = 0.07 exp(x1), alpha_n = 0.1 exprelr(x1),
//   beta_m = 4 exp(x2), beta_h = 1 / (exp(x2) + 1), beta_n = 0.125 exp(x2),
// with x1 = -(v + c1) / d1, x2 = -(v + c2) / d2 and the gate's constants.
// Written without branches on j, so that lanes integrating different
// gates of one wavefront do not serialise; each rate is the same expression
// as the gate-specific form.
template <class T>
__device__ __forceinline__ void hh_rate_pair(T v, int j, T &a, T &b) {
    const bool h = (j == 1);
    const T c1 = j == 0 ? T(40) : (h ? T(65) : T(55));
    const T d1 = h ? T(20) : T(10);
    const T c2 = h ? T(35) : T(65);
    const T d2 = j == 0 ? T(18) : (h ? T(10) : T(80));
    const T x1 = -(v + c1) / d1;
    const T x2 = -(v + c2) / d2;
    const T em1 = dexpm1(x1), e1 = dexp(x1), e2 = dexp(x2);
    const T rel = (x1 == T(0)) ? T(1) : x1 / em1;
    a = h ? T(0.07) * e1 : (j == 0 ? rel : T(0.1) * rel);
    b = h ? T(1) / (e2 + T(1)) : (j == 0 ? T(4) : T(0.125)) * e2;
}

// Mixed form: the same rates in FP32 with the hardware exponential and
// reciprocal (a few ulp), and expm1 by its Taylor series below |x| = 0.1,
// where exp(x) - 1 would cancel.
template <>
__device__ __forceinline__ void hh_rate_pair<float>(float v, int j, float &a, float &b) {
    const bool h = (j == 1);
    const float c1 = j == 0 ? 40.0f : (h ? 65.0f : 55.0f);
    const float d1 = h ? 20.0f : 10.0f;
    const float c2 = h ? 35.0f : 65.0f;
    const float d2 = j == 0 ? 18.0f : (h ? 10.0f : 80.0f);
    const float x1 = -__fdividef(v + c1, d1);
    const float x2 = -__fdividef(v + c2, d2);
    const float e1 = __expf(x1), e2 = __expf(x2);
    const float em1 = fabsf(x1) < 0.1f
                          ? x1 * (1.0f + x1 * (0.5f + x1 * (1.0f / 6.0f + x1 * (1.0f / 24.0f + x1 * (1.0f / 120.0f)))))
                          : e1 - 1.0f;
    const float rel = (x1 == 0.0f) ? 1.0f : __fdividef(x1, em1);
    a = h ? 0.07f * e1 : (j == 0 ? rel : 0.1f * rel);
    b = h ? __fdividef(1.0f, e2 + 1.0f) : (j == 0 ? 4.0f : 0.125f) * e2;
}

template <class T>
__device__ __forceinline__ void hh_rates(T v, T r[6]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) hh_rate_pair<T>(v, j, r[2 * j], r[2 * j + 1]);
}

// State views: the same device functions update state held in global
// memory (plain form, base 0) or staged in LDS for an epoch (fused form,
// base = first index owned by the workgroup).
template <class T>
struct GateView {
    T *m, *h, *n;
    uint32_t base;
};

template <class T>
struct SynView {
    T *g, *c;
    double *h, *z;
    uint32_t base;
};

// Per-synapse constants (reversal potential, decay factor, kind), global
// or staged in LDS (base as in SynView).
template <class T>
struct SynConst {
    const double *erev;
    const T *decay;
    const uint8_t *kind;
    uint32_t base;
};

// Exact exponential integration of gate j (0 = m, 1 = h, 2 = n) at the new
// voltage: x <- x_inf + (x - x_inf) exp(-dt (alpha + beta)).
template <class T>
__device__ __forceinline__ T gate_next(T x, T v, T dt, int j) {
    T a, b;
    hh_rate_pair<T>(v, j, a, b);
    const T xinf = a / (a + b);
    return xinf + (x - xinf) * dexp(-dt * (a + b));
}

template <>
__device__ __forceinline__ float gate_next<float>(float x, float v, float dt, int j) {
    float a, b;
    hh_rate_pair<float>(v, j, a, b);
    const float xinf = __fdividef(a, a + b);
    return xinf + (x - xinf) * __expf(-dt * (a + b));
}

// --------------------------------------------------------------- coherent access
// Loads and stores that are coherent across the whole device (they do not
// stop in the non-coherent per-XCD L2 cache).  Spike rings and their
// counters are written by one workgroup and read by another within a launch
// of the resident multi-epoch kernel, so they are accessed only this way.
template <class U>
__device__ __forceinline__ U ld_coh(const U *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class U>
__device__ __forceinline__ void st_coh(U *p, U v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// --------------------------------------------------------------- flags
__device__ inline void raise_flag(const DevNet &d, uint32_t flag, uint32_t cell) {
    uint32_t old = atomicOr(&d.ctr->flags, flag);
    if (old == 0) d.ctr->bad_cell = cell;
}

// --------------------------------------------------------------- events
__device__ __forceinline__ bool ev_before(const Event &a, const Event &b) {
    if (a.t != b.t) return a.t < b.t;
    if (a.src != b.src) return a.src < b.src;
    if (a.conn != b.conn) return a.conn < b.conn;
    return a.port < b.port;
}

// Applies one event (synapse s, port, weight w) to the synapse state;
// returns the conductance added (0 for the calcium port).
template <class T>
__device__ __forceinline__ T apply_event(const DevNet &d, uint32_t s, uint32_t port, double w,
                                         const SynView<T> &sv, const SynConst<T> &sc) {
    const uint32_t j = s - sv.base;
    if (port == 1) {
        T dg;
        const uint8_t kind = sc.kind[s - sc.base];
        if (kind == 1) {
            const double h0 = d.stc.h0;
            dg = (T)(w * ((sv.h[j] + h0 * sv.z[j]) / h0));
        } else if (kind == 2) {
            // STDP: the present weight clipped to [0, w_max], then the pre
            // trace jumps and the weight takes the post trace
            const double wt = sv.h[j];
            const double wc = wt < 0.0 ? 0.0 : (wt > d.stdp.w_max ? d.stdp.w_max : wt);
            dg = (T)(w * wc);
            sv.c[j] = sv.c[j] + (T)d.stdp.a_pre;
            sv.h[j] = wt + sv.z[j];
        } else {
            dg = (T)w;
        }
        sv.g[j] = sv.g[j] + dg;
        return dg;
    }
    sv.c[j] = sv.c[j] + (T)d.stc.c_pre;
    return T(0);
}

// Sorts cnt events in place into delivery order (t_e, source, connection,
// port); the events of one (cell, step) slot are few, so insertion sort.
__device__ inline void sort_slot(Event *ev, uint32_t cnt) {
    for (uint32_t i = 1; i < cnt; ++i) {
        Event x = ev[i];
        uint32_t j = i;
        while (j > 0 && ev_before(x, ev[j - 1])) {
            ev[j] = ev[j - 1];
            --j;
        }
        ev[j] = x;
    }
}

// Records the spike of `cell` at step n (crossing time ts) in the cell's
// ring and in the spike history.  Only the cell's own lane writes its ring;
// entries and counters are written with device-coherent stores, so that
// workgroups of a resident launch read them after the grid barrier.
__device__ inline void record_spike(const DevNet &d, uint32_t cell, uint64_t n, double ts) {
    const uint32_t k = ld_coh(d.spk_n + cell);
    uint64_t *r = (uint64_t *)(d.spk + (uint64_t)cell * d.H + (k & (d.H - 1)));
    st_coh(r, (uint64_t)__double_as_longlong(ts));
    st_coh(r + 1, (uint64_t)(uint32_t)n | ((uint64_t)k << 32));
    st_coh(d.spk_n + cell, k + 1);
    st_coh(d.spk_last + cell, (uint32_t)n + 1u);
    const uint64_t pos = atomicAdd((unsigned long long *)&d.ctr->hist_n, 1ull);
    if (pos < d.hist_cap) {
        d.hist_gid[pos] = cell;
        d.hist_step[pos] = n;
        d.hist_t[pos] = ts;
    } else {
        raise_flag(d, FLAG_HISTORY, cell);
    }
}

// The events of incoming connection q due in the steps [n0, n0 + nst):
// for every spike of the source recent enough to matter, a conductance
// event at t_e = t* + d and, with the calcium port, a calcium event at
// t_e + t_c,delay, each due at step floor(t_e / dt); emit(st, e) receives
// the step within the epoch and the event.  Spikes of the running epoch
// (step >= n0) and ring entries not yet holding the spike looked for are
// skipped.  The ring holds every spike that can still be due (sized on the
// host from the longest delay, a cell fires at most every second step).
// COH: the rings were written within the running launch (resident form), so
// they are read with device-coherent loads; otherwise an earlier launch
// wrote them and ordinary (cached) loads see them.
template <bool COH, class U>
__device__ __forceinline__ U ld_ring(const U *p) {
    if constexpr (COH) return ld_coh(p);
    else return *p;
}
template <bool COH, class F>
__device__ __forceinline__ void conn_events(const DevNet &d, uint64_t q, uint64_t n0, uint32_t nst, F &&emit) {
    // the source's counters and the connection's constants are loaded
    // together, and both words of a ring entry at once
    const uint32_t src = d.in_src[q];
    const uint32_t last = ld_ring<COH>(d.spk_last + src);
    const uint32_t cnt = ld_ring<COH>(d.spk_n + src);
    const int64_t lo = (int64_t)n0 - (int64_t)d.in_lag[q];
    if (last == 0 || (int64_t)last - 1 < lo) return;
    const uint32_t stop = cnt > d.H ? cnt - d.H : 0u;
    const uint8_t ports = d.in_ports[q];
    const double dly = d.in_d[q];
    Event e;
    e.w = d.in_w[q];
    e.syn = d.in_syn[q];
    e.src = src;
    e.conn = d.in_cid[q];
    const uint64_t n1 = n0 + nst;
    for (uint32_t k = cnt; k-- > stop;) {
        const uint64_t *r = (const uint64_t *)(d.spk + (uint64_t)src * d.H + (k & (d.H - 1)));
        const uint64_t w1 = ld_ring<COH>(r + 1);
        const uint64_t w0 = ld_ring<COH>(r);
        if ((uint32_t)(w1 >> 32) != k) continue;
        const uint64_t ns = (uint32_t)w1;
        if (ns >= n0) continue;
        if ((int64_t)ns < lo) break;
        const double ts = __longlong_as_double((long long)w0);
        const double te = ts + dly;
        if (ports & 1) {
            const uint64_t s = (uint64_t)floor(te / d.dt);
            if (s <= ns) raise_flag(d, FLAG_LATE, src);
            if (s >= n0 && s < n1) {
                e.t = te;
                e.port = 1;
                emit((uint32_t)(s - n0), e);
            }
        }
        if (ports & 2) {
            const double tc = te + d.stc.t_cd;
            const uint64_t s = (uint64_t)floor(tc / d.dt);
            if (s <= ns) raise_flag(d, FLAG_LATE, src);
            if (s >= n0 && s < n1) {
                e.t = tc;
                e.port = 2;
                emit((uint32_t)(s - n0), e);
            }
        }
    }
}

// The arrivals of explicit train tr due in [n0, n0 + nst), per port from
// that port's cursor (the calcium port t_c,delay later); `advance` moves
// the cursors past them.
template <class F>
__device__ inline void train_events(const DevNet &d, uint32_t tr, uint64_t n0, uint32_t nst, bool advance,
                                    F &&emit) {
    const uint64_t end = d.tr_off[tr + 1], n1 = n0 + nst;
    Event e;
    e.w = d.tr_w[tr];
    e.syn = d.tr_syn[tr];
    e.src = d.n_cells + tr;
    e.conn = 0;
    const uint8_t ports = d.tr_ports[tr];
    for (uint32_t p = 1; p <= 2; ++p) {
        if (!(ports & p)) continue;
        const double shift = p == 2 ? d.stc.t_cd : 0.0;
        uint64_t j = d.tr_cur[2 * tr + p - 1];
        for (; j < end; ++j) {
            const double t = p == 2 ? d.tr_t[j] + shift : d.tr_t[j];
            const uint64_t s = (uint64_t)floor(t / d.dt);
            if (s >= n1) break;
            if (s < n0) {
                // an arrival before the epoch: the cursor missed it
                raise_flag(d, FLAG_LATE, d.tr_cell[tr]);
                continue;
            }
            e.t = t;
            e.port = p;
            emit((uint32_t)(s - n0), e);
        }
        if (advance) d.tr_cur[2 * tr + p - 1] = j;
    }
}

// The arrivals of Poisson source k due in [n0, n0 + nst): each port walks
// the source's arrival sequence with a state of its own (next arrival time
// and index), the calcium port t_c,delay later; `advance` stores the state.
template <class F>
__device__ inline void poisson_events(const DevNet &d, uint32_t k, uint64_t n0, uint32_t nst, bool advance,
                                      F &&emit) {
    const uint64_t n1 = n0 + nst;
    Event e;
    e.w = d.pois_w[k];
    e.syn = d.pois_syn[k];
    e.src = d.n_cells + d.n_trains + k;
    e.conn = 0;
    const uint8_t ports = d.pois_ports[k];
    const double rate = d.pois_rate[k];
    for (uint32_t p = 1; p <= 2; ++p) {
        if (!(ports & p)) continue;
        double t = d.pois_t[2 * k + p - 1];
        uint64_t j = d.pois_j[2 * k + p - 1];
        for (;;) {
            const double te = p == 2 ? t + d.stc.t_cd : t;
            const double sf = floor(te / d.dt);
            if (!(sf < (double)n1)) break;
            if (sf >= (double)n0) {
                e.t = te;
                e.port = p;
                emit((uint32_t)((uint64_t)sf - n0), e);
            } else {
                raise_flag(d, FLAG_LATE, d.pois_cell[k]);
            }
            ++j;
            t = t + poisson_isi(d.seed, k, j, rate);
        }
        if (advance) {
            d.pois_t[2 * k + p - 1] = t;
            d.pois_j[2 * k + p - 1] = j;
        }
    }
}

// --------------------------------------------------------------- currents
// Membrane current (nA, outward positive) and dI/dV (uS) of one CV at V^n:
// HH (gate slot k, -1 if none), the CV's synapses q0..q1-1 in (CV, id) order,
// then its clamps cl0..cl1-1 active at t_n.
// P: gNa, gK, gL, ENa, EK, EL of the HH slot; sca: 1e-2 x lateral area.
template <class T>
__device__ inline void cv_current(const DevNet &d, int32_t k, const double *P, double sca, double v, double tn,
                                  const GateView<T> &gv, const SynView<T> &sv, const SynConst<T> &sc,
                                  uint32_t q0, uint32_t q1, uint32_t cl0, uint32_t cl1, double &Iout, double &Gout) {
    double I = 0.0, G = 0.0;
    if (k >= 0) {
        const uint32_t j = (uint32_t)k - gv.base;
        const double m = (double)gv.m[j];
        const double hh = (double)gv.h[j];
        const double nn = (double)gv.n[j];
        const double gna = P[0] * m * m * m * hh;
        const double gk = P[1] * nn * nn * nn * nn;
        const double idens = gna * (v - P[3]) + gk * (v - P[4]) + P[2] * (v - P[5]);
        I = sca * idens;
        G = sca * (gna + gk + P[2]);
    }
    uint32_t q = q0;
    for (; q + 4 <= q1; q += 4) {
        double gs[4], er[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            gs[j] = (double)sv.g[q + j - sv.base];
            er[j] = sc.erev[q + j - sc.base];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            I += gs[j] * (v - er[j]);
            G += gs[j];
        }
    }
    for (; q < q1; ++q) {
        const double gs = (double)sv.g[q - sv.base];
        I += gs * (v - sc.erev[q - sc.base]);
        G += gs;
    }
    for (uint32_t q = cl0; q < cl1; ++q) {
        if (d.cl_t0[q] <= tn && tn < d.cl_t0[q] + d.cl_dur[q]) I -= d.cl_amp[q];
    }
    Iout = I;
    Gout = G;
}

// Membrane current and dI/dV of one CV from HH (slot k, -1 if none), the
// CV's summed synaptic conductance gs = sum g and gs_e = sum g E (so that
// sum g (v - E) = gs v - gs_e), then its clamps active at t_n.
template <class T>
__device__ inline void cv_current_sums(const DevNet &d, int32_t k, const double *P, double sca, double v, double tn,
                                       const GateView<T> &gv, double gs, double gs_e, uint32_t cl0, uint32_t cl1,
                                       double &Iout, double &Gout) {
    double I = 0.0, G = 0.0;
    if (k >= 0) {
        const uint32_t j = (uint32_t)k - gv.base;
        const double m = (double)gv.m[j];
        const double hh = (double)gv.h[j];
        const double nn = (double)gv.n[j];
        const double gna = P[0] * m * m * m * hh;
        const double gk = P[1] * nn * nn * nn * nn;
        const double idens = gna * (v - P[3]) + gk * (v - P[4]) + P[2] * (v - P[5]);
        I = sca * idens;
        G = sca * (gna + gk + P[2]);
    }
    I += gs * v - gs_e;
    G += gs;
    for (uint32_t q = cl0; q < cl1; ++q) {
        if (d.cl_t0[q] <= tn && tn < d.cl_t0[q] + d.cl_dur[q]) I -= d.cl_amp[q];
    }
    Iout = I;
    Gout = G;
}

// Orders the LDS accesses of the lanes of one wavefront (a barrier among
// the wavefront's own lanes).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum of x over the 64 lanes of a wavefront with data-parallel-primitive
// lane shifts (no LDS traffic): an inclusive scan inside each row of 16
// lanes (shifts by 1, 2, 4, 8), then row 0's total added into row 1 and
// row 2's into row 3, then the first half's total into the second half;
// lane 63 ends with the sum, which is broadcast.  The summation order is
// fixed, so the result is deterministic.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_shift_add(double x) {
    const uint64_t u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xf, false);
    return x + __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t lane) {
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t u = (uint32_t)__shfl_up((int)v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double x) {
    x = dpp_shift_add<0x111, 0xf>(x);  // row_shr:1
    x = dpp_shift_add<0x112, 0xf>(x);  // row_shr:2
    x = dpp_shift_add<0x114, 0xf>(x);  // row_shr:4
    x = dpp_shift_add<0x118, 0xf>(x);  // row_shr:8
    x = dpp_shift_add<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x = dpp_shift_add<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    const uint64_t u = __double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// --------------------------------------------------------------- cable
// Quotient x / y.  EXACT: IEEE division (bitwise equal to the sequential
// CPU elimination).  Otherwise (mixed form) x times a reciprocal refined by
// two Newton steps from the hardware estimate: FP64 accurate to about one
// ulp, with a third of the dependent latency.
template <bool EXACT>
__device__ __forceinline__ double qdiv(double x, double y) {
    if constexpr (EXACT) {
        return x / y;
    } else {
        double r = __builtin_amdgcn_rcp(y);
        double e = fma(-y, r, 1.0);
        r = fma(e, r, r);
        e = fma(-y, r, 1.0);
        r = fma(e, r, r);
        return x * r;
    }
}

// Hines elimination of one cell's tree system in descending index order
// (parent[i] < i), then substitution in ascending order.  D and B hold the
// assembled diagonal and right-hand side and are overwritten; V receives the
// solution.  Indices b0..b1-1 and par[] are in the same index space; run[i]
// counts the consecutive nodes ending at i whose parent is their
// predecessor.  Along such runs eight nodes' operands are loaded ahead and
// the diagonal and right-hand side of the node being eliminated are carried
// in registers; the floating-point operations and their order are those of
// the plain elimination.  Returns false if a voltage is not finite.
template <bool EXACT>
__device__ inline bool hines_solve(double *D, double *B, double *V, const int32_t *par,
                                   const double *ax, const uint16_t *run, uint32_t b0, uint32_t b1) {
    double dc = D[b1 - 1], bc = B[b1 - 1];
    uint32_t i = b1 - 1;
    while (i > b0) {
        if (i >= b0 + 8 && run[i] >= 8) {
            double U[8], Dp[8], Bp[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                U[j] = -ax[i - j];
                Dp[j] = D[i - j - 1];
                Bp[j] = B[i - j - 1];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const double f = qdiv<EXACT>(U[j], dc);
                D[i - j] = dc;
                B[i - j] = bc;
                dc = Dp[j] - f * U[j];
                bc = Bp[j] - f * bc;
            }
            i -= 8;
            continue;
        }
        const int32_t p = par[i];
        const double u = -ax[i];
        const double f = qdiv<EXACT>(u, dc);
        D[i] = dc;
        B[i] = bc;
        if ((uint32_t)p == i - 1) {
            dc = D[p] - f * u;
            bc = B[p] - f * bc;
        } else {
            D[p] -= f * u;
            B[p] -= f * bc;
            dc = D[i - 1];
            bc = B[i - 1];
        }
        --i;
    }
    D[b0] = dc;
    B[b0] = bc;
    bool ok = true;
    double vp = qdiv<EXACT>(bc, dc);
    V[b0] = vp;
    ok = ok && isfinite(vp);
    i = b0 + 1;
    while (i < b1) {
        if (i + 8 <= b1 && run[i + 7] >= 8) {
            double U[8], Dl[8], Bl[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                U[j] = -ax[i + j];
                Dl[j] = D[i + j];
                Bl[j] = B[i + j];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                vp = qdiv<EXACT>(Bl[j] - U[j] * vp, Dl[j]);
                V[i + j] = vp;
                ok = ok && isfinite(vp);
            }
            i += 8;
            continue;
        }
        const int32_t p = par[i];
        const double u = -ax[i];
        const double vpar = ((uint32_t)p == i - 1) ? vp : V[p];
        vp = qdiv<EXACT>(B[i] - u * vpar, D[i]);
        V[i] = vp;
        ok = ok && isfinite(vp);
        ++i;
    }
    return ok;
}

// Nodes whose operands the segment sweeps load ahead of the dependent chain.
constexpr uint32_t SEG_PRELOAD = 8;

// Elimination of one unbranched segment [a, b] (every node after a has its
// predecessor as parent and only child), from the bottom node b, whose
// diagonal and right-hand side (after its children's contributions) are
// dc, bc.  Stores every node's final diagonal and right-hand side and
// returns those of the head a in dc, bc.
template <bool EXACT>
__device__ inline void seg_backward(double *D, double *B, const double *ax, uint32_t a, uint32_t b,
                                    double &dc, double &bc) {
    uint32_t i = b;
    while (i >= a + SEG_PRELOAD) {
        double U[SEG_PRELOAD], Dp[SEG_PRELOAD], Bp[SEG_PRELOAD];
#pragma unroll
        for (uint32_t j = 0; j < SEG_PRELOAD; ++j) {
            U[j] = -ax[i - j];
            Dp[j] = D[i - j - 1];
            Bp[j] = B[i - j - 1];
        }
#pragma unroll
        for (uint32_t j = 0; j < SEG_PRELOAD; ++j) {
            const double f = qdiv<EXACT>(U[j], dc);
            D[i - j] = dc;
            B[i - j] = bc;
            dc = Dp[j] - f * U[j];
            bc = Bp[j] - f * bc;
        }
        i -= SEG_PRELOAD;
    }
    // the last nodes (fewer than SEG_PRELOAD): their operands are loaded
    // before the chain too, so no LDS access sits inside it
    const uint32_t r = i - a;
    if (r) {
        double U[SEG_PRELOAD], Dp[SEG_PRELOAD], Bp[SEG_PRELOAD];
#pragma unroll
        for (uint32_t j = 0; j < SEG_PRELOAD; ++j) {
            if (j < r) {
                U[j] = -ax[i - j];
                Dp[j] = D[i - j - 1];
                Bp[j] = B[i - j - 1];
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < SEG_PRELOAD; ++j) {
            if (j < r) {
                const double f = qdiv<EXACT>(U[j], dc);
                D[i - j] = dc;
                B[i - j] = bc;
                dc = Dp[j] - f * U[j];
                bc = Bp[j] - f * bc;
            }
        }
    }
    D[a] = dc;
    B[a] = bc;
}

// Substitution along an unbranched segment [a, b] given V[a].
template <bool EXACT>
__device__ inline bool seg_forward(const double *D, const double *B, double *V, const double *ax,
                                   uint32_t a, uint32_t b) {
    double vp = V[a];
    bool ok = isfinite(vp);
    uint32_t i = a + 1;
    while (i + SEG_PRELOAD <= b + 1) {
        double U[SEG_PRELOAD], Dl[SEG_PRELOAD], Bl[SEG_PRELOAD];
#pragma unroll
        for (uint32_t j = 0; j < SEG_PRELOAD; ++j) {
            U[j] = -ax[i + j];
            Dl[j] = D[i + j];
            Bl[j] = B[i + j];
        }
#pragma unroll
        for (uint32_t j = 0; j < SEG_PRELOAD; ++j) {
            vp = qdiv<EXACT>(Bl[j] - U[j] * vp, Dl[j]);
            V[i + j] = vp;
            ok = ok && isfinite(vp);
        }
        i += SEG_PRELOAD;
    }
    const uint32_t r = b + 1 - i;
    if (r) {
        double U[SEG_PRELOAD], Dl[SEG_PRELOAD], Bl[SEG_PRELOAD];
#pragma unroll
        for (uint32_t j = 0; j < SEG_PRELOAD; ++j) {
            if (j < r) {
                U[j] = -ax[i + j];
                Dl[j] = D[i + j];
                Bl[j] = B[i + j];
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < SEG_PRELOAD; ++j) {
            if (j < r) {
                vp = qdiv<EXACT>(Bl[j] - U[j] * vp, Dl[j]);
                V[i + j] = vp;
                ok = ok && isfinite(vp);
            }
        }
    }
    return ok;
}

// --------------------------------------------------------------- synapses
// Conductance decay, then for tagging-and-capture synapses one step of
// Eqs. 17-20 from step-start h, z, c and the cell's step-start p.  If the
// cell fired in the previous step, the post-synaptic calcium jump is added
// first (after this step's events, as in the sequential definition).  The
// decayed conductance goes to gout (sv.g itself, or the other half of a
// double buffer).  Returns |h - h0| of step start (0 for plain synapses).
// One backward-Euler step of a diffusing species over the CVs b0..b1-1 of
// a cell whose constant tree system was eliminated beforehand: per CV the
// coupling u to the parent, the factor f = u / D' and the eliminated
// diagonal D'.  bx holds the right-hand side (amounts) and is swept in
// place; X receives the concentrations.  The operations and their order are
// those of the full elimination.
__device__ inline void species_sweep(double *bx, double *X, const int32_t *par, const double *f, const double *u,
                                     const double *dp, uint32_t b0, uint32_t b1) {
    for (uint32_t i = b1 - 1; i > b0; --i) bx[par[i]] -= f[i] * bx[i];
    X[b0] = bx[b0] / dp[b0];
    for (uint32_t i = b0 + 1; i < b1; ++i) X[i] = (bx[i] - u[i] * X[par[i]]) / dp[i];
}

template <class T>
struct SynIn {
    T g, dec, c;
    double h, z;
};

template <class T>
struct SynOut {
    T g, c;
    double h, z, absdh, th;
};

// The arithmetic of one synapse's update from its loaded operands (no
// memory access, so that several synapses of one lane can be interleaved);
// the caller adds the noise where out.th > 0 and stores the plastic state
// only for tagging-and-capture synapses.
template <class T>
__device__ __forceinline__ SynOut<T> syn_compute(const DevNet &d, double p, bool post, const SynIn<T> &x) {
    const Stc &P = d.stc;
    SynOut<T> o;
    o.g = x.g * x.dec;
    const T c = post ? x.c + (T)P.c_post : x.c;
    const double h = x.h, z = x.z, h0 = P.h0;
    const double thp = (c - (T)P.theta_p > T(0)) ? 1.0 : 0.0;
    const double thd = (c - (T)P.theta_d > T(0)) ? 1.0 : 0.0;
    const double ah = d.dt / P.tau_h;
    // Below both calcium thresholds (most synapses, most steps) the drift's
    // threshold terms are signed zeros and add nothing: the short form gives
    // the same bits as the full expression, which a wavefront computes only
    // when one of its lanes crossed a threshold.
    double drift = 0.1 * (h0 - h);
    if (__any(thp + thd > 0.0)) drift = drift + P.gamma_p * (10.0 - h) * thp - P.gamma_d * h * thd;
    o.h = h + ah * drift;
    o.th = thp + thd;
    const double tagp = ((h - h0) - P.theta_tag > 0.0) ? 1.0 : 0.0;
    const double tagd = ((h0 - h) - P.theta_tag > 0.0) ? 1.0 : 0.0;
    const double az = d.dt / P.tau_z;
    // likewise without a tag z keeps its value (z is never a negative zero:
    // it starts at +0 and sums of non-negative-zero operands stay so)
    o.z = z;
    if (__any(tagp + tagd > 0.0)) o.z = z + az * p * P.f_int * ((1.0 - z) * tagp - (z + 0.5) * tagd);
    if constexpr (sizeof(T) == 8) o.c = c * (T)d.r_c;
    else o.c = c * d.r_c_f;
    o.absdh = fabs(h - h0);
    return o;
}

// syn_compute of two synapses of one lane with one wavefront vote per
// short form for both: a taken full form gives a synapse whose own lanes
// would have taken the short form the same bits (its terms are signed
// zeros), so the outputs equal two syn_compute calls, while the two
// synapses' arithmetic stays interleaved between the votes.
template <class T>
__device__ __forceinline__ void syn_compute2(const DevNet &d, double p1, double p2, bool post, const SynIn<T> &x1,
                                             const SynIn<T> &x2, SynOut<T> &o1, SynOut<T> &o2) {
    const Stc &P = d.stc;
    const double h0 = P.h0, ah = d.dt / P.tau_h, az = d.dt / P.tau_z;
    o1.g = x1.g * x1.dec;
    o2.g = x2.g * x2.dec;
    const T c1 = post ? x1.c + (T)P.c_post : x1.c;
    const T c2 = post ? x2.c + (T)P.c_post : x2.c;
    const double h1 = x1.h, z1 = x1.z, h2 = x2.h, z2 = x2.z;
    const double thp1 = (c1 - (T)P.theta_p > T(0)) ? 1.0 : 0.0, thd1 = (c1 - (T)P.theta_d > T(0)) ? 1.0 : 0.0;
    const double thp2 = (c2 - (T)P.theta_p > T(0)) ? 1.0 : 0.0, thd2 = (c2 - (T)P.theta_d > T(0)) ? 1.0 : 0.0;
    double drift1 = 0.1 * (h0 - h1), drift2 = 0.1 * (h0 - h2);
    if (__any(thp1 + thd1 + thp2 + thd2 > 0.0)) {
        drift1 = drift1 + P.gamma_p * (10.0 - h1) * thp1 - P.gamma_d * h1 * thd1;
        drift2 = drift2 + P.gamma_p * (10.0 - h2) * thp2 - P.gamma_d * h2 * thd2;
    }
    o1.h = h1 + ah * drift1;
    o2.h = h2 + ah * drift2;
    o1.th = thp1 + thd1;
    o2.th = thp2 + thd2;
    const double tagp1 = ((h1 - h0) - P.theta_tag > 0.0) ? 1.0 : 0.0, tagd1 = ((h0 - h1) - P.theta_tag > 0.0) ? 1.0 : 0.0;
    const double tagp2 = ((h2 - h0) - P.theta_tag > 0.0) ? 1.0 : 0.0, tagd2 = ((h0 - h2) - P.theta_tag > 0.0) ? 1.0 : 0.0;
    o1.z = z1;
    o2.z = z2;
    if (__any(tagp1 + tagd1 + tagp2 + tagd2 > 0.0)) {
        o1.z = z1 + az * p1 * P.f_int * ((1.0 - z1) * tagp1 - (z1 + 0.5) * tagd1);
        o2.z = z2 + az * p2 * P.f_int * ((1.0 - z2) * tagp2 - (z2 + 0.5) * tagd2);
    }
    if constexpr (sizeof(T) == 8) {
        o1.c = c1 * (T)d.r_c;
        o2.c = c2 * (T)d.r_c;
    } else {
        o1.c = c1 * d.r_c_f;
        o2.c = c2 * d.r_c_f;
    }
    o1.absdh = fabs(h1 - h0);
    o2.absdh = fabs(h2 - h0);
}

// Noise increment of Eq. 18 added to the new h where a threshold is crossed.
template <class T>
__device__ __forceinline__ void syn_noise(const DevNet &d, uint32_t s, uint64_t n, SynOut<T> &o) {
    if (o.th > 0.0) {
        if constexpr (sizeof(T) == 8)
            o.h += noise_increment(d.seed, d.syn_sid[s], n, d.stc.sigma_pl, o.th, d.dt / d.stc.tau_h);
        else
            o.h += noise_increment_f32(d.seed, d.syn_sid[s], n, d.stc.sigma_pl, o.th, d.dt / d.stc.tau_h);
    }
}

// Whether a synapse with step-start calcium c draws noise at this step:
// the calcium after the post-synaptic jump above either threshold, the
// comparisons of syn_compute in the same precision (its threshold sum is
// then positive).
template <class T>
__device__ __forceinline__ bool syn_draws(const Stc &P, bool post, T c) {
    const T cc = post ? c + (T)P.c_post : c;
    return (cc - (T)P.theta_p > T(0)) || (cc - (T)P.theta_d > T(0));
}

// The STDP synapse's step in place of the tagging-and-capture outputs: the
// post-synaptic hook (a_post += A_post, w += a_pre), then both traces decay.
template <class T>
__device__ __forceinline__ void stdp_compute(const DevNet &d, bool post, const SynIn<T> &x, SynOut<T> &o) {
    const StdpK &P = d.stdp;
    o.h = post ? x.h + (double)x.c : x.h;
    const double ap = post ? x.z + P.a_post : x.z;
    o.z = ap * P.r_post;
    if constexpr (sizeof(T) == 8) o.c = x.c * (T)P.r_pre;
    else o.c = x.c * P.r_pre_f;
    o.absdh = 0.0;
}

template <class T>
__device__ __forceinline__ double syn_store(const SynView<T> &sv, uint32_t j, bool plastic, const SynOut<T> &o,
                                            T *gout) {
    gout[j] = o.g;
    if (!plastic) return 0.0;
    sv.h[j] = o.h;
    sv.z[j] = o.z;
    sv.c[j] = o.c;
    return o.absdh;
}

template <class T>
__device__ inline double syn_update(const DevNet &d, uint32_t s, uint64_t n, double p, bool post,
                                    const SynView<T> &sv, const SynConst<T> &sc, T *gout) {
    const uint32_t j = s - sv.base, jc = s - sc.base;
    const SynIn<T> x{sv.g[j], sc.decay[jc], sv.c[j], sv.h[j], sv.z[j]};
    const uint8_t kind = sc.kind[jc];
    SynOut<T> o = syn_compute<T>(d, p, post, x);
    if (kind == 1) syn_noise<T>(d, s, n, o);
    if (kind == 2) stdp_compute<T>(d, post, x, o);
    return syn_store<T>(sv, j, kind != 0, o, gout);
}

// --------------------------------------------------------------- cells
__device__ inline double prp_next(const DevNet &d, double p, double S) {
    const double ap = d.dt / d.stc.tau_p;
    const double trig = (S - d.stc.theta_pro > 0.0) ? 1.0 : 0.0;
    return p + ap * (-p + d.stc.p_max * trig);
}

// Threshold crossing V^n < theta <= V^{n+1} of the detector, and the
// linearly interpolated crossing time.
__device__ __forceinline__ bool crossed(const DevNet &d, double v0, double v1) {
    return v0 < d.theta && v1 >= d.theta;
}

__device__ __forceinline__ double spike_time(const DevNet &d, uint64_t n, double v0, double v1) {
    const double tn = (double)n * d.dt;
    return tn + d.dt * ((d.theta - v0) / (v1 - v0));
}

}  // namespace pa
