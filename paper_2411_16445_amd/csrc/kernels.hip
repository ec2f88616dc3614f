// HIP kernels (gfx950) of one implicit-Euler step of a plastic network of
// multi-compartment neurons, and of the spike exchange between epochs.
//
// Plain form: per epoch one kernel gathering every cell's events of the
// epoch into its queue; per step one kernel per stage (deliver, currents,
// solve, gates+sum, synapses, cells), each one lane per cell / CV / synapse.
// Batched form (kernels_fused.hip): one kernel per epoch.
//
// Arithmetic follows the definitions of the model term by term, in a fixed
// order and without contraction into FMA (the library is built with
// -ffp-contract=off), so that every FP64 result that does not go through a
// transcendental function is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "sim.hpp"
#include "device_common.hpp"

namespace pa {

// ----------------------------------------------------------------- init
template <class T>
__global__ void k_init(DevNet d) {
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.n_hh) return;
    T v = (T)d.V[d.hh_cv[k]];
    T r[6];
    hh_rates<T>(v, r);
    ((T *)d.gm)[k] = r[0] / (r[0] + r[1]);
    ((T *)d.gh)[k] = r[2] / (r[2] + r[3]);
    ((T *)d.gn)[k] = r[4] / (r[4] + r[5]);
}

// Both arrival streams of Poisson source k (conductance and calcium port)
// start at its first arrival.
__global__ void k_init_poisson(DevNet d) {
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.n_pois) return;
    const double t0 = d.pois_rate[k] > 0.0 ? poisson_isi(d.seed, k, 0, d.pois_rate[k]) : INFINITY;
    d.pois_j[2 * k] = d.pois_j[2 * k + 1] = 0;
    d.pois_t[2 * k] = d.pois_t[2 * k + 1] = t0;
}

// ----------------------------------------------------------------- gather
// The events of the epoch [n0, n0 + nst) of one cell per wavefront, into
// the cell's queue: a counting pass over its incoming connections, trains
// and Poisson sources (count per step of the epoch), a wavefront prefix sum
// over the steps, a scatter pass, then each step's events sorted into
// delivery order (one lane per step).  LDS: 2 K words per wavefront.
__global__ void k_gather(DevNet d, uint64_t n0, uint32_t nst) {
    extern __shared__ uint32_t gsh[];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint32_t cell = blockIdx.x * (blockDim.x >> 6) + wave;
    if (cell >= d.n_cells) return;
    const uint32_t K = d.K;
    uint32_t *cnt = gsh + 2 * K * wave, *cur = cnt + K;
    for (uint32_t st = lane; st < nst; st += 64) cnt[st] = 0;
    wave_sync();
    const uint64_t qa = d.in_off[cell], qb = d.in_off[cell + 1];
    const uint32_t ta = d.tr_cell_off[cell], tb = d.tr_cell_off[cell + 1];
    const uint32_t pa = d.po_cell_off[cell], pb = d.po_cell_off[cell + 1];
    auto count = [&](uint32_t st, const Event &) { atomicAdd(&cnt[st], 1u); };
    for (uint64_t q = qa + lane; q < qb; q += 64) conn_events<false>(d, q, n0, nst, count);
    for (uint32_t x = ta + lane; x < tb; x += 64) train_events(d, d.tr_by_cell[x], n0, nst, false, count);
    for (uint32_t x = pa + lane; x < pb; x += 64) poisson_events(d, d.po_by_cell[x], n0, nst, false, count);
    wave_sync();
    uint32_t base = 0;
    for (uint32_t s0 = 0; s0 < nst; s0 += 64) {
        const uint32_t st = s0 + lane;
        const uint32_t v = st < nst ? cnt[st] : 0u;
        const uint32_t inc = wave_incl_scan(v, lane);
        if (st < nst) cur[st] = base + inc - v;
        base += (uint32_t)__shfl((int)inc, 63, 64);
    }
    const uint64_t q0 = d.q_off[cell];
    const uint64_t room = d.q_off[cell + 1] - q0;
    if (base > room && lane == 0) raise_flag(d, FLAG_QUEUE, cell);
    wave_sync();
    Event *Q = d.q_ev + q0;
    auto place = [&](uint32_t st, const Event &e) {
        const uint32_t pos = atomicAdd(&cur[st], 1u);
        if (pos < room) Q[pos] = e;
    };
    for (uint64_t q = qa + lane; q < qb; q += 64) conn_events<false>(d, q, n0, nst, place);
    for (uint32_t x = ta + lane; x < tb; x += 64) train_events(d, d.tr_by_cell[x], n0, nst, true, place);
    for (uint32_t x = pa + lane; x < pb; x += 64) poisson_events(d, d.po_by_cell[x], n0, nst, true, place);
    wave_sync();
    for (uint32_t st = lane; st < nst; st += 64) {
        const uint32_t c = cnt[st];
        const uint32_t off = cur[st] - c;
        const uint32_t m = off >= room ? 0u : (uint32_t)min<uint64_t>(c, room - off);
        sort_slot(Q + off, m);
        d.ev_n[(uint64_t)cell * K + st] = m;
        d.ev_off[(uint64_t)cell * K + st] = off;
    }
}

// ----------------------------------------------------------------- views
template <class T>
__device__ __forceinline__ SynView<T> global_syn(const DevNet &d) {
    return SynView<T>{(T *)d.g, (T *)d.c, d.h, d.z, 0u};
}
template <class T>
__device__ __forceinline__ GateView<T> global_gates(const DevNet &d) {
    return GateView<T>{(T *)d.gm, (T *)d.gh, (T *)d.gn, 0u};
}
template <class T>
__device__ __forceinline__ SynConst<T> global_const(const DevNet &d) {
    if constexpr (sizeof(T) == 8) return SynConst<T>{d.syn_erev, (const T *)d.syn_decay, d.syn_kind, 0u};
    else return SynConst<T>{d.syn_erev, (const T *)d.syn_decay_f, d.syn_kind, 0u};
}

// ----------------------------------------------------------------- deliver
// The events of step n of each cell (lane per cell), in their sorted order;
// n0 is the first step of the epoch the queues were gathered for.
template <class T>
__global__ void k_deliver(DevNet d, uint64_t n, uint64_t n0) {
    uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= d.n_cells) return;
    const uint64_t slot = (uint64_t)cell * d.K + (n - n0);
    const uint32_t cnt = d.ev_n[slot];
    if (!cnt) return;
    const Event *ev = d.q_ev + d.q_off[cell] + d.ev_off[slot];
    const SynView<T> sv = global_syn<T>(d);
    const SynConst<T> sc = global_const<T>(d);
    for (uint32_t i = 0; i < cnt; ++i) {
        const Event e = ev[i];
        apply_event<T>(d, e.syn, e.port, e.w, sv, sc);
        d.ev_cnt[2 * e.syn + e.port - 1] += 1ull;
        d.ev_sum[2 * e.syn + e.port - 1] += (unsigned long long)n;
    }
    atomicAdd((unsigned long long *)&d.ctr->events, (unsigned long long)cnt);
}

// ----------------------------------------------------------------- currents
template <class T>
__global__ void k_current(DevNet d, double tn) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.n_cv) return;
    double I, G;
    const int32_t hk = d.hh_of[i];
    const double *P = hk >= 0 ? d.hh_par + 6 * (size_t)hk : nullptr;
    const double sca = hk >= 0 ? d.hh_scale[hk] : 0.0;
    cv_current<T>(d, hk, P, sca, d.V[i], tn, global_gates<T>(d), global_syn<T>(d), global_const<T>(d),
                  d.cv_syn_off[i], d.cv_syn_off[i + 1], d.cv_cl_off[i], d.cv_cl_off[i + 1], I, G);
    d.I[i] = I;
    d.G[i] = G;
}

// ----------------------------------------------------------------- solve
// Assembly of the backward-Euler cable system and Hines elimination, one
// lane per cell.
__global__ void k_solve(DevNet d) {
    uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= d.n_cells) return;
    const uint32_t b0 = d.cv_off[cell], b1 = d.cv_off[cell + 1];
    d.vdet_old[cell] = d.V[d.det_cv[cell]];
    for (uint32_t i = b0; i < b1; ++i) {
        double v = d.V[i];
        double G = d.G[i];
        d.D[i] = d.d0[i] + G;
        d.b[i] = ((d.cdt[i] * v + d.gpas_e[i]) - d.I[i]) + G * v;
    }
    const bool ok = d.mixed ? hines_solve<false>(d.D, d.b, d.V, d.parent, d.axial, d.run, b0, b1)
                            : hines_solve<true>(d.D, d.b, d.V, d.parent, d.axial, d.run, b0, b1);
    if (!ok) raise_flag(d, FLAG_NONFINITE, cell);
}

// ----------------------------------------------------------------- gates, S
// One wavefront per cell: the cell's HH gates at V^{n+1} (one lane per
// gate) and its protein trigger sum S over the plastic synapses, lane l
// taking the cell's synapses l, l+64, ... and a fixed lane-shift tree
// adding the lanes (the order of the fused form).
template <class T>
__global__ void k_cellpre(DevNet d) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t cell = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (cell >= d.n_cells) return;
    const uint32_t k0 = d.hh_off[cell], nh = d.hh_off[cell + 1] - k0;
    T *gates[3] = {(T *)d.gm, (T *)d.gh, (T *)d.gn};
    for (uint32_t t = lane; t < 3 * nh; t += 64) {
        const uint32_t k = k0 + t / 3, j = t % 3;
        T *x = gates[j] + k;
        *x = gate_next<T>(*x, (T)d.V[d.hh_cv[k]], (T)d.dt, (int)j);
    }
    const double h0 = d.stc.h0;
    double S = 0.0;
    for (uint32_t s = d.syn_off[cell] + lane; s < d.syn_off[cell + 1]; s += 64)
        S += d.syn_kind[s] == 1 ? fabs(d.h[s] - h0) : 0.0;
    S = wave_sum(S);
    if (lane == 0) d.S[cell] = S;
}

// ----------------------------------------------------------------- synapses
// With particle diffusion, z takes the protein concentration of the
// synapse's CV, and the step's change of |h - h0| is kept for the release
// of the synthesis-triggering signal.
template <class T>
__global__ void k_syn(DevNet d, uint64_t n) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.n_syn) return;
    const uint32_t cell = d.syn_cell[s];
    const SynView<T> sv = global_syn<T>(d);
    const double p = d.dif ? d.prp[d.syn_cv[s]] : d.p[cell];
    const double a0 = syn_update<T>(d, s, n, p, d.post[cell] != 0, sv, global_const<T>(d), sv.g);
    if (d.dif) d.dlt[s] = d.syn_kind[s] == 1 ? fabs(d.h[s] - d.stc.h0) - a0 : 0.0;
}

// ----------------------------------------------------------------- species
// One lane per cell: the step of both diffusing species (synthesis trigger
// from the step-start SPS concentration at the soma; SPS with the step's
// release per CV, the sum over the CV's plastic synapses in (CV, id)
// order; PRP with decay and synthesis).  d.b serves as the right-hand
// side (the cable solve is done with it).
__global__ void k_species(DevNet d) {
    uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= d.n_cells) return;
    const uint32_t b0 = d.cv_off[cell], b1 = d.cv_off[cell + 1];
    const uint32_t soma = d.det_cv[cell];
    const double trig = (d.sps[soma] - d.dif_thr[cell] > 0.0) ? 1.0 : 0.0;
    double *bx = d.b;
    for (uint32_t i = b0; i < b1; ++i) {
        double r = 0.0;
        for (uint32_t q = d.cv_syn_off[i]; q < d.cv_syn_off[i + 1]; ++q)
            if (d.syn_kind[q] == 1) r += d.dlt[q];
        bx[i] = d.dvol[i] * d.sps[i] + r;
    }
    species_sweep(bx, d.sps, d.parent, d.sps_f, d.sps_u, d.sps_dp, b0, b1);
    const double ap = d.dt / d.stc.tau_p;
    for (uint32_t i = b0; i < b1; ++i) {
        const double x = d.prp[i];
        bx[i] = d.dvol[i] * (x + ap * (-x));
    }
    bx[soma] += ap * d.dif_pv[cell] * trig;
    species_sweep(bx, d.prp, d.parent, d.prp_f, d.prp_u, d.prp_dp, b0, b1);
}

// ----------------------------------------------------------------- cells
__global__ void k_cellpost(DevNet d, uint64_t n) {
    uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= d.n_cells) return;
    if (!d.dif) d.p[cell] = prp_next(d, d.p[cell], d.S[cell]);
    const double v0 = d.vdet_old[cell], v1 = d.V[d.det_cv[cell]];
    const bool fired = crossed(d, v0, v1);
    if (fired) record_spike(d, cell, n, spike_time(d, n, v0, v1));
    d.post[cell] = fired ? 1 : 0;
}

// ----------------------------------------------------------------- probes
// Probes due after step n (stride dividing n): probe k's sample of step n
// goes to entry n / stride - first / stride - 1 of its region, `first` being
// the first step of the present drain interval.
template <class T>
__global__ void k_probe(DevNet d, uint64_t n, uint64_t first) {
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.n_probes) return;
    const uint32_t str = d.pr_stride[k];
    if (n % str != 0) return;
    const uint64_t i = d.pr_idx[k];
    double v = 0.0;
    switch (d.pr_what[k]) {
    case 0: v = d.V[i]; break;
    case 1: v = (double)((const T *)d.g)[i]; break;
    case 2: v = (double)((const T *)d.c)[i]; break;
    case 3: v = d.h[i]; break;
    case 4: v = d.z[i]; break;
    case 6: v = d.sps[i]; break;
    case 7: v = d.prp[i]; break;
    default: v = d.p[i]; break;
    }
    d.pr_buf[d.pr_off[k] + n / str - first / str - 1] = v;
}

// A state array into a caller's device buffer: element q (words 64-bit
// words each, or one FP32 value widened) to position perm[q] (or q).
__global__ void k_state_out(const void *src, uint32_t words, uint32_t narrow, const uint32_t *perm, uint64_t n,
                            void *dst) {
    const uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const uint64_t o = perm ? perm[q] : q;
    if (narrow) {
        ((double *)dst)[o] = (double)((const float *)src)[q];
    } else {
        for (uint32_t j = 0; j < words; ++j) ((uint64_t *)dst)[o * words + j] = ((const uint64_t *)src)[q * words + j];
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ----------------------------------------------------------------- fast-forward
// n_long long steps of the slow plasticity variables, one wavefront per
// cell (the cell's S couples its synapses): per step S over the cell's
// plastic synapses from step-start h (lane l takes synapses l, l+64, ...,
// then the fixed lane-shift tree), h relaxing to h0 and z from step-start
// h, z, p (Eqs. 17 and 20 without calcium), conductance and calcium decay
// by their factors over a long step (gdec per synapse, rc), then p (Eq.
// 21).  Membrane state is not touched.
template <class T>
__global__ void k_fast_forward(DevNet d, uint64_t n_long, double ah, double az, double ap, const double *gdec,
                               double rc) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t cell = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (cell >= d.n_cells) return;
    const uint32_t a = d.syn_off[cell], e = d.syn_off[cell + 1];
    const Stc &P = d.stc;
    const double h0 = P.h0;
    T *g = (T *)d.g, *c = (T *)d.c;
    double p = d.p[cell];
    for (uint64_t k = 0; k < n_long; ++k) {
        double S = 0.0;
        for (uint32_t s = a + lane; s < e; s += 64) S += d.syn_kind[s] == 1 ? fabs(d.h[s] - h0) : 0.0;
        S = wave_sum(S);
        for (uint32_t s = a + lane; s < e; s += 64) {
            g[s] = g[s] * (T)gdec[s];
            if (d.syn_kind[s] != 1) continue;
            const double h = d.h[s], z = d.z[s];
            const double tagp = ((h - h0) - P.theta_tag > 0.0) ? 1.0 : 0.0;
            const double tagd = ((h0 - h) - P.theta_tag > 0.0) ? 1.0 : 0.0;
            d.h[s] = h + ah * (0.1 * (h0 - h));
            d.z[s] = z + az * p * P.f_int * ((1.0 - z) * tagp - (z + 0.5) * tagd);
            c[s] = c[s] * (T)rc;
        }
        const double trig = (S - P.theta_pro > 0.0) ? 1.0 : 0.0;
        p = p + ap * (-p + P.p_max * trig);
    }
    if (lane == 0) {
        d.p[cell] = p;
        d.post[cell] = 0;
        d.spk_n[cell] = 0;
        d.spk_last[cell] = 0;
    }
}

// After a jump to step n_new: a Poisson source whose next arrival falls
// before it draws that arrival again (index + 1) from the new time; both
// port streams continue from the conductance stream's arrival (everything
// earlier, calcium events included, is dropped).
__global__ void k_ff_poisson(DevNet d, uint64_t n_new) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.n_pois) return;
    double t = d.pois_t[2 * k];
    uint64_t j = d.pois_j[2 * k];
    if (d.pois_rate[k] > 0.0 && floor(t / d.dt) < (double)n_new) {
        j += 1;
        t = (double)n_new * d.dt + poisson_isi(d.seed, k, j, d.pois_rate[k]);
    }
    d.pois_t[2 * k] = d.pois_t[2 * k + 1] = t;
    d.pois_j[2 * k] = d.pois_j[2 * k + 1] = j;
}

// ================================================================= launchers
static inline dim3 grid_for(uint64_t n, uint32_t block) {
    uint64_t g = (n + block - 1) / block;
    return dim3((uint32_t)(g ? g : 1));
}

int launch_init(const DevNet &d, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (d.n_pois) hipLaunchKernelGGL(k_init_poisson, grid_for(d.n_pois, 256), dim3(256), 0, s, d);
    if (d.n_hh == 0) return (int)hipGetLastError();
    if (d.mixed) hipLaunchKernelGGL(k_init<float>, grid_for(d.n_hh, 256), dim3(256), 0, s, d);
    else hipLaunchKernelGGL(k_init<double>, grid_for(d.n_hh, 256), dim3(256), 0, s, d);
    return (int)hipGetLastError();
}

int launch_gather(const DevNet &d, uint64_t n0, uint32_t nsteps, void *stream) {
    hipLaunchKernelGGL(k_gather, grid_for((uint64_t)d.n_cells * 64, 256), dim3(256), 4 * 2 * d.K * sizeof(uint32_t),
                       (hipStream_t)stream, d, n0, nsteps);
    return (int)hipGetLastError();
}

template <class T>
static int step_plain(const DevNet &d, uint64_t n, uint64_t n0, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const dim3 b(256);
    const double tn = (double)n * d.dt;
    hipLaunchKernelGGL(k_deliver<T>, grid_for(d.n_cells, 256), b, 0, s, d, n, n0);
    hipLaunchKernelGGL(k_current<T>, grid_for(d.n_cv, 256), b, 0, s, d, tn);
    hipLaunchKernelGGL(k_solve, grid_for(d.n_cells, 64), dim3(64), 0, s, d);
    hipLaunchKernelGGL(k_cellpre<T>, grid_for((uint64_t)d.n_cells * 64, 256), b, 0, s, d);
    if (e0) (void)hipEventRecord(e0, s);
    if (d.n_syn) hipLaunchKernelGGL(k_syn<T>, grid_for(d.n_syn, 256), b, 0, s, d, n);
    if (e1) (void)hipEventRecord(e1, s);
    if (d.dif) hipLaunchKernelGGL(k_species, grid_for(d.n_cells, 64), dim3(64), 0, s, d);
    hipLaunchKernelGGL(k_cellpost, grid_for(d.n_cells, 256), b, 0, s, d, n);
    return (int)hipGetLastError();
}

int launch_step_plain(const DevNet &d, uint64_t n, uint64_t n0, void *stream, void *ev_begin, void *ev_end) {
    if (d.mixed)
        return step_plain<float>(d, n, n0, (hipStream_t)stream, (hipEvent_t)ev_begin, (hipEvent_t)ev_end);
    return step_plain<double>(d, n, n0, (hipStream_t)stream, (hipEvent_t)ev_begin, (hipEvent_t)ev_end);
}

int launch_probe(const DevNet &d, uint64_t n, uint64_t first, void *stream) {
    if (d.n_probes == 0) return 0;
    if (d.mixed)
        hipLaunchKernelGGL(k_probe<float>, grid_for(d.n_probes, 256), dim3(256), 0, (hipStream_t)stream, d, n, first);
    else
        hipLaunchKernelGGL(k_probe<double>, grid_for(d.n_probes, 256), dim3(256), 0, (hipStream_t)stream, d, n, first);
    return (int)hipGetLastError();
}

int launch_state_out(const void *src, uint32_t words, bool narrow, const uint32_t *perm, uint64_t n, void *dst,
                     void *stream) {
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_state_out, grid_for(n, 256), dim3(256), 0, (hipStream_t)stream, src, words,
                       narrow ? 1u : 0u, perm, n, dst);
    return (int)hipGetLastError();
}

int launch_fast_forward(const DevNet &d, uint64_t n_long, double dt_long, const double *gdec, double rc,
                        uint64_t n_new, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    const double ah = dt_long / d.stc.tau_h, az = dt_long / d.stc.tau_z, ap = dt_long / d.stc.tau_p;
    if (d.mixed)
        hipLaunchKernelGGL(k_fast_forward<float>, grid_for((uint64_t)d.n_cells * 64, 256), dim3(256), 0, s, d, n_long,
                           ah, az, ap, gdec, rc);
    else
        hipLaunchKernelGGL(k_fast_forward<double>, grid_for((uint64_t)d.n_cells * 64, 256), dim3(256), 0, s, d, n_long,
                           ah, az, ap, gdec, rc);
    if (d.n_pois) hipLaunchKernelGGL(k_ff_poisson, grid_for(d.n_pois, 256), dim3(256), 0, s, d, n_new);
    return (int)hipGetLastError();
}

int launch_fill_u32(uint32_t *p, uint32_t v, size_t n, void *stream) {
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_fill_u32, grid_for(n, 256), dim3(256), 0, (hipStream_t)stream, p, v, n);
    return (int)hipGetLastError();
}

}  // namespace pa
