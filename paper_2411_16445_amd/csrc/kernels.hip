// HIP kernels (gfx950) of one implicit-Euler step of a plastic network of
// multi-compartment neurons, and of the spike exchange between epochs.
//
// Plain form: one kernel per stage per step (deliver, currents, solve,
// gates+sum, synapses, cells), each one lane per cell / CV / synapse.
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

__global__ void k_init_poisson(DevNet d) {
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.n_pois) return;
    d.pois_j[k] = 0;
    d.pois_t[k] = d.pois_rate[k] > 0.0 ? poisson_isi(d.seed, k, 0, d.pois_rate[k]) : INFINITY;
}

// ----------------------------------------------------------------- trains
// At the start of an epoch ending at `epoch_end`, move every train arrival
// whose delivery step falls before epoch_end into the target cell's ring.
__global__ void k_inject(DevNet d, uint32_t nsteps) {
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t epoch_start = d.ctr->step, epoch_end = epoch_start + nsteps;
    if (x < d.n_trains) inject_train(d, x, epoch_start, epoch_end);
    else if (x - d.n_trains < d.n_pois) inject_poisson(d, x - d.n_trains, epoch_start, epoch_end);
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
template <class T>
__global__ void k_deliver(DevNet d, uint64_t n) {
    uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= d.n_cells) return;
    const uint64_t ring = (uint64_t)cell * d.R + (uint32_t)(n % d.R);
    const uint32_t cnt = d.ev_n[ring];
    if (!cnt) return;
    deliver_slot<T>(d, cell, n, cnt, global_syn<T>(d), global_const<T>(d));
    d.ev_n[ring] = 0;
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
template <class T>
__global__ void k_syn(DevNet d, uint64_t n) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= d.n_syn) return;
    const uint32_t cell = d.syn_cell[s];
    const SynView<T> sv = global_syn<T>(d);
    (void)syn_update<T>(d, s, n, d.p[cell], d.post[cell] != 0, sv, global_const<T>(d), sv.g);
}

// ----------------------------------------------------------------- cells
__global__ void k_cellpost(DevNet d, uint64_t n) {
    uint32_t cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= d.n_cells) return;
    d.p[cell] = prp_next(d, d.p[cell], d.S[cell]);
    d.post[cell] = detect(d, cell, n, d.vdet_old[cell], d.V[d.det_cv[cell]]) ? 1 : 0;
}

// ----------------------------------------------------------------- exchange
// One wavefront per spike of the epoch (grid-stride), lanes over the
// source's outgoing connections; each connection port becomes one event in
// the target cell's ring.  Also appends the epoch's spikes to the history.
__global__ void k_expand(DevNet d, uint32_t nsteps) {
    const uint64_t epoch_end = d.ctr->step + nsteps;
    const uint32_t n_sp = d.ctr->ep_n;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n_waves = (gridDim.x * blockDim.x) >> 6;
    const uint64_t hist0 = d.ctr->hist_n;
    for (uint32_t k = wave; k < n_sp; k += n_waves) {
        const uint32_t gid = d.ep_gid[k];
        const double ts = d.ep_t[k];
        if (lane == 0) {
            uint64_t hpos = hist0 + k;
            if (hpos < d.hist_cap) {
                d.hist_gid[hpos] = gid;
                d.hist_step[hpos] = d.ep_step[k];
                d.hist_t[hpos] = ts;
            } else {
                raise_flag(d, FLAG_OVERFLOW, gid);
            }
        }
        expand_spike(d, gid, ts, lane, epoch_end);
    }
    // the last workgroup to finish closes the epoch: the spikes join the
    // history and the epoch's first step advances
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&d.ctr->blocks_done, 1u);
        if (prev == gridDim.x - 1) {
            __threadfence();
            d.ctr->hist_n += n_sp;
            d.ctr->ep_n = 0;
            d.ctr->step += nsteps;
            d.ctr->blocks_done = 0;
            __threadfence();
        }
    }
}



// ----------------------------------------------------------------- probes
template <class T>
__global__ void k_probe(DevNet d, uint64_t row) {
    uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.n_probes) return;
    const uint64_t i = d.pr_idx[k];
    double v = 0.0;
    switch (d.pr_what[k]) {
    case 0: v = d.V[i]; break;
    case 1: v = (double)((const T *)d.g)[i]; break;
    case 2: v = (double)((const T *)d.c)[i]; break;
    case 3: v = d.h[i]; break;
    case 4: v = d.z[i]; break;
    default: v = d.p[i]; break;
    }
    d.pr_buf[row * d.n_probes + k] = v;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
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

int launch_inject(const DevNet &d, uint32_t nsteps, void *stream) {
    if (d.n_trains + d.n_pois == 0) return 0;
    hipLaunchKernelGGL(k_inject, grid_for((uint64_t)d.n_trains + d.n_pois, 256), dim3(256), 0,
                       (hipStream_t)stream, d, nsteps);
    return (int)hipGetLastError();
}

template <class T>
static int step_plain(const DevNet &d, uint64_t n, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const dim3 b(256);
    const double tn = (double)n * d.dt;
    hipLaunchKernelGGL(k_deliver<T>, grid_for(d.n_cells, 256), b, 0, s, d, n);
    hipLaunchKernelGGL(k_current<T>, grid_for(d.n_cv, 256), b, 0, s, d, tn);
    hipLaunchKernelGGL(k_solve, grid_for(d.n_cells, 64), dim3(64), 0, s, d);
    hipLaunchKernelGGL(k_cellpre<T>, grid_for((uint64_t)d.n_cells * 64, 256), b, 0, s, d);
    if (e0) (void)hipEventRecord(e0, s);
    if (d.n_syn) hipLaunchKernelGGL(k_syn<T>, grid_for(d.n_syn, 256), b, 0, s, d, n);
    if (e1) (void)hipEventRecord(e1, s);
    hipLaunchKernelGGL(k_cellpost, grid_for(d.n_cells, 256), b, 0, s, d, n);
    return (int)hipGetLastError();
}

int launch_step_plain(const DevNet &d, uint64_t n, void *stream, void *ev_begin, void *ev_end) {
    if (d.mixed)
        return step_plain<float>(d, n, (hipStream_t)stream, (hipEvent_t)ev_begin, (hipEvent_t)ev_end);
    return step_plain<double>(d, n, (hipStream_t)stream, (hipEvent_t)ev_begin, (hipEvent_t)ev_end);
}

int launch_expand(const DevNet &d, uint32_t nsteps, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    // enough wavefronts for a busy epoch, bounded so an idle epoch is cheap
    uint64_t waves = (uint64_t)d.n_cells * d.K;
    if (waves > 4096) waves = 4096;
    if (waves < 4) waves = 4;
    hipLaunchKernelGGL(k_expand, grid_for(waves * 64, 256), dim3(256), 0, s, d, nsteps);
    return (int)hipGetLastError();
}

int launch_probe(const DevNet &d, uint64_t row, void *stream) {
    if (d.n_probes == 0) return 0;
    if (d.mixed)
        hipLaunchKernelGGL(k_probe<float>, grid_for(d.n_probes, 256), dim3(256), 0, (hipStream_t)stream, d, row);
    else
        hipLaunchKernelGGL(k_probe<double>, grid_for(d.n_probes, 256), dim3(256), 0, (hipStream_t)stream, d, row);
    return (int)hipGetLastError();
}

int launch_fill_u32(uint32_t *p, uint32_t v, size_t n, void *stream) {
    if (n == 0) return 0;
    hipLaunchKernelGGL(k_fill_u32, grid_for(n, 256), dim3(256), 0, (hipStream_t)stream, p, v, n);
    return (int)hipGetLastError();
}

}  // namespace pa
