// Batched form: one fused kernel per epoch.
//
// Cells only interact through spike events, and an event is delivered at
// least one epoch (K steps, K dt below the smallest delay) after the spike
// that caused it.  Within an epoch every cell therefore evolves on its own:
// a workgroup owns a packed run of consecutive cells (their CVs, HH CVs
// and synapses are contiguous in memory) and advances them through all K
// steps of the epoch, synchronising only with __syncthreads between the
// stages of a step.  The per-cell serial work (Hines elimination, the
// protein trigger sum, event delivery) reads and writes the cable system in
// LDS: voltage, diagonal, right-hand side, axial conductance, parent, the
// |h - h0| terms and the per-cell p stay on chip for the whole epoch.
//
// Every stage calls the same device functions as the plain form in the
// same order, so the two forms give bitwise identical results.
//
// The host part packs cells into workgroups under an LDS budget and picks
// the number of cells per workgroup by timing trial epochs (autotuning),
// then captures a graph of several epochs (inject, fused step kernel,
// expand, close) that the advance loop replays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/plasticarbor.h"
#include "device_common.hpp"
#include "sim.hpp"

namespace pa {

constexpr uint32_t FUSED_THREADS = 256;

// LDS bytes of a workgroup owning nv CVs, ns synapses and nc cells.
__host__ __device__ inline size_t fused_lds_bytes(uint32_t nv, uint32_t ns, uint32_t nc) {
    return (size_t)nv * (4 * 8 + 4) + (size_t)ns * 8 + (size_t)nc * 16;
}

template <class T>
__global__ __launch_bounds__(FUSED_THREADS) void k_epoch(DevNet d, const uint32_t *__restrict__ blk,
                                                         uint32_t nsteps) {
    extern __shared__ double lds[];
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t c0 = blk[blockIdx.x], c1 = blk[blockIdx.x + 1];
    const uint32_t ncb = c1 - c0;
    const uint32_t v0 = d.cv_off[c0], nv = d.cv_off[c1] - v0;
    const uint32_t s0 = d.syn_off[c0], ns = d.syn_off[c1] - s0;
    const uint32_t k0 = d.hh_off[c0], nhh = d.hh_off[c1] - k0;
    double *sV = lds;
    double *sD = sV + nv;
    double *sB = sD + nv;
    double *sAx = sB + nv;
    double *sAbs = sAx + nv;
    double *sP = sAbs + ns;
    double *sVold = sP + ncb;
    int32_t *sPar = (int32_t *)(sVold + ncb);

    for (uint32_t i = tid; i < nv; i += nt) {
        sV[i] = d.V[v0 + i];
        sAx[i] = d.axial[v0 + i];
        const int32_t p = d.parent[v0 + i];
        sPar[i] = p < 0 ? -1 : p - (int32_t)v0;
    }
    for (uint32_t c = tid; c < ncb; c += nt) sP[c] = d.p[c0 + c];
    const uint64_t n0 = d.ctr->step;
    const double h0 = d.stc.h0;
    __syncthreads();

    for (uint32_t st = 0; st < nsteps; ++st) {
        const uint64_t n = n0 + st;
        const double tn = (double)n * d.dt;
        // A. events due at step n, then the post-synaptic hook
        for (uint32_t c = tid; c < ncb; c += nt) deliver_cell<T>(d, c0 + c, n);
        __syncthreads();
        // B. currents at V^n and assembly of the cable system
        for (uint32_t i = tid; i < nv; i += nt) {
            const double v = sV[i];
            double I, G;
            cv_current<T>(d, v0 + i, v, tn, I, G);
            sD[i] = d.d0[v0 + i] + G;
            sB[i] = ((d.cdt[v0 + i] * v + d.gpas_e[v0 + i]) - I) + G * v;
        }
        __syncthreads();
        // C. Hines elimination, one lane per cell
        for (uint32_t c = tid; c < ncb; c += nt) {
            const uint32_t b0 = d.cv_off[c0 + c] - v0, b1 = d.cv_off[c0 + c + 1] - v0;
            sVold[c] = sV[d.det_cv[c0 + c] - v0];
            for (uint32_t i = b1 - 1; i > b0; --i) {
                const int32_t p = sPar[i];
                const double u = -sAx[i];
                const double f = u / sD[i];
                sD[p] -= f * u;
                sB[p] -= f * sB[i];
            }
            bool ok = true;
            const double vr = sB[b0] / sD[b0];
            sV[b0] = vr;
            ok = ok && isfinite(vr);
            for (uint32_t i = b0 + 1; i < b1; ++i) {
                const double u = -sAx[i];
                const double v = (sB[i] - u * sV[sPar[i]]) / sD[i];
                sV[i] = v;
                ok = ok && isfinite(v);
            }
            if (!ok) raise_flag(d, FLAG_NONFINITE, c0 + c);
        }
        __syncthreads();
        // D. gates at V^{n+1}; synapses (decay, plasticity from step-start
        //    values); |h - h0| of step start for the protein trigger
        for (uint32_t k = tid; k < nhh; k += nt) gate_update<T>(d, k0 + k, sV[d.hh_cv[k0 + k] - v0]);
        for (uint32_t s = tid; s < ns; s += nt) {
            const uint32_t q = s0 + s;
            sAbs[s] = (d.syn_kind[q] == 1) ? fabs(d.h[q] - h0) : 0.0;
            syn_update<T>(d, q, n, sP[d.syn_cell[q] - c0]);
        }
        __syncthreads();
        // E. protein synthesis and threshold detection, one lane per cell
        for (uint32_t c = tid; c < ncb; c += nt) {
            double S = 0.0;
            for (uint32_t s = d.syn_off[c0 + c] - s0; s < d.syn_off[c0 + c + 1] - s0; ++s) S += sAbs[s];
            const double ap = d.dt / d.stc.tau_p;
            const double trig = (S - d.stc.theta_pro > 0.0) ? 1.0 : 0.0;
            const double p = sP[c];
            sP[c] = p + ap * (-p + d.stc.p_max * trig);
            detect(d, c0 + c, n, sVold[c], sV[d.det_cv[c0 + c] - v0]);
        }
        __syncthreads();
    }
    for (uint32_t i = tid; i < nv; i += nt) d.V[v0 + i] = sV[i];
    for (uint32_t c = tid; c < ncb; c += nt) d.p[c0 + c] = sP[c];
}

int launch_epoch_fused(const DevNet &d, uint32_t nsteps, const uint32_t *blk, uint32_t n_blocks,
                       size_t lds_bytes, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (d.mixed)
        hipLaunchKernelGGL(k_epoch<float>, dim3(n_blocks), dim3(FUSED_THREADS), lds_bytes, s, d, blk, nsteps);
    else
        hipLaunchKernelGGL(k_epoch<double>, dim3(n_blocks), dim3(FUSED_THREADS), lds_bytes, s, d, blk, nsteps);
    return (int)hipGetLastError();
}

}  // namespace pa

// ======================================================================
// Host side of the batched form.
using namespace pa;

DevNet &pa_devnet(pa_sim *s);
hipStream_t pa_stream(pa_sim *s);
void *pa_dev_alloc(pa_sim *s, size_t bytes);
pa_status pa_fail(pa_sim *s, pa_status st, const char *msg);
const pa_config &pa_cfg(pa_sim *s);
pa_status pa_snapshot(pa_sim *s, int restore);

struct BatchedPlan {
    std::vector<uint32_t> blk;  // cell boundaries, n_blocks + 1
    uint32_t *d_blk = nullptr;
    size_t lds = 0;
    uint32_t cells_per_block = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t graph_epochs = 0;
};

BatchedPlan *&pa_plan(pa_sim *s);

namespace {

constexpr size_t LDS_BUDGET = 64 * 1024;   // per workgroup: 2 resident per CU
constexpr size_t LDS_MAX = 160 * 1024;

// Packs consecutive cells, at most cpb per workgroup, within the LDS budget.
bool pack(const std::vector<uint32_t> &cv_off, const std::vector<uint32_t> &syn_off, uint32_t cpb,
          std::vector<uint32_t> &blk, size_t &lds) {
    const uint32_t nc = (uint32_t)cv_off.size() - 1;
    blk.assign(1, 0);
    lds = 0;
    uint32_t c = 0;
    while (c < nc) {
        uint32_t e = c + 1;
        size_t b = fused_lds_bytes(cv_off[e] - cv_off[c], syn_off[e] - syn_off[c], 1);
        if (b > LDS_MAX) return false;
        while (e < nc && e - c < cpb) {
            size_t b2 = fused_lds_bytes(cv_off[e + 1] - cv_off[c], syn_off[e + 1] - syn_off[c], e + 1 - c);
            if (b2 > LDS_BUDGET) break;
            b = b2;
            ++e;
        }
        lds = std::max(lds, b);
        blk.push_back(e);
        c = e;
    }
    return true;
}

pa_status upload_plan(pa_sim *s, BatchedPlan &P) {
    P.d_blk = (uint32_t *)pa_dev_alloc(s, P.blk.size() * 4);
    if (!P.d_blk) return pa_fail(s, PA_ENOMEM, "block table");
    if (hipMemcpy(P.d_blk, P.blk.data(), P.blk.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return pa_fail(s, PA_EDEVICE, "block table upload");
    return PA_OK;
}

int enqueue_epoch(const DevNet &d, const BatchedPlan &P, uint32_t nsteps, hipStream_t st,
                  hipEvent_t e0, hipEvent_t e1) {
    int r = launch_inject(d, nsteps, st);
    if (e0) (void)hipEventRecord(e0, st);
    r |= launch_epoch_fused(d, nsteps, P.d_blk, (uint32_t)P.blk.size() - 1, P.lds, st);
    if (e1) (void)hipEventRecord(e1, st);
    r |= launch_expand(d, nsteps, st);
    return r;
}

}  // namespace

pa_status batched_setup(pa_sim *s) {
    DevNet &d = pa_devnet(s);
    hipStream_t st = pa_stream(s);
    BatchedPlan *&plan = pa_plan(s);
    plan = new BatchedPlan();
    // host copies of the offsets for packing
    std::vector<uint32_t> cv_off(d.n_cells + 1), syn_off(d.n_cells + 1);
    if (hipMemcpy(cv_off.data(), d.cv_off, cv_off.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(syn_off.data(), d.syn_off, syn_off.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return pa_fail(s, PA_EDEVICE, "offsets");
    std::vector<uint32_t> cands;
    const uint32_t fixed = pa_cfg(s).cells_per_block;
    if (fixed) cands.push_back(fixed);
    else
        for (uint32_t c : {1u, 2u, 4u, 8u, 16u, 32u, 64u})
            if (c <= std::max<uint32_t>(1, d.n_cells)) cands.push_back(c);
    double best_ms = INFINITY;
    uint32_t best = 0;
    const bool tune = cands.size() > 1;
    if (tune && pa_snapshot(s, 0) != PA_OK) return PA_EDEVICE;
    for (uint32_t cpb : cands) {
        BatchedPlan P;
        if (!pack(cv_off, syn_off, cpb, P.blk, P.lds)) continue;
        if (!tune) {
            best = cpb;
            break;
        }
        if (upload_plan(s, P) != PA_OK) return PA_EDEVICE;
        // trial: 1 warm epoch, then time 4 epochs of K steps
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
            return pa_fail(s, PA_EDEVICE, "event");
        int r = enqueue_epoch(d, P, d.K, st, nullptr, nullptr);
        r |= (int)hipEventRecord(a, st);
        for (int e = 0; e < 4; ++e) r |= enqueue_epoch(d, P, d.K, st, nullptr, nullptr);
        r |= (int)hipEventRecord(b, st);
        if (r || hipEventSynchronize(b) != hipSuccess) return pa_fail(s, PA_EDEVICE, "autotune trial");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (ms < best_ms) {
            best_ms = ms;
            best = cpb;
        }
        if (pa_snapshot(s, 1) != PA_OK) return PA_EDEVICE;
    }
    if (!best) return pa_fail(s, PA_EINVAL, "a cell does not fit the LDS of one workgroup");
    plan->cells_per_block = best;
    pack(cv_off, syn_off, best, plan->blk, plan->lds);
    if (upload_plan(s, *plan) != PA_OK) return PA_EDEVICE;
    // graph of G full epochs
    plan->graph_epochs = 8;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return pa_fail(s, PA_EDEVICE, "graph capture");
    int r = 0;
    for (uint32_t e = 0; e < plan->graph_epochs; ++e) r |= enqueue_epoch(d, *plan, d.K, st, nullptr, nullptr);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(st, &g) != hipSuccess || r) return pa_fail(s, PA_EDEVICE, "graph capture");
    plan->graph = g;
    if (hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0) != hipSuccess)
        return pa_fail(s, PA_EDEVICE, "graph instantiate");
    return PA_OK;
}

void batched_release(pa_sim *s) {
    BatchedPlan *&plan = pa_plan(s);
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    plan = nullptr;
}

uint32_t batched_cells_per_block(pa_sim *s) {
    BatchedPlan *p = pa_plan(s);
    return p ? p->cells_per_block : 0;
}

// One epoch (or a piece of one) of nsteps steps, launched directly.
pa_status run_epoch_batched(pa_sim *s, uint32_t nsteps, hipEvent_t e0, hipEvent_t e1) {
    const BatchedPlan &P = *pa_plan(s);
    if (enqueue_epoch(pa_devnet(s), P, nsteps, pa_stream(s), e0, e1))
        return pa_fail(s, PA_EDEVICE, "fused epoch launch");
    return PA_OK;
}

// Replays the captured graph: graph_epochs epochs of K steps.
pa_status run_graph_batched(pa_sim *s, uint32_t &steps_done) {
    const BatchedPlan &P = *pa_plan(s);
    if (hipGraphLaunch(P.exec, pa_stream(s)) != hipSuccess) return pa_fail(s, PA_EDEVICE, "graph launch");
    steps_done = P.graph_epochs * pa_devnet(s).K;
    return PA_OK;
}

uint32_t batched_graph_steps(pa_sim *s) {
    BatchedPlan *p = pa_plan(s);
    return p ? p->graph_epochs * pa_devnet(s).K : 0;
}
