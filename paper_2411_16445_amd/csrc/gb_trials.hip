// Batched trials of the calcium-based plasticity rule of Graupner and Brunel
// (Sec. 3.3, Eqs. 10-12, Table 3) under the pairing protocol of its DP
// curve: thousands of independent single synapses, one lane each, in one
// launch.  Every trial integrates the same protocol with its own delay
// between the presynaptic and the imposed postsynaptic spike, its own
// initial weight and its own noise stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/plasticarbor.h"
#include "sim.hpp"
#include "device_common.hpp"

namespace pa {
namespace {

struct GbK {
    double w_star, gamma_p, gamma_d, theta_p, theta_d, sigma, c_pre, c_post, t_cd;
    double ah, rc;                 // dt / tau_w, exp(-dt / tau_c)
    double dt, t0, period;
    uint64_t n_end, seed;
    uint32_t n_pairs;
};

// One trial per lane: per step n the calcium jumps due at n (presynaptic
// ones t_c,delay after the protocol's spikes, then the imposed postsynaptic
// ones), the Euler-Maruyama step of w from the step-start calcium with the
// threshold-gated noise, then the calcium's exact decay.
__global__ void k_gb_trials(GbK k, uint64_t n_trials, const double *__restrict__ delay,
                            const double *__restrict__ w0, double *__restrict__ w_out, double *__restrict__ c_out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_trials) return;
    const double dly = delay[i];
    double w = w0[i], c = 0.0;
    uint32_t kp = 0, kq = 0;
    // steps of the next presynaptic and postsynaptic jump
    auto pre_step = [&](uint32_t q) { return floor((k.t0 + (double)q * k.period + k.t_cd) / k.dt); };
    auto post_step = [&](uint32_t q) { return floor((k.t0 + (double)q * k.period + dly) / k.dt); };
    double np = kp < k.n_pairs ? pre_step(kp) : INFINITY;
    double nq = kq < k.n_pairs ? post_step(kq) : INFINITY;
    for (uint64_t n = 0; n < k.n_end; ++n) {
        const double nd = (double)n;
        while (np <= nd) {
            c += k.c_pre;
            ++kp;
            np = kp < k.n_pairs ? pre_step(kp) : INFINITY;
        }
        while (nq <= nd) {
            c += k.c_post;
            ++kq;
            nq = kq < k.n_pairs ? post_step(kq) : INFINITY;
        }
        const double thp = (c - k.theta_p > 0.0) ? 1.0 : 0.0;
        const double thd = (c - k.theta_d > 0.0) ? 1.0 : 0.0;
        const double drift = -w * (1.0 - w) * (k.w_star - w) + k.gamma_p * (1.0 - w) * thp - k.gamma_d * w * thd;
        double wn = w + k.ah * drift;
        if (thp + thd > 0.0) wn += noise_increment(k.seed, i, n, k.sigma, thp + thd, k.ah);
        w = wn;
        c = c * k.rc;
    }
    w_out[i] = w;
    if (c_out) c_out[i] = c;
}

}  // namespace
}  // namespace pa

extern "C" pa_status pa_gb_trials(const pa_gb_params *p, double dt_ms, uint64_t n_trials, const double *delay_ms,
                                  const double *w0, uint32_t n_pairs, double period_ms, double t0_ms,
                                  uint64_t seed, double *w_final, double *c_final, void *hip_stream) {
    if (!p) return PA_EINVAL;
    if (!(dt_ms > 0.0) || !std::isfinite(dt_ms) || !(p->tau_w > 0.0) || !(p->tau_c > 0.0) ||
        !std::isfinite(period_ms) || !std::isfinite(t0_ms) || !(p->sigma >= 0.0))
        return PA_EINVAL;
    if (n_trials == 0) return PA_OK;
    if (!delay_ms || !w0 || !w_final) return PA_EINVAL;
    const double span = std::floor((t0_ms + (double)n_pairs * period_ms) / dt_ms);
    if (!(span >= 0.0) || span > 1e12) return PA_ERANGE;
    pa::GbK k{p->w_star, p->gamma_p, p->gamma_d, p->theta_p, p->theta_d, p->sigma, p->c_pre, p->c_post, p->t_cd,
              dt_ms / p->tau_w, std::exp(-dt_ms / p->tau_c), dt_ms, t0_ms, period_ms, (uint64_t)span, seed, n_pairs};
    const uint32_t bs = 128;
    const uint64_t grid = (n_trials + bs - 1) / bs;
    if (grid > 0x7fffffffull) return PA_ERANGE;
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(pa::k_gb_trials, dim3((uint32_t)grid), dim3(bs), 0, st, k, n_trials, delay_ms, w0, w_final,
                       c_final);
    if (hipGetLastError() != hipSuccess) return PA_EDEVICE;
    return hipStreamSynchronize(st) == hipSuccess ? PA_OK : PA_EDEVICE;
}
