// C ABI of the engine: network description, validation, the host-side
// build of the device layout (invariants of the cable system, synapse
// ordering, connection table, event rings), device memory, and the epoch
// loop of pa_advance.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdarg>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/plasticarbor.h"
#include "sim.hpp"

using namespace pa;

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr uint64_t HIST_CAP = 1ull << 24;   // spikes held on the device per chunk
constexpr uint64_t SP_STAGE = 1ull << 16;   // spikes copied to the host per transfer
constexpr double QUEUE_BUDGET = 12.0 * (1ull << 30);  // bytes of per-epoch event queues the epoch length aims at

struct Alloc {
    void *p;
    size_t bytes;
};

}  // namespace

struct BatchedPlan;
struct pa_sim;
void batched_release(pa_sim *s);

struct pa_sim {
    pa_config cfg{};
    pa_stc_params stc{};
    int state = 0;  // 0 build, 1 ready, 2 failed
    std::string err;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool stream_set = false;  // caller chose a stream (possibly the null stream)
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *alloc_ctx = nullptr;
    std::vector<Alloc> allocs;
    size_t device_bytes = 0;

    // description (host)
    std::vector<int64_t> cv_off{0};
    std::vector<int32_t> parent;
    std::vector<double> length, diam;
    std::vector<uint8_t> mech;
    std::vector<int32_t> detector;
    std::vector<pa_cell_params> cparams;
    std::vector<uint32_t> syn_cell, syn_cv;
    std::vector<uint8_t> syn_kind;
    std::vector<double> syn_tau, syn_erev;
    std::vector<uint32_t> conn_src, conn_dst;
    std::vector<uint8_t> conn_ports;
    std::vector<double> conn_w, conn_d;
    std::vector<uint32_t> tr_dst;
    std::vector<uint8_t> tr_ports;
    std::vector<double> tr_w;
    std::vector<uint64_t> tr_off{0};
    std::vector<double> tr_t;
    std::vector<uint32_t> po_dst;
    std::vector<uint8_t> po_ports;
    std::vector<double> po_w, po_rate;
    std::vector<uint32_t> cl_cell, cl_cv;
    std::vector<double> cl_t0, cl_dur, cl_amp;
    std::vector<int32_t> pr_what;
    std::vector<uint64_t> pr_index;
    std::vector<uint32_t> pr_stride;
    double *ff_gdec = nullptr;    // per sorted synapse: conductance decay over a fast-forward step
    pa_stdp_params stdp{};        // STDP synapses
    bool stdp_set = false;
    bool dif_on = false;          // SPS / PRP diffusion model
    double dif_sps = 0.0, dif_prp = 0.0;

    // derived
    std::vector<uint32_t> syn_perm;   // sorted position -> synapse id
    std::vector<uint32_t> syn_rank;   // synapse id -> sorted position
    std::vector<uint32_t> hh_cv;      // HH CVs in CV order
    uint64_t n_stc = 0;
    DevNet d{};
    uint64_t step = 0;
    uint64_t events = 0;
    std::vector<uint32_t> sp_gid;
    std::vector<uint64_t> sp_step;
    std::vector<double> sp_t;
    bool spikes_sorted = true;
    std::vector<std::vector<double>> probe_samples;  // per probe
    std::vector<uint64_t> pr_off_host;                // region of each probe in the device buffer
    uint64_t pr_buf_len = 0;
    uint64_t drained_to = 0;      // steps whose probe samples the host holds
    Counters *ctr_host = nullptr; // pinned: copy of the device counters, then a zero word
    double *pr_host = nullptr;    // pinned staging of the probe buffer
    uint8_t *sp_host = nullptr;   // pinned staging of spikes: SP_STAGE x (gid, step, t)
    uint64_t queue_events = 0;    // capacity of the per-epoch queues
    double advance_ms = 0.0;
    BatchedPlan *plan = nullptr;        // batched form
    void *snap = nullptr;               // device copy of the mutable state (autotuning)
    uint64_t chunk = 0;  // steps between drains of the spike history

    // kernel timing
    bool timing = false;
    std::vector<hipEvent_t> tev;  // pairs
    size_t tev_used = 0;
    double timed_ms = 0.0;
    uint64_t timed_launches = 0;
};

namespace {

pa_status fail(pa_sim *s, pa_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
pa_status fail(pa_sim *s, pa_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    return st;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

pa_status hip_fail(pa_sim *s, hipError_t e, const char *what) {
    s->state = 2;
    return fail(s, PA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHECK(sim, expr, what)                          \
    do {                                                   \
        hipError_t e_ = (expr);                            \
        if (e_ != hipSuccess) return hip_fail(sim, e_, what); \
    } while (0)

void *dev_alloc(pa_sim *s, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (s->alloc_fn) {
        p = s->alloc_fn(bytes, s->alloc_ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) {
        s->allocs.push_back({p, bytes});
        s->device_bytes += bytes;
    }
    return p;
}

template <class T>
T *upload(pa_sim *s, const std::vector<T> &v, bool &ok) {
    if (!ok) return nullptr;
    T *p = (T *)dev_alloc(s, v.size() * sizeof(T));
    if (!p) { ok = false; return nullptr; }
    if (!v.empty() && hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        ok = false;
        return nullptr;
    }
    return p;
}

template <class T>
T *zeros(pa_sim *s, size_t n, bool &ok) {
    if (!ok) return nullptr;
    T *p = (T *)dev_alloc(s, n * sizeof(T));
    if (!p) { ok = false; return nullptr; }
    if (hipMemset(p, 0, std::max<size_t>(n * sizeof(T), 1)) != hipSuccess) { ok = false; return nullptr; }
    return p;
}

}  // namespace

// ======================================================================
extern "C" {

const char *pa_status_str(pa_status st) {
    switch (st) {
    case PA_OK: return "ok";
    case PA_EINVAL: return "invalid argument";
    case PA_ESTATE: return "call not allowed in this state";
    case PA_ENOMEM: return "out of memory";
    case PA_EDEVICE: return "device error";
    case PA_ERANGE: return "time or event out of range";
    case PA_EOVERFLOW: return "event queue or spike history overflow";
    case PA_ENUMERIC: return "non-finite membrane voltage";
    default: return "unknown status";
    }
}

const char *pa_last_error(const pa_sim *s) { return s ? s->err.c_str() : "null simulation"; }

pa_status pa_sim_create(const pa_config *cfg, const pa_stc_params *stc, pa_sim **out) {
    if (!cfg || !stc || !out) return PA_EINVAL;
    *out = nullptr;
    if (!finite_pos(cfg->dt_ms) || !std::isfinite(cfg->threshold_mV)) return PA_EINVAL;
    if (cfg->precision != PA_FP64 && cfg->precision != PA_MIXED) return PA_EINVAL;
    if (cfg->mode != PA_PLAIN && cfg->mode != PA_BATCHED) return PA_EINVAL;
    if (cfg->flags != 0) return PA_EINVAL;
    if (cfg->block_threads != 0 && cfg->block_threads != 64 && cfg->block_threads != 128 &&
        cfg->block_threads != 256)
        return PA_EINVAL;
    if (cfg->exchange > PA_EXCHANGE_RESIDENT) return PA_EINVAL;
    if (cfg->solver_waves > 3 || (cfg->block_threads && cfg->solver_waves &&
                                  cfg->block_threads > 64 && cfg->solver_waves >= cfg->block_threads / 64))
        return PA_EINVAL;
    const double taus[] = {stc->tau_c, stc->tau_h, stc->tau_p, stc->tau_z};
    for (double t : taus)
        if (!finite_pos(t)) return PA_EINVAL;
    const double vals[] = {stc->gamma_p, stc->gamma_d, stc->theta_p, stc->theta_d, stc->sigma_pl,
                           stc->p_max, stc->f_int, stc->t_cd, stc->h0, stc->theta_pro,
                           stc->theta_tag, stc->c_pre, stc->c_post};
    for (double v : vals)
        if (!std::isfinite(v)) return PA_EINVAL;
    if (!(stc->h0 > 0) || stc->t_cd < 0 || stc->sigma_pl < 0) return PA_EINVAL;
    pa_sim *s = new (std::nothrow) pa_sim();
    if (!s) return PA_ENOMEM;
    s->cfg = *cfg;
    s->stc = *stc;
    *out = s;
    return PA_OK;
}

void pa_sim_destroy(pa_sim *s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    batched_release(s);
    if (s->ctr_host) (void)hipHostFree(s->ctr_host);
    if (s->pr_host) (void)hipHostFree(s->pr_host);
    if (s->sp_host) (void)hipHostFree(s->sp_host);
    for (hipEvent_t e : s->tev) (void)hipEventDestroy(e);
    for (auto &a : s->allocs) {
        if (s->free_fn) s->free_fn(a.p, s->alloc_ctx);
        else (void)hipFree(a.p);
    }
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

pa_status pa_set_stream(pa_sim *s, void *stream) {
    if (!s) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "stream must be set before pa_finalize");
    s->stream = (hipStream_t)stream;
    s->own_stream = false;
    s->stream_set = stream != nullptr;
    return PA_OK;
}

pa_status pa_set_allocator(pa_sim *s, void *(*alloc)(size_t, void *), void (*release)(void *, void *),
                           void *ctx) {
    if (!s) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "allocator must be set before pa_finalize");
    if ((alloc == nullptr) != (release == nullptr)) return fail(s, PA_EINVAL, "alloc and release go together");
    s->alloc_fn = alloc;
    s->free_fn = release;
    s->alloc_ctx = ctx;
    return PA_OK;
}

pa_status pa_cells_add(pa_sim *s, uint32_t n, const int64_t *cv_off, const int32_t *parent,
                       const double *length, const double *diam, const uint8_t *mech,
                       const int32_t *detector, const pa_cell_params *params, uint32_t *first_gid) {
    if (!s) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "cells cannot be added after pa_finalize");
    if (n == 0) {
        if (first_gid) *first_gid = (uint32_t)(s->cv_off.size() - 1);
        return PA_OK;
    }
    if (!cv_off || !parent || !length || !diam || !mech || !detector || !params)
        return fail(s, PA_EINVAL, "null array");
    if (cv_off[0] != 0) return fail(s, PA_EINVAL, "cv_off[0] must be 0");
    if (s->cv_off.size() - 1 + (uint64_t)n > 0xffffffffull) return fail(s, PA_EINVAL, "too many cells");
    for (uint32_t c = 0; c < n; ++c) {
        const int64_t b0 = cv_off[c], b1 = cv_off[c + 1];
        if (b1 <= b0) return fail(s, PA_EINVAL, "cell %u has no CV", c);
        if (detector[c] < 0 || detector[c] >= b1 - b0) return fail(s, PA_EINVAL, "cell %u: detector CV out of range", c);
        const pa_cell_params &P = params[c];
        if (!finite_pos(P.cm) || !finite_pos(P.ra) || !std::isfinite(P.v_init) || !(P.g_pas >= 0) ||
            !std::isfinite(P.e_pas) || !(P.gna >= 0) || !(P.gk >= 0) || !(P.gl >= 0) ||
            !std::isfinite(P.ena) || !std::isfinite(P.ek) || !std::isfinite(P.el) || !std::isfinite(P.g_pas))
            return fail(s, PA_EINVAL, "cell %u: invalid membrane parameters", c);
        for (int64_t i = b0; i < b1; ++i) {
            const int32_t p = parent[i];
            if (i == b0 ? p != -1 : (p < 0 || p >= i - b0))
                return fail(s, PA_EINVAL, "cell %u: parent[0] must be -1 and 0 <= parent[i] < i", c);
            if (!finite_pos(length[i]) || !finite_pos(diam[i])) return fail(s, PA_EINVAL, "cell %u: CV geometry must be positive", c);
            if (mech[i] > 1) return fail(s, PA_EINVAL, "cell %u: unknown mechanism", c);
        }
    }
    const uint64_t total = (uint64_t)cv_off[n];
    if (s->cv_off.back() + total > 0xffffffffull) return fail(s, PA_EINVAL, "too many CVs");
    if (first_gid) *first_gid = (uint32_t)(s->cv_off.size() - 1);
    const int64_t base = s->cv_off.back();
    for (uint32_t c = 0; c < n; ++c) {
        s->cv_off.push_back(base + cv_off[c + 1]);
        s->detector.push_back(detector[c]);
        s->cparams.push_back(params[c]);
    }
    s->parent.insert(s->parent.end(), parent, parent + total);
    s->length.insert(s->length.end(), length, length + total);
    s->diam.insert(s->diam.end(), diam, diam + total);
    s->mech.insert(s->mech.end(), mech, mech + total);
    return PA_OK;
}

pa_status pa_synapses_add(pa_sim *s, uint32_t n, const uint32_t *gid, const uint32_t *cv,
                          const uint8_t *kind, const double *tau, const double *erev, uint32_t *first_sid) {
    if (!s) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "synapses cannot be added after pa_finalize");
    if (n && (!gid || !cv || !kind || !tau || !erev)) return fail(s, PA_EINVAL, "null array");
    const uint64_t ncell = s->cv_off.size() - 1;
    if (s->syn_cell.size() + (uint64_t)n > 0xffffffffull) return fail(s, PA_EINVAL, "too many synapses");
    for (uint32_t k = 0; k < n; ++k) {
        if (gid[k] >= ncell) return fail(s, PA_EINVAL, "synapse %u: unknown cell %u", k, gid[k]);
        if ((int64_t)cv[k] >= s->cv_off[gid[k] + 1] - s->cv_off[gid[k]]) return fail(s, PA_EINVAL, "synapse %u: CV out of range", k);
        if (kind[k] > 2) return fail(s, PA_EINVAL, "synapse %u: unknown kind", k);
        if (!finite_pos(tau[k]) || !std::isfinite(erev[k])) return fail(s, PA_EINVAL, "synapse %u: invalid tau or reversal", k);
    }
    if (first_sid) *first_sid = (uint32_t)s->syn_cell.size();
    s->syn_cell.insert(s->syn_cell.end(), gid, gid + n);
    s->syn_cv.insert(s->syn_cv.end(), cv, cv + n);
    s->syn_kind.insert(s->syn_kind.end(), kind, kind + n);
    s->syn_tau.insert(s->syn_tau.end(), tau, tau + n);
    s->syn_erev.insert(s->syn_erev.end(), erev, erev + n);
    return PA_OK;
}

pa_status pa_connect(pa_sim *s, uint64_t n, const uint32_t *src, const uint32_t *dst, const uint8_t *ports,
                     const double *w, const double *delay) {
    if (!s) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "connections cannot be added after pa_finalize");
    if (n && (!src || !dst || !ports || !w || !delay)) return fail(s, PA_EINVAL, "null array");
    const uint64_t ncell = s->cv_off.size() - 1, nsyn = s->syn_cell.size();
    if (s->conn_src.size() + n > 0xffffffffull) return fail(s, PA_EINVAL, "too many connections");
    for (uint64_t k = 0; k < n; ++k) {
        if (src[k] >= ncell) return fail(s, PA_EINVAL, "connection %llu: unknown source cell", (unsigned long long)k);
        if (dst[k] >= nsyn) return fail(s, PA_EINVAL, "connection %llu: unknown target synapse", (unsigned long long)k);
        if (ports[k] == 0 || ports[k] > 3) return fail(s, PA_EINVAL, "connection %llu: ports must be G, CA or both", (unsigned long long)k);
        if ((ports[k] & PA_PORT_CA) && s->syn_kind[dst[k]] != PA_SYN_STC)
            return fail(s, PA_EINVAL, "connection %llu: calcium port needs a PA_SYN_STC target", (unsigned long long)k);
        if (!std::isfinite(w[k])) return fail(s, PA_EINVAL, "connection %llu: weight not finite", (unsigned long long)k);
        if (!std::isfinite(delay[k]) || !(delay[k] >= s->cfg.dt_ms))
            return fail(s, PA_EINVAL, "connection %llu: delay %g below dt", (unsigned long long)k, delay[k]);
    }
    s->conn_src.insert(s->conn_src.end(), src, src + n);
    s->conn_dst.insert(s->conn_dst.end(), dst, dst + n);
    s->conn_ports.insert(s->conn_ports.end(), ports, ports + n);
    s->conn_w.insert(s->conn_w.end(), w, w + n);
    s->conn_d.insert(s->conn_d.end(), delay, delay + n);
    return PA_OK;
}

pa_status pa_trains_add(pa_sim *s, uint32_t n, const uint32_t *dst, const uint8_t *ports, const double *w,
                        const int64_t *off, const double *times) {
    if (!s) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "trains cannot be added after pa_finalize");
    if (n && (!dst || !ports || !w || !off)) return fail(s, PA_EINVAL, "null array");
    if (n && off[0] != 0) return fail(s, PA_EINVAL, "time_off[0] must be 0");
    const uint64_t nsyn = s->syn_cell.size();
    for (uint32_t k = 0; k < n; ++k) {
        if (dst[k] >= nsyn) return fail(s, PA_EINVAL, "train %u: unknown target synapse", k);
        if (ports[k] == 0 || ports[k] > 3) return fail(s, PA_EINVAL, "train %u: bad ports", k);
        if ((ports[k] & PA_PORT_CA) && s->syn_kind[dst[k]] != PA_SYN_STC)
            return fail(s, PA_EINVAL, "train %u: calcium port needs a PA_SYN_STC target", k);
        if (!std::isfinite(w[k])) return fail(s, PA_EINVAL, "train %u: weight not finite", k);
        if (off[k + 1] < off[k]) return fail(s, PA_EINVAL, "train %u: offsets decrease", k);
        if (off[k + 1] > off[k] && !times) return fail(s, PA_EINVAL, "null times");
        for (int64_t j = off[k]; j < off[k + 1]; ++j) {
            if (!std::isfinite(times[j]) || times[j] < 0) return fail(s, PA_EINVAL, "train %u: times must be finite and >= 0", k);
            if (j > off[k] && times[j] < times[j - 1]) return fail(s, PA_EINVAL, "train %u: times must not decrease", k);
        }
    }
    const uint64_t base = s->tr_off.back();
    for (uint32_t k = 0; k < n; ++k) {
        s->tr_dst.push_back(dst[k]);
        s->tr_ports.push_back(ports[k]);
        s->tr_w.push_back(w[k]);
        s->tr_off.push_back(base + (uint64_t)off[k + 1]);
    }
    if (n) s->tr_t.insert(s->tr_t.end(), times, times + off[n]);
    return PA_OK;
}

pa_status pa_poisson_add(pa_sim *s, uint32_t n, const uint32_t *dst, const uint8_t *ports, const double *w,
                         const double *rate) {
    if (!s) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "Poisson sources cannot be added after pa_finalize");
    if (n && (!dst || !ports || !w || !rate)) return fail(s, PA_EINVAL, "null array");
    const uint64_t nsyn = s->syn_cell.size();
    for (uint32_t k = 0; k < n; ++k) {
        if (dst[k] >= nsyn) return fail(s, PA_EINVAL, "Poisson source %u: unknown target synapse", k);
        if (ports[k] == 0 || ports[k] > 3) return fail(s, PA_EINVAL, "Poisson source %u: bad ports", k);
        if ((ports[k] & PA_PORT_CA) && s->syn_kind[dst[k]] != PA_SYN_STC)
            return fail(s, PA_EINVAL, "Poisson source %u: calcium port needs a PA_SYN_STC target", k);
        if (!std::isfinite(w[k]) || !std::isfinite(rate[k]) || rate[k] < 0)
            return fail(s, PA_EINVAL, "Poisson source %u: weight and rate must be finite, rate >= 0", k);
    }
    s->po_dst.insert(s->po_dst.end(), dst, dst + n);
    s->po_ports.insert(s->po_ports.end(), ports, ports + n);
    s->po_w.insert(s->po_w.end(), w, w + n);
    s->po_rate.insert(s->po_rate.end(), rate, rate + n);
    return PA_OK;
}

pa_status pa_clamps_add(pa_sim *s, uint32_t n, const uint32_t *gid, const uint32_t *cv, const double *t0,
                        const double *dur, const double *amp) {
    if (!s) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "clamps cannot be added after pa_finalize");
    if (n && (!gid || !cv || !t0 || !dur || !amp)) return fail(s, PA_EINVAL, "null array");
    const uint64_t ncell = s->cv_off.size() - 1;
    for (uint32_t k = 0; k < n; ++k) {
        if (gid[k] >= ncell || (int64_t)cv[k] >= s->cv_off[gid[k] + 1] - s->cv_off[gid[k]])
            return fail(s, PA_EINVAL, "clamp %u: bad cell or CV", k);
        if (!std::isfinite(t0[k]) || !(dur[k] >= 0) || !std::isfinite(amp[k]))
            return fail(s, PA_EINVAL, "clamp %u: bad time or amplitude", k);
    }
    for (uint32_t k = 0; k < n; ++k) {
        s->cl_cell.push_back(gid[k]);
        s->cl_cv.push_back(cv[k]);
        s->cl_t0.push_back(t0[k]);
        s->cl_dur.push_back(dur[k]);
        s->cl_amp.push_back(amp[k]);
    }
    return PA_OK;
}

pa_status pa_set_stdp(pa_sim *s, const pa_stdp_params *p) {
    if (!s || !p) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "STDP parameters are set before pa_finalize");
    if (!(p->tau_pre > 0.0) || !(p->tau_post > 0.0) || !std::isfinite(p->tau_pre) || !std::isfinite(p->tau_post) ||
        !std::isfinite(p->a_pre) || !std::isfinite(p->a_post) || !std::isfinite(p->w0) || !(p->w_max >= 0.0) ||
        !std::isfinite(p->w_max))
        return fail(s, PA_EINVAL, "STDP time constants must be positive and every parameter finite");
    s->stdp = *p;
    s->stdp_set = true;
    return PA_OK;
}

pa_status pa_set_diffusion(pa_sim *s, double d_sps, double d_prp) {
    if (!s) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "the protein model is set before pa_finalize");
    if (!(d_sps >= 0.0) || !(d_prp >= 0.0) || !std::isfinite(d_sps) || !std::isfinite(d_prp))
        return fail(s, PA_EINVAL, "diffusivities must be finite and >= 0");
    s->dif_on = true;
    s->dif_sps = d_sps;
    s->dif_prp = d_prp;
    return PA_OK;
}

pa_status pa_probes_add(pa_sim *s, uint32_t n, const int32_t *what, const uint64_t *index,
                        const uint32_t *stride_steps, uint32_t *first) {
    if (!s) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "probes cannot be added after pa_finalize");
    if (n && (!what || !index || !stride_steps)) return fail(s, PA_EINVAL, "null array");
    for (uint32_t k = 0; k < n; ++k) {
        const uint64_t i = index[k];
        if (stride_steps[k] == 0) return fail(s, PA_EINVAL, "probe %u: stride must be >= 1", k);
        switch (what[k]) {
        case PA_PROBE_V:
        case PA_PROBE_SPS:
        case PA_PROBE_PRP:
            if (i >= (uint64_t)s->cv_off.back()) return fail(s, PA_EINVAL, "probe %u: CV out of range", k);
            break;
        case PA_PROBE_G:
            if (i >= s->syn_cell.size()) return fail(s, PA_EINVAL, "probe %u: synapse out of range", k);
            break;
        case PA_PROBE_CA: case PA_PROBE_H: case PA_PROBE_Z:
            if (i >= s->syn_cell.size() || s->syn_kind[i] == PA_SYN_EXP)
                return fail(s, PA_EINVAL, "probe %u: needs a PA_SYN_STC or PA_SYN_STDP synapse", k);
            break;
        case PA_PROBE_P:
            if (i >= s->cv_off.size() - 1) return fail(s, PA_EINVAL, "probe %u: cell out of range", k);
            break;
        default: return fail(s, PA_EINVAL, "probe %u: unknown quantity", k);
        }
    }
    if (first) *first = (uint32_t)s->pr_what.size();
    s->pr_what.insert(s->pr_what.end(), what, what + n);
    s->pr_index.insert(s->pr_index.end(), index, index + n);
    s->pr_stride.insert(s->pr_stride.end(), stride_steps, stride_steps + n);
    return PA_OK;
}

}  // extern "C"

// ======================================================================
// Build of the device layout.
namespace {

pa_status build(pa_sim *s) {
    const uint32_t nc = (uint32_t)(s->cv_off.size() - 1);
    const uint32_t ncv = (uint32_t)s->cv_off.back();
    const uint32_t ns = (uint32_t)s->syn_cell.size();
    const double dt = s->cfg.dt_ms;
    DevNet &d = s->d;
    d = DevNet{};
    d.n_cells = nc;
    d.n_cv = ncv;
    d.n_syn = ns;
    d.n_trains = (uint32_t)s->tr_dst.size();
    d.n_probes = (uint32_t)s->pr_what.size();
    d.dt = dt;
    d.theta = s->cfg.threshold_mV;
    d.seed = s->cfg.seed;
    d.mixed = s->cfg.precision == PA_MIXED;
    const pa_stc_params &P = s->stc;
    d.stc = Stc{P.tau_c, P.tau_h, P.tau_p, P.tau_z, P.gamma_p, P.gamma_d, P.theta_p, P.theta_d,
                P.sigma_pl, P.p_max, P.f_int, P.t_cd, P.h0, P.theta_pro, P.theta_tag, P.c_pre, P.c_post};
    d.r_c = std::exp(-dt / P.tau_c);
    d.r_c_f = (float)d.r_c;
    if (s->stdp_set) {
        const pa_stdp_params &Q = s->stdp;
        d.stdp = StdpK{Q.a_pre, Q.a_post, Q.w_max, std::exp(-dt / Q.tau_pre), std::exp(-dt / Q.tau_post), 0.f};
        d.stdp.r_pre_f = (float)d.stdp.r_pre;
    }

    // ---- epoch length: spikes of an epoch may only be delivered after it
    double dmin = INFINITY, dmax = 0.0;
    for (double x : s->conn_d) { dmin = std::min(dmin, x); dmax = std::max(dmax, x); }
    uint32_t K;
    if (s->conn_d.empty()) K = 32;
    else {
        double q = dmin / dt;
        long k = (long)std::ceil(q - 1e-9) - 1;
        K = (uint32_t)std::max<long>(1, std::min<long>(k, 256));
        // The per-epoch queues hold, per incoming connection and port, the
        // most spikes a source can make in an epoch's window (K / 2 + 2);
        // with thousands of inputs per cell and long epochs that bound alone
        // would take tens of GB, so the epoch is shortened until it fits
        // QUEUE_BUDGET (any K up to the delay bound is exact).
        uint64_t ports = 0;
        for (uint8_t pr : s->conn_ports) ports += ((pr & 1) ? 1 : 0) + ((pr & 2) ? 1 : 0);
        while (K > 1 && 32.0 * (double)ports * (double)(K / 2 + 2) > QUEUE_BUDGET) K = std::max<uint32_t>(1, K * 3 / 4);
    }
    const double tcd = P.t_cd;
    d.K = K;
    // Spike rings.  An epoch's gather looks back in_lag steps from its first
    // step (the longest delay, calcium port included, plus a margin for the
    // crossing time and rounding), while the ring's own cell may already be
    // writing spikes of the running epoch; a cell crosses the threshold at
    // most every second step (V^n < theta <= V^{n+1} needs V back below
    // theta), so that many steps hold at most half as many spikes.
    const uint32_t lag_max = (uint32_t)std::ceil((dmax + tcd) / dt) + 3;
    {
        const uint32_t need = (lag_max + K + 1) / 2 + 2;
        uint32_t H = 1;
        while (H < need) H <<= 1;
        d.H = H;
    }

    // ---- synapse order (cell, CV, id) == (global CV, id)
    std::vector<uint32_t> &perm = s->syn_perm;
    perm.resize(ns);
    std::iota(perm.begin(), perm.end(), 0u);
    std::vector<uint32_t> gcv(ns);
    for (uint32_t k = 0; k < ns; ++k) gcv[k] = (uint32_t)s->cv_off[s->syn_cell[k]] + s->syn_cv[k];
    std::stable_sort(perm.begin(), perm.end(), [&](uint32_t a, uint32_t b) { return gcv[a] < gcv[b]; });
    s->syn_rank.assign(ns, 0);
    for (uint32_t q = 0; q < ns; ++q) s->syn_rank[perm[q]] = q;

    // ---- per-CV invariants of the cable system
    std::vector<int32_t> gparent(ncv);
    std::vector<double> cdt(ncv), gpas(ncv), gpas_e(ncv), axial(ncv, 0.0), d0(ncv);
    std::vector<double> dgeo(ncv, 0.0);  // cross-section / length of the CV-parent pair (diffusion)
    std::vector<int32_t> hh_of(ncv, -1);
    std::vector<uint32_t> hh_cv;
    std::vector<double> hh_scale, hh_par;
    std::vector<uint32_t> hh_off(nc + 1, 0), det(nc), cvoff(nc + 1);
    std::vector<double> V(ncv);
    for (uint32_t c = 0; c < nc; ++c) {
        const pa_cell_params &C = s->cparams[c];
        const uint32_t b0 = (uint32_t)s->cv_off[c], b1 = (uint32_t)s->cv_off[c + 1];
        cvoff[c] = b0;
        det[c] = b0 + (uint32_t)s->detector[c];
        hh_off[c] = (uint32_t)hh_cv.size();
        for (uint32_t i = b0; i < b1; ++i) {
            gparent[i] = (i == b0) ? -1 : (int32_t)(b0 + s->parent[i]);
            const double area = PI * s->diam[i] * s->length[i];   // lateral area, um^2
            cdt[i] = (1e-5 * C.cm * area) / dt;                     // C / dt in uS
            if (s->mech[i] == PA_MECH_HH) {
                hh_of[i] = (int32_t)hh_cv.size();
                hh_cv.push_back(i);
                hh_scale.push_back(1e-2 * area);
                const double pp[6] = {C.gna, C.gk, C.gl, C.ena, C.ek, C.el};
                hh_par.insert(hh_par.end(), pp, pp + 6);
                gpas[i] = 0.0;
                gpas_e[i] = 0.0;
            } else {
                gpas[i] = 1e-2 * C.g_pas * area;
                gpas_e[i] = gpas[i] * C.e_pas;
            }
            V[i] = C.v_init;
        }
        for (uint32_t i = b0 + 1; i < b1; ++i) {
            const uint32_t k = (uint32_t)gparent[i];
            const double ri = 0.5 * s->diam[i], rk = 0.5 * s->diam[k];
            const double rsum = s->length[i] / (2.0 * PI * ri * ri) + s->length[k] / (2.0 * PI * rk * rk);
            axial[i] = 1e2 / (C.ra * rsum);  // uS between the two CV centres
            dgeo[i] = 1.0 / rsum;            // um: the same series form for a diffusive flux
        }
    }
    cvoff[nc] = ncv;
    hh_off[nc] = (uint32_t)hh_cv.size();
    {
        std::vector<double> axsum(axial);
        for (uint32_t i = 0; i < ncv; ++i)
            if (gparent[i] >= 0) axsum[gparent[i]] += axial[i];
        for (uint32_t i = 0; i < ncv; ++i) d0[i] = (cdt[i] + gpas[i]) + axsum[i];
    }
    d.n_hh = (uint32_t)hh_cv.size();
    s->hh_cv = hh_cv;

    // ---- particle diffusion: CV volumes, per cell V_tot, and both species'
    // constant tree systems (V_i + dt sum a) X_i - dt sum a X_j eliminated
    // in the order of the Hines sweep
    std::vector<double> dvol, sps_u, sps_f, sps_dp, prp_u, prp_f, prp_dp, dif_thr, dif_pv;
    if (s->dif_on) {
        dvol.resize(ncv);
        dif_thr.resize(nc);
        dif_pv.resize(nc);
        for (uint32_t c = 0; c < nc; ++c) {
            double vt = 0.0;
            for (uint32_t i = cvoff[c]; i < cvoff[c + 1]; ++i) {
                const double r = 0.5 * s->diam[i];
                dvol[i] = PI * r * r * s->length[i];
                vt += dvol[i];
            }
            dif_thr[c] = P.theta_pro / vt;
            dif_pv[c] = P.p_max * vt;
        }
        auto factor = [&](double dc, std::vector<double> &U, std::vector<double> &F, std::vector<double> &Dp) {
            U.assign(ncv, 0.0);
            F.assign(ncv, 0.0);
            Dp = dvol;
            for (uint32_t c = 0; c < nc; ++c) {
                const uint32_t b0 = cvoff[c], b1 = cvoff[c + 1];
                for (uint32_t i = b0 + 1; i < b1; ++i) {
                    const double a = dt * (dc * dgeo[i]);
                    Dp[i] += a;
                    Dp[gparent[i]] += a;
                }
                for (uint32_t i = b1 - 1; i > b0; --i) {
                    const double u = -(dt * (dc * dgeo[i]));
                    const double f = u / Dp[i];
                    Dp[gparent[i]] -= f * u;
                    U[i] = u;
                    F[i] = f;
                }
            }
        };
        factor(s->dif_sps, sps_u, sps_f, sps_dp);
        factor(s->dif_prp, prp_u, prp_f, prp_dp);
    }
    for (int32_t w : s->pr_what)
        if ((w == PA_PROBE_SPS || w == PA_PROBE_PRP) && !s->dif_on)
            return fail(s, PA_EINVAL, "SPS / PRP probes need pa_set_diffusion");

    // ---- synapses in sorted order
    std::vector<uint32_t> ssid(ns), scell(ns), scv(ns), syn_off(nc + 1, 0), cv_syn_off(ncv + 1, 0);
    std::vector<uint8_t> skind(ns);
    std::vector<double> serev(ns), sdecay(ns), h(ns);
    std::vector<float> sdecay_f(ns);
    s->n_stc = 0;
    for (uint32_t q = 0; q < ns; ++q) {
        const uint32_t k = perm[q];
        ssid[q] = k;
        scell[q] = s->syn_cell[k];
        scv[q] = gcv[k];
        skind[q] = s->syn_kind[k];
        serev[q] = s->syn_erev[k];
        sdecay[q] = std::exp(-dt / s->syn_tau[k]);
        sdecay_f[q] = (float)sdecay[q];
        h[q] = skind[q] == PA_SYN_STC ? P.h0 : (skind[q] == PA_SYN_STDP ? s->stdp.w0 : 0.0);
        if (skind[q] == PA_SYN_STDP && !s->stdp_set) return fail(s, PA_EINVAL, "PA_SYN_STDP synapses need pa_set_stdp");
        s->n_stc += skind[q] == PA_SYN_STC;
        cv_syn_off[gcv[k] + 1]++;
        syn_off[scell[q] + 1]++;
    }
    for (uint32_t i = 0; i < ncv; ++i) cv_syn_off[i + 1] += cv_syn_off[i];
    for (uint32_t c = 0; c < nc; ++c) syn_off[c + 1] += syn_off[c];
    // per-CV decay factor where all of a CV's synapses share one
    std::vector<double> cv_dec(ncv, 1.0);
    bool dec_uniform = true;
    for (uint32_t i = 0; i < ncv; ++i)
        for (uint32_t q = cv_syn_off[i]; q < cv_syn_off[i + 1]; ++q) {
            if (q == cv_syn_off[i]) cv_dec[i] = sdecay[q];
            else if (sdecay[q] != cv_dec[i]) dec_uniform = false;
        }

    // ---- clamps sorted by (CV, id)
    const uint32_t ncl = (uint32_t)s->cl_cell.size();
    std::vector<uint32_t> clp(ncl), cl_cv_g(ncl), cv_cl_off(ncv + 1, 0);
    std::iota(clp.begin(), clp.end(), 0u);
    for (uint32_t k = 0; k < ncl; ++k) cl_cv_g[k] = (uint32_t)s->cv_off[s->cl_cell[k]] + s->cl_cv[k];
    std::stable_sort(clp.begin(), clp.end(), [&](uint32_t a, uint32_t b) { return cl_cv_g[a] < cl_cv_g[b]; });
    std::vector<double> clt0(ncl), cldur(ncl), clamp(ncl);
    for (uint32_t q = 0; q < ncl; ++q) {
        clt0[q] = s->cl_t0[clp[q]];
        cldur[q] = s->cl_dur[clp[q]];
        clamp[q] = s->cl_amp[clp[q]];
        cv_cl_off[cl_cv_g[clp[q]] + 1]++;
    }
    for (uint32_t i = 0; i < ncv; ++i) cv_cl_off[i + 1] += cv_cl_off[i];

    // ---- incoming connections by target cell, in connection id order
    const uint64_t ncon = s->conn_src.size();
    std::vector<uint64_t> in_off(nc + 1, 0);
    for (uint64_t k = 0; k < ncon; ++k) in_off[s->syn_cell[s->conn_dst[k]] + 1]++;
    for (uint32_t c = 0; c < nc; ++c) in_off[c + 1] += in_off[c];
    std::vector<uint32_t> in_src(ncon), in_syn(ncon), in_cid(ncon), in_lag(ncon);
    std::vector<uint8_t> in_ports(ncon);
    std::vector<double> in_w(ncon), in_d(ncon);
    // room of each cell's queue for one epoch: the events of an epoch's
    // steps come from source spikes within K + 2 steps, at most K / 2 + 2 of
    // them per source
    std::vector<uint64_t> qcap(nc, 0);
    const uint64_t spk_per_window = K / 2 + 2;
    {
        std::vector<uint64_t> fill(in_off.begin(), in_off.end() - 1);
        for (uint64_t k = 0; k < ncon; ++k) {
            const uint32_t tc = s->syn_cell[s->conn_dst[k]];
            const uint64_t q = fill[tc]++;
            in_src[q] = s->conn_src[k];
            in_syn[q] = s->syn_rank[s->conn_dst[k]];
            in_cid[q] = (uint32_t)k;
            in_ports[q] = s->conn_ports[k];
            in_w[q] = s->conn_w[k];
            in_d[q] = s->conn_d[k];
            const double dq = s->conn_d[k] + ((s->conn_ports[k] & PA_PORT_CA) ? tcd : 0.0);
            in_lag[q] = (uint32_t)std::ceil(dq / dt) + 3;
            qcap[tc] += spk_per_window * (uint64_t)(((s->conn_ports[k] & 1) ? 1 : 0) + ((s->conn_ports[k] & 2) ? 1 : 0));
        }
    }

    // ---- trains: their arrivals in any K consecutive steps, per port, add
    // to the target cell's queue room
    const uint32_t ntr = d.n_trains;
    std::vector<uint32_t> tr_syn(ntr), tr_cell(ntr);
    for (uint32_t k = 0; k < ntr; ++k) {
        tr_syn[k] = s->syn_rank[s->tr_dst[k]];
        tr_cell[k] = s->syn_cell[s->tr_dst[k]];
        for (uint32_t p = 1; p <= 2; ++p) {
            if (!(s->tr_ports[k] & p)) continue;
            uint64_t best = 0, a = s->tr_off[k];
            for (uint64_t j = s->tr_off[k]; j < s->tr_off[k + 1]; ++j) {
                const double tj = p == 2 ? s->tr_t[j] + tcd : s->tr_t[j];
                const double sj = std::floor(tj / dt);
                for (;;) {
                    const double ta = p == 2 ? s->tr_t[a] + tcd : s->tr_t[a];
                    if (std::floor(ta / dt) + K <= sj) ++a;
                    else break;
                }
                best = std::max<uint64_t>(best, j - a + 1);
            }
            qcap[tr_cell[k]] += best;
        }
    }

    // ---- Poisson sources: room for far more arrivals per epoch than their
    // rate makes likely (mean + 12 standard deviations + 16); a source that
    // exceeds its cell's room fails the advance with PA_EOVERFLOW
    const uint32_t npo = (uint32_t)s->po_dst.size();
    d.n_pois = npo;
    std::vector<uint32_t> po_syn(npo), po_cell(npo);
    for (uint32_t k = 0; k < npo; ++k) {
        po_syn[k] = s->syn_rank[s->po_dst[k]];
        po_cell[k] = s->syn_cell[s->po_dst[k]];
        const double m = s->po_rate[k] * 1e-3 * K * dt;
        const uint64_t cap = (uint64_t)std::ceil(m + 12.0 * std::sqrt(m) + 16.0);
        qcap[po_cell[k]] += cap * (uint64_t)(((s->po_ports[k] & 1) ? 1 : 0) + ((s->po_ports[k] & 2) ? 1 : 0));
    }
    std::vector<uint64_t> q_off(nc + 1, 0);
    for (uint32_t c = 0; c < nc; ++c) q_off[c + 1] = q_off[c] + qcap[c];
    s->queue_events = q_off[nc];

    // ---- trains and Poisson sources grouped by target cell
    std::vector<uint32_t> tr_cell_off(nc + 1, 0), tr_by_cell(ntr), po_cell_off(nc + 1, 0), po_by_cell(npo);
    for (uint32_t k = 0; k < ntr; ++k) tr_cell_off[tr_cell[k] + 1]++;
    for (uint32_t k = 0; k < npo; ++k) po_cell_off[po_cell[k] + 1]++;
    for (uint32_t c = 0; c < nc; ++c) {
        tr_cell_off[c + 1] += tr_cell_off[c];
        po_cell_off[c + 1] += po_cell_off[c];
    }
    {
        std::vector<uint32_t> ft(tr_cell_off.begin(), tr_cell_off.end() - 1), fp(po_cell_off.begin(), po_cell_off.end() - 1);
        for (uint32_t k = 0; k < ntr; ++k) tr_by_cell[ft[tr_cell[k]]++] = k;
        for (uint32_t k = 0; k < npo; ++k) po_by_cell[fp[po_cell[k]]++] = k;
    }

    // ---- probes: internal indices
    std::vector<uint64_t> pr_idx(d.n_probes);
    for (uint32_t k = 0; k < d.n_probes; ++k) {
        const int32_t w = s->pr_what[k];
        pr_idx[k] = (w >= PA_PROBE_G && w <= PA_PROBE_Z) ? s->syn_rank[s->pr_index[k]] : s->pr_index[k];
    }

    // ---- device memory
    bool ok = true;
    d.cv_off = upload(s, cvoff, ok);
    d.det_cv = upload(s, det, ok);
    d.syn_off = upload(s, syn_off, ok);
    d.hh_off = upload(s, hh_off, ok);
    d.p = zeros<double>(s, nc, ok);
    d.S = zeros<double>(s, nc, ok);
    d.vdet_old = zeros<double>(s, nc, ok);
    d.post = zeros<uint8_t>(s, nc, ok);
    d.parent = upload(s, gparent, ok);
    {
        // run length of parent == predecessor links ending at each CV
        std::vector<uint16_t> run(ncv, 0);
        for (uint32_t i = 0; i < ncv; ++i)
            if (gparent[i] >= 0 && (uint32_t)gparent[i] == i - 1) run[i] = (uint16_t)std::min<uint32_t>(run[i - 1] + 1u, 60000u);
        d.run = upload(s, run, ok);
        // branch segments per cell
        bool too_deep = false;
        std::vector<uint32_t> nkid(ncv, 0);
        for (uint32_t i = 0; i < ncv; ++i)
            if (gparent[i] >= 0) nkid[gparent[i]]++;
        std::vector<uint32_t> seg_off(nc + 1, 0), seg_a, seg_b, kid_off{0}, kids, seg_of(ncv);
        std::vector<uint8_t> seg_lvl;
        for (uint32_t c = 0; c < nc; ++c) {
            seg_off[c] = (uint32_t)seg_a.size();
            const uint32_t b0 = cvoff[c], b1 = cvoff[c + 1];
            for (uint32_t i = b0; i < b1; ++i) {
                const bool cont = i > b0 && (uint32_t)gparent[i] == i - 1 && nkid[i - 1] == 1;
                if (!cont) {
                    seg_a.push_back(i);
                    seg_b.push_back(i);
                    const uint32_t lvl = (i == b0) ? 0u : seg_lvl[seg_of[gparent[i]]] + 1u;
                    seg_lvl.push_back((uint8_t)std::min<uint32_t>(lvl, 255u));
                    if (lvl > 255) too_deep = true;
                } else {
                    seg_b.back() = i;
                }
                seg_of[i] = (uint32_t)seg_a.size() - 1;
            }
        }
        seg_off[nc] = (uint32_t)seg_a.size();
        const uint32_t nseg = (uint32_t)seg_a.size();
        // children of each segment's bottom node, in descending head index
        std::vector<std::vector<uint32_t>> ch(nseg);
        for (uint32_t g = 0; g < nseg; ++g)
            if (gparent[seg_a[g]] >= 0) ch[seg_of[gparent[seg_a[g]]]].push_back(g);
        for (uint32_t g = 0; g < nseg; ++g) {
            std::sort(ch[g].begin(), ch[g].end(), [&](uint32_t x, uint32_t y) { return seg_a[x] > seg_a[y]; });
            kids.insert(kids.end(), ch[g].begin(), ch[g].end());
            kid_off.push_back((uint32_t)kids.size());
        }
        d.n_seg = nseg;
        d.seg_off = upload(s, seg_off, ok);
        d.seg_a = upload(s, seg_a, ok);
        d.seg_b = upload(s, seg_b, ok);
        d.seg_lvl = upload(s, seg_lvl, ok);
        d.kid_off = upload(s, kid_off, ok);
        d.kids = upload(s, kids, ok);
        if (too_deep) return fail(s, PA_EINVAL, "a tree is deeper than 255 branch levels");
    }
    d.cdt = upload(s, cdt, ok);
    d.d0 = upload(s, d0, ok);
    d.gpas_e = upload(s, gpas_e, ok);
    d.axial = upload(s, axial, ok);
    d.hh_of = upload(s, hh_of, ok);
    d.cv_syn_off = upload(s, cv_syn_off, ok);
    d.cv_dec = upload(s, cv_dec, ok);
    d.cv_dec_uniform = dec_uniform ? 1u : 0u;
    // the conductances start at zero, and so do their carried sums
    if (d.mixed && dec_uniform) {
        d.gsum = zeros<double>(s, ncv, ok);
        d.gesum = zeros<double>(s, ncv, ok);
    }
    d.cv_cl_off = upload(s, cv_cl_off, ok);
    d.V = upload(s, V, ok);
    d.I = zeros<double>(s, ncv, ok);
    d.G = zeros<double>(s, ncv, ok);
    d.D = zeros<double>(s, ncv, ok);
    d.b = zeros<double>(s, ncv, ok);
    d.hh_cv = upload(s, hh_cv, ok);
    d.hh_scale = upload(s, hh_scale, ok);
    d.hh_par = upload(s, hh_par, ok);
    const size_t tsz = d.mixed ? 4 : 8;
    d.gm = zeros<uint8_t>(s, d.n_hh * tsz, ok);
    d.gh = zeros<uint8_t>(s, d.n_hh * tsz, ok);
    d.gn = zeros<uint8_t>(s, d.n_hh * tsz, ok);
    d.syn_cell = upload(s, scell, ok);
    d.syn_cv = upload(s, scv, ok);
    d.syn_kind = upload(s, skind, ok);
    d.syn_erev = upload(s, serev, ok);
    d.syn_decay = upload(s, sdecay, ok);
    d.syn_decay_f = upload(s, sdecay_f, ok);
    d.syn_sid = upload(s, ssid, ok);
    d.g = zeros<uint8_t>(s, (size_t)ns * tsz, ok);
    d.c = zeros<uint8_t>(s, (size_t)ns * tsz, ok);
    d.h = upload(s, h, ok);
    d.z = zeros<double>(s, ns, ok);
    d.ev_cnt = zeros<unsigned long long>(s, 2 * (size_t)ns, ok);
    d.ev_sum = zeros<unsigned long long>(s, 2 * (size_t)ns, ok);
    d.in_off = upload(s, in_off, ok);
    d.in_src = upload(s, in_src, ok);
    d.in_syn = upload(s, in_syn, ok);
    d.in_cid = upload(s, in_cid, ok);
    d.in_lag = upload(s, in_lag, ok);
    d.in_ports = upload(s, in_ports, ok);
    d.in_w = upload(s, in_w, ok);
    d.in_d = upload(s, in_d, ok);
    d.spk = zeros<SpikeRec>(s, (size_t)nc * d.H, ok);
    d.spk_n = zeros<uint32_t>(s, nc, ok);
    d.spk_last = zeros<uint32_t>(s, nc, ok);
    d.tr_syn = upload(s, tr_syn, ok);
    d.tr_cell = upload(s, tr_cell, ok);
    d.tr_ports = upload(s, s->tr_ports, ok);
    d.tr_w = upload(s, s->tr_w, ok);
    d.tr_t = upload(s, s->tr_t, ok);
    d.tr_off = upload(s, s->tr_off, ok);
    {
        // each train's two cursors start at its first arrival
        std::vector<uint64_t> cur(2 * (size_t)ntr);
        for (uint32_t k = 0; k < ntr; ++k) cur[2 * k] = cur[2 * k + 1] = s->tr_off[k];
        d.tr_cur = upload(s, cur, ok);
    }
    d.tr_cell_off = upload(s, tr_cell_off, ok);
    d.tr_by_cell = upload(s, tr_by_cell, ok);
    d.po_cell_off = upload(s, po_cell_off, ok);
    d.po_by_cell = upload(s, po_by_cell, ok);
    d.pois_syn = upload(s, po_syn, ok);
    d.pois_cell = upload(s, po_cell, ok);
    d.pois_ports = upload(s, s->po_ports, ok);
    d.pois_w = upload(s, s->po_w, ok);
    d.pois_rate = upload(s, s->po_rate, ok);
    d.pois_t = zeros<double>(s, 2 * (size_t)npo, ok);
    d.pois_j = zeros<uint64_t>(s, 2 * (size_t)npo, ok);
    d.cl_t0 = upload(s, clt0, ok);
    d.cl_dur = upload(s, cldur, ok);
    d.cl_amp = upload(s, clamp, ok);
    d.q_off = upload(s, q_off, ok);
    if (s->dif_on) {
        d.dif = 1;
        d.dvol = upload(s, dvol, ok);
        d.sps_u = upload(s, sps_u, ok);
        d.sps_f = upload(s, sps_f, ok);
        d.sps_dp = upload(s, sps_dp, ok);
        d.prp_u = upload(s, prp_u, ok);
        d.prp_f = upload(s, prp_f, ok);
        d.prp_dp = upload(s, prp_dp, ok);
        d.dif_thr = upload(s, dif_thr, ok);
        d.dif_pv = upload(s, dif_pv, ok);
        d.sps = zeros<double>(s, ncv, ok);
        d.prp = zeros<double>(s, ncv, ok);
        d.dlt = zeros<double>(s, ns, ok);
    }
    if (ok) {
        d.q_ev = (Event *)dev_alloc(s, std::max<uint64_t>(1, q_off[nc]) * sizeof(Event));
        if (!d.q_ev) ok = false;
    }
    if (s->cfg.mode == PA_PLAIN) {
        d.ev_n = zeros<uint32_t>(s, (size_t)nc * K, ok);
        d.ev_off = zeros<uint32_t>(s, (size_t)nc * K, ok);
    }
    d.blk_done = zeros<uint64_t>(s, std::max<size_t>(1, nc), ok);
    d.bar_grp = zeros<uint32_t>(s, 34 * 32, ok);  // 32 group counters, top counter, release word
    d.hist_cap = HIST_CAP;
    d.hist_gid = zeros<uint32_t>(s, HIST_CAP, ok);
    d.hist_step = zeros<uint64_t>(s, HIST_CAP, ok);
    d.hist_t = zeros<double>(s, HIST_CAP, ok);
    d.ctr = zeros<Counters>(s, 1, ok);
    d.pr_what = upload(s, s->pr_what, ok);
    d.pr_idx = upload(s, pr_idx, ok);
    d.pr_stride = upload(s, s->pr_stride, ok);
    // chunk of steps between drains: the history must hold every spike (a
    // cell crosses at most every second step) and the probe buffer every
    // sample (at most 8 M values); a whole number of epochs
    uint64_t chunk = std::max<uint64_t>(1, 2 * (d.hist_cap / std::max<uint32_t>(1, nc)));
    chunk = std::min<uint64_t>(chunk, 1u << 20);
    double per_step = 0.0;
    for (uint32_t str : s->pr_stride) per_step += 1.0 / str;
    if (per_step > 0) chunk = std::min<uint64_t>(chunk, std::max<uint64_t>(1, (uint64_t)((8u << 20) / per_step)));
    chunk = std::max<uint64_t>(chunk / K * K, K);
    s->chunk = chunk;
    s->pr_off_host.assign(d.n_probes + 1, 0);
    for (uint32_t k = 0; k < d.n_probes; ++k) s->pr_off_host[k + 1] = s->pr_off_host[k] + chunk / s->pr_stride[k] + 2;
    s->pr_buf_len = s->pr_off_host[d.n_probes];
    s->probe_samples.assign(d.n_probes, {});
    d.pr_off = upload(s, s->pr_off_host, ok);
    d.pr_buf = zeros<double>(s, std::max<uint64_t>(1, s->pr_buf_len), ok);
    if (ok && (hipHostMalloc((void **)&s->ctr_host, sizeof(Counters) + 64, hipHostMallocDefault) != hipSuccess ||
               hipHostMalloc((void **)&s->pr_host, std::max<uint64_t>(1, s->pr_buf_len) * 8, hipHostMallocDefault) != hipSuccess ||
               hipHostMalloc((void **)&s->sp_host, SP_STAGE * 20, hipHostMallocDefault) != hipSuccess))
        ok = false;
    if (ok) std::memset((uint8_t *)s->ctr_host + sizeof(Counters), 0, 64);
    if (!ok) return fail(s, PA_ENOMEM, "device allocation or upload failed (%.1f MB requested so far)",
                         s->device_bytes / 1048576.0);
    return PA_OK;
}

}  // namespace

// ----------------------------------------------------------------------
// Batched form (kernels_fused.hip).
struct BatchedPlan;
pa_status batched_setup(pa_sim *s);
void batched_release(pa_sim *s);
uint32_t batched_cells_per_block(pa_sim *s);
void batched_plan_shape(pa_sim *s, uint32_t &threads, uint32_t &solver_waves, uint32_t &exchange);
uint32_t batched_resident_steps(pa_sim *s);
pa_status run_resident_batched(pa_sim *s, uint32_t nsteps, hipEvent_t e0, hipEvent_t e1);
pa_status run_epoch_batched(pa_sim *s, uint32_t nsteps, hipEvent_t e0, hipEvent_t e1);
pa_status run_graph_batched(pa_sim *s, uint32_t &steps_done);
uint32_t batched_graph_steps(pa_sim *s);

extern "C" pa_status pa_finalize(pa_sim *s) {
    if (!s) return PA_EINVAL;
    if (s->state != 0) return fail(s, PA_ESTATE, "already finalized");
    if (s->cv_off.size() < 2) return fail(s, PA_EINVAL, "no cells");
    int ndev = 0;
    hipError_t de = hipGetDeviceCount(&ndev);
    if (de != hipSuccess || ndev == 0)
        return fail(s, PA_EDEVICE, "no HIP device (%s, count %d)", hipGetErrorString(de), ndev);
    if (!s->stream && !s->stream_set) {
        HIPCHECK(s, hipStreamCreate(&s->stream), "hipStreamCreate");
        s->own_stream = true;
    }
    pa_status st = build(s);
    if (st != PA_OK) return st;
    if (launch_init(s->d, s->stream)) return hip_fail(s, hipGetLastError(), "init kernel");
    if (s->cfg.mode == PA_BATCHED) {
        st = batched_setup(s);
        if (st != PA_OK) return st;
    }
    HIPCHECK(s, hipStreamSynchronize(s->stream), "finalize");
    s->state = 1;
    return PA_OK;
}

// ----------------------------------------------------------------------
// Epoch loop.
namespace {

// After an advance: reads the device counters and the probe samples of the
// steps since the last drain with one synchronisation of the stream, then
// the spikes recorded (if any) and resets the spike history.
pa_status drain(pa_sim *s) {
    DevNet &d = s->d;
    const uint64_t first = s->drained_to, last = s->step;
    HIPCHECK(s, hipMemcpyAsync(s->ctr_host, d.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s->stream), "read counters");
    bool samples = false;
    for (uint32_t k = 0; k < d.n_probes; ++k) samples |= last / s->pr_stride[k] > first / s->pr_stride[k];
    if (samples)
        HIPCHECK(s, hipMemcpyAsync(s->pr_host, d.pr_buf, s->pr_buf_len * 8, hipMemcpyDeviceToHost, s->stream), "read probes");
    HIPCHECK(s, hipStreamSynchronize(s->stream), "drain");
    const Counters c = *s->ctr_host;
    for (uint32_t k = 0; samples && k < d.n_probes; ++k) {
        const uint64_t m = last / s->pr_stride[k] - first / s->pr_stride[k];
        const double *src = s->pr_host + s->pr_off_host[k];
        s->probe_samples[k].insert(s->probe_samples[k].end(), src, src + m);
    }
    s->drained_to = last;
    if (c.hist_n) {
        const uint64_t n = std::min<uint64_t>(c.hist_n, d.hist_cap);
        const size_t n0 = s->sp_gid.size();
        s->sp_gid.resize(n0 + n);
        s->sp_step.resize(n0 + n);
        s->sp_t.resize(n0 + n);
        uint32_t *hg = (uint32_t *)s->sp_host;
        uint64_t *hs = (uint64_t *)(s->sp_host + SP_STAGE * 4);
        double *ht = (double *)(s->sp_host + SP_STAGE * 12);
        for (uint64_t a = 0; a < n; a += SP_STAGE) {
            const uint64_t m = std::min<uint64_t>(SP_STAGE, n - a);
            HIPCHECK(s, hipMemcpyAsync(hg, d.hist_gid + a, m * 4, hipMemcpyDeviceToHost, s->stream), "read spikes");
            HIPCHECK(s, hipMemcpyAsync(hs, d.hist_step + a, m * 8, hipMemcpyDeviceToHost, s->stream), "read spikes");
            HIPCHECK(s, hipMemcpyAsync(ht, d.hist_t + a, m * 8, hipMemcpyDeviceToHost, s->stream), "read spikes");
            HIPCHECK(s, hipStreamSynchronize(s->stream), "drain");
            std::memcpy(s->sp_gid.data() + n0 + a, hg, m * 4);
            std::memcpy(s->sp_step.data() + n0 + a, hs, m * 8);
            std::memcpy(s->sp_t.data() + n0 + a, ht, m * 8);
        }
        s->spikes_sorted = false;
        // the next advance starts an empty history (ordered before its kernels)
        HIPCHECK(s, hipMemcpyAsync(&d.ctr->hist_n, (uint8_t *)s->ctr_host + sizeof(Counters), 8,
                                   hipMemcpyHostToDevice, s->stream), "reset history");
    }
    if (c.flags) {
        s->state = 2;
        if (c.flags & FLAG_NONFINITE) return fail(s, PA_ENUMERIC, "non-finite voltage in cell %u", c.bad_cell);
        if (c.flags & FLAG_QUEUE)
            return fail(s, PA_EOVERFLOW, "the events of one epoch exceeded the queue of the cells from cell %u "
                                         "(Poisson arrivals far above their rate)", c.bad_cell);
        if (c.flags & FLAG_HISTORY) return fail(s, PA_EOVERFLOW, "spike history overflowed (cell %u)", c.bad_cell);
        if (c.flags & FLAG_BARRIER) return fail(s, PA_EDEVICE, "grid barrier of the multi-epoch kernel timed out");
        return fail(s, PA_ERANGE, "an event of a spike of cell %u was due before the spike", c.bad_cell);
    }
    return PA_OK;
}


// Sums the durations of completed timed launches and recycles their events.
pa_status fold_timing(pa_sim *s) {
    if (!s->tev_used) return PA_OK;
    HIPCHECK(s, hipStreamSynchronize(s->stream), "timing");
    for (size_t k = 0; k < s->tev_used; k += 2) {
        float ms = 0.f;
        HIPCHECK(s, hipEventElapsedTime(&ms, s->tev[k], s->tev[k + 1]), "elapsed");
        s->timed_ms += ms;
        s->timed_launches++;
    }
    s->tev_used = 0;
    return PA_OK;
}

// A pair of events bracketing the next launch of the timed kernel.
pa_status timing_events(pa_sim *s, hipEvent_t &b, hipEvent_t &e) {
    if (s->tev_used >= 16384 && fold_timing(s) != PA_OK) return PA_EDEVICE;
    if (s->tev_used + 2 > s->tev.size()) {
        hipEvent_t x, y;
        HIPCHECK(s, hipEventCreate(&x), "event");
        HIPCHECK(s, hipEventCreate(&y), "event");
        s->tev.push_back(x);
        s->tev.push_back(y);
    }
    b = s->tev[s->tev_used];
    e = s->tev[s->tev_used + 1];
    s->tev_used += 2;
    return PA_OK;
}

}  // namespace

// The first step after `after` at which some probe samples (UINT64_MAX
// without probes).
static uint64_t next_sample(const pa_sim *s, uint64_t after) {
    uint64_t best = UINT64_MAX;
    for (uint32_t str : s->pr_stride) best = std::min<uint64_t>(best, (after / str + 1) * str);
    return best;
}

extern "C" pa_status pa_advance_steps(pa_sim *s, uint64_t n_steps) {
    if (!s) return PA_EINVAL;
    if (s->state == 0) return fail(s, PA_ESTATE, "pa_finalize first");
    if (s->state == 2) return fail(s, PA_ESTATE, "simulation failed earlier: %s", s->err.c_str());
    if (n_steps == 0) return PA_OK;
    if (s->step + n_steps >= 0xffffffffull) return fail(s, PA_ERANGE, "step counts beyond 2^32 - 1 are not supported");
    auto t_start = std::chrono::steady_clock::now();
    DevNet &d = s->d;
    const uint64_t chunk = s->chunk;
    const uint64_t n_end = s->step + n_steps;
    while (s->step < n_end) {
        const uint64_t c_end = std::min(n_end, s->step + chunk);
        while (s->step < c_end) {
            const uint64_t e0 = s->step;
            const uint64_t sample = next_sample(s, e0);
            if (s->cfg.mode == PA_BATCHED) {
                // epochs end at probe samples
                const uint64_t stop = std::min(c_end, sample);
                const uint32_t max_res = batched_resident_steps(s);
                const uint32_t gsteps = batched_graph_steps(s);
                hipEvent_t tb = nullptr, te = nullptr;
                if (max_res) {
                    // steps in one resident launch
                    const uint32_t ns = (uint32_t)std::min<uint64_t>(stop - e0, max_res);
                    if (s->timing && timing_events(s, tb, te) != PA_OK) return PA_EDEVICE;
                    pa_status st = run_resident_batched(s, ns, tb, te);
                    if (st != PA_OK) return st;
                    s->step = e0 + ns;
                } else if (!s->timing && gsteps && stop - e0 >= gsteps) {
                    // replay the captured graph of whole epochs
                    uint32_t done = 0;
                    pa_status st = run_graph_batched(s, done);
                    if (st != PA_OK) return st;
                    s->step = e0 + done;
                } else {
                    const uint64_t e1 = std::min(stop, e0 + d.K);
                    if (s->timing && timing_events(s, tb, te) != PA_OK) return PA_EDEVICE;
                    pa_status st = run_epoch_batched(s, (uint32_t)(e1 - e0), tb, te);
                    if (st != PA_OK) return st;
                    s->step = e1;
                }
                if (s->step == sample && launch_probe(d, sample, s->drained_to, s->stream))
                    return hip_fail(s, hipGetLastError(), "probe");
                continue;
            }
            // plain form: gather the epoch's events, then one kernel per stage
            // and step; probes after the steps they sample
            const uint64_t e1 = std::min(c_end, e0 + d.K);
            if (launch_gather(d, e0, (uint32_t)(e1 - e0), s->stream)) return hip_fail(s, hipGetLastError(), "gather");
            uint64_t smp = sample;
            for (uint64_t n = e0; n < e1; ++n) {
                hipEvent_t tb = nullptr, te = nullptr;
                if (s->timing && timing_events(s, tb, te) != PA_OK) return PA_EDEVICE;
                if (launch_step_plain(d, n, e0, s->stream, tb, te)) return hip_fail(s, hipGetLastError(), "step");
                if (n + 1 == smp) {
                    if (launch_probe(d, n + 1, s->drained_to, s->stream)) return hip_fail(s, hipGetLastError(), "probe");
                    smp = next_sample(s, n + 1);
                }
            }
            s->step = e1;
        }
        pa_status st = drain(s);
        if (st != PA_OK) return st;
    }
    if (s->timing && fold_timing(s) != PA_OK) return PA_EDEVICE;
    s->advance_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return PA_OK;
}

extern "C" pa_status pa_advance(pa_sim *s, double t_until) {
    if (!s) return PA_EINVAL;
    if (s->state == 0) return fail(s, PA_ESTATE, "pa_finalize first");
    if (!std::isfinite(t_until)) return fail(s, PA_ERANGE, "time not finite");
    const double dt = s->cfg.dt_ms;
    const double q = t_until / dt;
    const double nr = std::nearbyint(q);
    if (std::fabs(nr * dt - t_until) > 1e-9 * std::max(1.0, std::fabs(t_until)) || nr < 0)
        return fail(s, PA_ERANGE, "t = %.17g is not on the dt grid", t_until);
    const uint64_t target = (uint64_t)nr;
    if (target < s->step) return fail(s, PA_ERANGE, "t = %g lies before the present time %g", t_until, s->step * dt);
    return pa_advance_steps(s, target - s->step);
}

// ----------------------------------------------------------------------
// Fast-forward and the device state dump.
extern "C" pa_status pa_retune(pa_sim *s) {
    if (!s) return PA_EINVAL;
    if (s->state == 0) return fail(s, PA_ESTATE, "pa_finalize first");
    if (s->state == 2) return fail(s, PA_ESTATE, "simulation failed earlier: %s", s->err.c_str());
    if (s->cfg.mode != PA_BATCHED) return fail(s, PA_EINVAL, "only the batched form has a plan to tune");
    // the grid barrier counts the barriers of the present plan (per
    // workgroup, per group of workgroups): a new plan starts them at zero,
    // as pa_finalize's allocation does
    HIPCHECK(s, hipMemsetAsync(s->d.bar_grp, 0, 34 * 32 * sizeof(uint32_t), s->stream), "retune");
    HIPCHECK(s, hipMemsetAsync(s->d.blk_done, 0, (size_t)s->d.n_cells * sizeof(uint64_t), s->stream), "retune");
    HIPCHECK(s, hipStreamSynchronize(s->stream), "retune");
    // the trials run from the present state and restore it (as at
    // pa_finalize); the old plan's block table stays allocated with the
    // simulation's other memory
    batched_release(s);
    const pa_status st = batched_setup(s);
    if (st != PA_OK) s->state = 2;
    return st;
}

extern "C" pa_status pa_fast_forward(pa_sim *s, uint64_t n_long, double dt_long) {
    if (!s) return PA_EINVAL;
    if (s->state == 0) return fail(s, PA_ESTATE, "pa_finalize first");
    if (s->state == 2) return fail(s, PA_ESTATE, "simulation failed earlier: %s", s->err.c_str());
    if (s->dif_on) return fail(s, PA_EINVAL, "fast-forward needs the per-cell protein model");
    const double dt = s->cfg.dt_ms;
    if (!std::isfinite(dt_long) || !(dt_long > 0.0)) return fail(s, PA_EINVAL, "dt_long must be positive");
    const double ratio_f = std::floor(dt_long / dt + 0.5);
    if (ratio_f < 1.0 || std::fabs(ratio_f * dt - dt_long) > 1e-9 * dt_long)
        return fail(s, PA_EINVAL, "dt_long must be a whole multiple of dt");
    const uint64_t ratio = (uint64_t)ratio_f;
    if (n_long == 0) return PA_OK;
    if (n_long > (0xffffffffull - s->step) / ratio) return fail(s, PA_ERANGE, "step counts beyond 2^32 - 1 are not supported");
    const uint64_t n_new = s->step + n_long * ratio;
    DevNet &d = s->d;
    const uint32_t ns = d.n_syn;
    if (!s->ff_gdec && ns) {
        s->ff_gdec = (double *)dev_alloc(s, (size_t)ns * 8);
        if (!s->ff_gdec) return fail(s, PA_ENOMEM, "fast-forward factors");
    }
    if (ns) {
        std::vector<double> gd(ns);
        for (uint32_t q = 0; q < ns; ++q) gd[q] = std::exp(-dt_long / s->syn_tau[s->syn_perm[q]]);
        HIPCHECK(s, hipMemcpyAsync(s->ff_gdec, gd.data(), (size_t)ns * 8, hipMemcpyHostToDevice, s->stream), "factors");
        HIPCHECK(s, hipStreamSynchronize(s->stream), "factors");
    }
    const double rc = std::exp(-dt_long / s->stc.tau_c);
    if (launch_fast_forward(d, n_long, dt_long, s->ff_gdec, rc, n_new, s->stream))
        return hip_fail(s, hipGetLastError(), "fast-forward");
    // train cursors: both ports at the first arrival from the new time on
    const uint32_t ntr = d.n_trains;
    if (ntr) {
        std::vector<uint64_t> cur(2 * (size_t)ntr);
        for (uint32_t k = 0; k < ntr; ++k) {
            uint64_t j = s->tr_off[k];
            while (j < s->tr_off[k + 1] && std::floor(s->tr_t[j] / dt) < (double)n_new) ++j;
            cur[2 * k] = cur[2 * k + 1] = j;
        }
        HIPCHECK(s, hipMemcpyAsync((void *)d.tr_cur, cur.data(), cur.size() * 8, hipMemcpyHostToDevice, s->stream), "cursors");
        HIPCHECK(s, hipStreamSynchronize(s->stream), "cursors");
    }
    // new conductances: their carried per-CV sums follow
    if (d.gsum && launch_carried_sums(d, s->stream) != 0) return fail(s, PA_EDEVICE, "carried sums");
    // the epoch counter the kernels start from
    Counters c{};
    HIPCHECK(s, hipMemcpyAsync(&c, d.ctr, sizeof c, hipMemcpyDeviceToHost, s->stream), "counters");
    HIPCHECK(s, hipStreamSynchronize(s->stream), "counters");
    c.step = n_new;
    HIPCHECK(s, hipMemcpyAsync(d.ctr, &c, sizeof c, hipMemcpyHostToDevice, s->stream), "counters");
    HIPCHECK(s, hipStreamSynchronize(s->stream), "fast-forward");
    s->step = n_new;
    s->drained_to = n_new;
    return PA_OK;
}

namespace {

struct StateHeader {
    uint64_t magic, version, n_cells, n_cv, n_syn, n_pois, n_trains, step, mixed, dif, bytes;
};
constexpr uint64_t STATE_MAGIC = 0x5041535441544531ull;  // "PASTATE1"

// The mutable device arrays of a simulation (the same list the autotuning
// snapshot saves), each padded to 256 bytes in the dump.
struct Span { void *p; size_t n; };
std::vector<Span> mutable_spans(pa_sim *s) {
    DevNet &d = s->d;
    const size_t t = d.mixed ? 4 : 8;
    return {
        {d.V, (size_t)d.n_cv * 8}, {d.gm, (size_t)d.n_hh * t}, {d.gh, (size_t)d.n_hh * t},
        {d.gn, (size_t)d.n_hh * t}, {d.g, (size_t)d.n_syn * t}, {d.c, (size_t)d.n_syn * t},
        {d.h, (size_t)d.n_syn * 8}, {d.z, (size_t)d.n_syn * 8}, {d.p, (size_t)d.n_cells * 8},
        {d.S, (size_t)d.n_cells * 8}, {d.vdet_old, (size_t)d.n_cells * 8}, {d.post, (size_t)d.n_cells},
        {d.ev_cnt, (size_t)d.n_syn * 16}, {d.ev_sum, (size_t)d.n_syn * 16},
        {d.gsum, d.gsum ? (size_t)d.n_cv * 8 : 0}, {d.gesum, d.gesum ? (size_t)d.n_cv * 8 : 0},
        {d.spk, (size_t)d.n_cells * d.H * sizeof(SpikeRec)}, {d.spk_n, (size_t)d.n_cells * 4},
        {d.spk_last, (size_t)d.n_cells * 4},
        {d.tr_cur, (size_t)d.n_trains * 16},
        {d.pois_t, (size_t)d.n_pois * 16}, {d.pois_j, (size_t)d.n_pois * 16},
        {d.sps, d.sps ? (size_t)d.n_cv * 8 : 0}, {d.prp, d.prp ? (size_t)d.n_cv * 8 : 0}};
}

uint64_t dump_bytes(pa_sim *s) {
    uint64_t total = 256;  // header
    for (const Span &x : mutable_spans(s)) total += (x.n + 255) & ~size_t(255);
    return total;
}

StateHeader header_of(pa_sim *s) {
    const DevNet &d = s->d;
    return StateHeader{STATE_MAGIC, 1, d.n_cells, d.n_cv, d.n_syn, d.n_pois, d.n_trains, s->step,
                       d.mixed, d.dif, dump_bytes(s)};
}

}  // namespace

extern "C" pa_status pa_state_size(pa_sim *s, uint64_t *bytes) {
    if (!s || !bytes) return PA_EINVAL;
    if (s->state == 0) return fail(s, PA_ESTATE, "pa_finalize first");
    *bytes = dump_bytes(s);
    return PA_OK;
}

extern "C" pa_status pa_state_save(pa_sim *s, void *buf, uint64_t bytes) {
    if (!s || !buf) return PA_EINVAL;
    if (s->state == 0) return fail(s, PA_ESTATE, "pa_finalize first");
    const StateHeader H = header_of(s);
    if (bytes < H.bytes) return fail(s, PA_EINVAL, "state dump needs %llu bytes", (unsigned long long)H.bytes);
    HIPCHECK(s, hipStreamSynchronize(s->stream), "sync");
    HIPCHECK(s, hipMemcpyAsync(buf, &H, sizeof H, hipMemcpyDefault, s->stream), "state save");
    uint64_t off = 256;
    for (const Span &x : mutable_spans(s)) {
        if (x.n) HIPCHECK(s, hipMemcpyAsync((uint8_t *)buf + off, x.p, x.n, hipMemcpyDefault, s->stream), "state save");
        off += (x.n + 255) & ~size_t(255);
    }
    HIPCHECK(s, hipStreamSynchronize(s->stream), "state save");
    return PA_OK;
}

extern "C" pa_status pa_state_load(pa_sim *s, const void *buf, uint64_t bytes) {
    if (!s || !buf) return PA_EINVAL;
    if (s->state == 0) return fail(s, PA_ESTATE, "pa_finalize first");
    StateHeader H{}, want = header_of(s);
    if (bytes < sizeof H) return fail(s, PA_EINVAL, "state dump too short");
    HIPCHECK(s, hipStreamSynchronize(s->stream), "sync");
    HIPCHECK(s, hipMemcpyAsync(&H, buf, sizeof H, hipMemcpyDefault, s->stream), "state load");
    HIPCHECK(s, hipStreamSynchronize(s->stream), "state load");
    if (H.magic != STATE_MAGIC || H.version != want.version || H.n_cells != want.n_cells || H.n_cv != want.n_cv ||
        H.n_syn != want.n_syn || H.n_pois != want.n_pois || H.n_trains != want.n_trains || H.mixed != want.mixed ||
        H.dif != want.dif || H.bytes != want.bytes || bytes < H.bytes)
        return fail(s, PA_EINVAL, "state dump does not belong to a network of this shape and form");
    if (H.step >= 0xffffffffull) return fail(s, PA_EINVAL, "state dump step out of range");
    uint64_t off = 256;
    for (const Span &x : mutable_spans(s)) {
        if (x.n) HIPCHECK(s, hipMemcpyAsync(x.p, (const uint8_t *)buf + off, x.n, hipMemcpyDefault, s->stream), "state load");
        off += (x.n + 255) & ~size_t(255);
    }
    Counters c{};
    HIPCHECK(s, hipMemcpyAsync(&c, s->d.ctr, sizeof c, hipMemcpyDeviceToHost, s->stream), "counters");
    HIPCHECK(s, hipStreamSynchronize(s->stream), "counters");
    c.step = H.step;
    c.flags = 0;
    HIPCHECK(s, hipMemcpyAsync(s->d.ctr, &c, sizeof c, hipMemcpyHostToDevice, s->stream), "counters");
    HIPCHECK(s, hipStreamSynchronize(s->stream), "state load");
    s->step = H.step;
    s->drained_to = H.step;
    if (s->state == 2) s->state = 1;
    return PA_OK;
}

// ----------------------------------------------------------------------
extern "C" pa_status pa_spikes_count(const pa_sim *s, uint64_t *n) {
    if (!s || !n) return PA_EINVAL;
    *n = s->sp_gid.size();
    return PA_OK;
}

extern "C" pa_status pa_spikes_read(const pa_sim *cs, uint32_t *gid, uint64_t *step, double *t, uint64_t cap,
                                    uint64_t *n) {
    if (!cs || !n) return PA_EINVAL;
    pa_sim *s = const_cast<pa_sim *>(cs);
    if (!s->spikes_sorted) {
        const size_t m = s->sp_gid.size();
        std::vector<size_t> idx(m);
        std::iota(idx.begin(), idx.end(), 0);
        std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
            if (s->sp_t[a] != s->sp_t[b]) return s->sp_t[a] < s->sp_t[b];
            return s->sp_gid[a] < s->sp_gid[b];
        });
        std::vector<uint32_t> g2(m);
        std::vector<uint64_t> s2(m);
        std::vector<double> t2(m);
        for (size_t k = 0; k < m; ++k) { g2[k] = s->sp_gid[idx[k]]; s2[k] = s->sp_step[idx[k]]; t2[k] = s->sp_t[idx[k]]; }
        s->sp_gid.swap(g2);
        s->sp_step.swap(s2);
        s->sp_t.swap(t2);
        s->spikes_sorted = true;
    }
    const uint64_t m = std::min<uint64_t>(cap, s->sp_gid.size());
    for (uint64_t k = 0; k < m; ++k) {
        if (gid) gid[k] = s->sp_gid[k];
        if (step) step[k] = s->sp_step[k];
        if (t) t[k] = s->sp_t[k];
    }
    *n = m;
    return PA_OK;
}

extern "C" pa_status pa_probe_count(const pa_sim *s, uint32_t probe_id, uint64_t *n) {
    if (!s || !n) return PA_EINVAL;
    if (probe_id >= s->probe_samples.size()) return PA_EINVAL;
    *n = s->probe_samples[probe_id].size();
    return PA_OK;
}

extern "C" pa_status pa_probe_read(const pa_sim *s, uint32_t probe_id, double *out, uint64_t cap, uint64_t *n) {
    if (!s || !n || (cap && !out)) return PA_EINVAL;
    if (probe_id >= s->probe_samples.size()) return PA_EINVAL;
    const std::vector<double> &v = s->probe_samples[probe_id];
    const uint64_t m = std::min<uint64_t>(cap, v.size());
    if (m) std::memcpy(out, v.data(), m * 8);
    *n = m;
    return PA_OK;
}

namespace {

// (device pointer, element size, count, permutation kind): 0 identity,
// 1 synapse (device sorted -> id order), 2 HH (CV order == slot order)
struct View {
    void *p;
    size_t esize;
    uint64_t n;
    int perm;
    bool narrow;  // FP32 storage widened on read
};

bool view_of(pa_sim *s, int32_t what, View &v) {
    DevNet &d = s->d;
    const bool m = d.mixed;
    switch (what) {
    case PA_STATE_V: v = {d.V, 8, d.n_cv, 0, false}; return true;
    case PA_STATE_M: v = {d.gm, m ? 4u : 8u, d.n_hh, 0, m}; return true;
    case PA_STATE_HHH: v = {d.gh, m ? 4u : 8u, d.n_hh, 0, m}; return true;
    case PA_STATE_N: v = {d.gn, m ? 4u : 8u, d.n_hh, 0, m}; return true;
    case PA_STATE_G: v = {d.g, m ? 4u : 8u, d.n_syn, 1, m}; return true;
    case PA_STATE_CA: v = {d.c, m ? 4u : 8u, d.n_syn, 1, m}; return true;
    case PA_STATE_H: v = {d.h, 8, d.n_syn, 1, false}; return true;
    case PA_STATE_Z: v = {d.z, 8, d.n_syn, 1, false}; return true;
    case PA_STATE_P: v = {d.p, 8, d.n_cells, 0, false}; return true;
    case PA_STATE_EVCOUNT: v = {d.ev_cnt, 16, d.n_syn, 1, false}; return true;
    case PA_STATE_EVSTEPSUM: v = {d.ev_sum, 16, d.n_syn, 1, false}; return true;
    case PA_STATE_SPS: v = {d.sps, 8, d.n_cv, 0, false}; return d.dif != 0;
    case PA_STATE_PRP: v = {d.prp, 8, d.n_cv, 0, false}; return d.dif != 0;
    default: return false;
    }
}

}  // namespace

extern "C" pa_status pa_state_read(pa_sim *s, int32_t what, void *out, uint64_t n) {
    if (!s || !out) return PA_EINVAL;
    if (s->state == 0) return fail(s, PA_ESTATE, "pa_finalize first");
    View v;
    if (!view_of(s, what, v)) return fail(s, PA_EINVAL, "unknown state array %d", what);
    const uint64_t count = (what == PA_STATE_EVCOUNT || what == PA_STATE_EVSTEPSUM) ? 2 * v.n : v.n;
    if (n != count) return fail(s, PA_EINVAL, "state array %d has %llu elements", what, (unsigned long long)count);
    std::vector<uint8_t> buf(v.n * v.esize);
    HIPCHECK(s, hipStreamSynchronize(s->stream), "sync");
    if (!buf.empty()) HIPCHECK(s, hipMemcpyAsync(buf.data(), v.p, buf.size(), hipMemcpyDeviceToHost, s->stream), "state read");
    HIPCHECK(s, hipStreamSynchronize(s->stream), "sync");
    for (uint64_t q = 0; q < v.n; ++q) {
        const uint64_t dst = v.perm == 1 ? s->syn_perm[q] : q;
        if (v.narrow) {
            float f;
            std::memcpy(&f, buf.data() + q * 4, 4);
            ((double *)out)[dst] = (double)f;
        } else {
            std::memcpy((uint8_t *)out + dst * v.esize, buf.data() + q * v.esize, v.esize);
        }
    }
    return PA_OK;
}

extern "C" pa_status pa_state_read_device(pa_sim *s, int32_t what, void *out, uint64_t n) {
    if (!s || !out) return PA_EINVAL;
    if (s->state == 0) return fail(s, PA_ESTATE, "pa_finalize first");
    View v;
    if (!view_of(s, what, v)) return fail(s, PA_EINVAL, "unknown state array %d", what);
    const uint64_t count = (what == PA_STATE_EVCOUNT || what == PA_STATE_EVSTEPSUM) ? 2 * v.n : v.n;
    if (n != count) return fail(s, PA_EINVAL, "state array %d has %llu elements", what, (unsigned long long)count);
    const uint32_t words = v.narrow ? 1u : (uint32_t)(v.esize / 8);
    if (launch_state_out(v.p, words, v.narrow, v.perm == 1 ? s->d.syn_sid : nullptr, v.n, out, s->stream))
        return hip_fail(s, hipGetLastError(), "state copy");
    HIPCHECK(s, hipStreamSynchronize(s->stream), "state copy");
    return PA_OK;
}

extern "C" pa_status pa_state_write(pa_sim *s, int32_t what, const void *in, uint64_t n) {
    if (!s || !in) return PA_EINVAL;
    if (s->state == 0) return fail(s, PA_ESTATE, "pa_finalize first");
    if (what == PA_STATE_EVCOUNT || what == PA_STATE_EVSTEPSUM)
        return fail(s, PA_EINVAL, "state array %d is read-only", what);
    View v;
    if (!view_of(s, what, v)) return fail(s, PA_EINVAL, "unknown state array %d", what);
    if (n != v.n) return fail(s, PA_EINVAL, "state array %d has %llu elements", what, (unsigned long long)v.n);
    std::vector<uint8_t> buf(v.n * v.esize);
    for (uint64_t q = 0; q < v.n; ++q) {
        const uint64_t src = v.perm == 1 ? s->syn_perm[q] : q;
        const double x = ((const double *)in)[src];
        if (v.narrow) {
            float f = (float)x;
            std::memcpy(buf.data() + q * 4, &f, 4);
        } else {
            std::memcpy(buf.data() + q * 8, &x, 8);
        }
    }
    HIPCHECK(s, hipStreamSynchronize(s->stream), "sync");
    if (!buf.empty()) HIPCHECK(s, hipMemcpyAsync(v.p, buf.data(), buf.size(), hipMemcpyHostToDevice, s->stream), "state write");
    // new conductances: their carried per-CV sums follow
    if (what == PA_STATE_G && launch_carried_sums(s->d, s->stream) != 0)
        return fail(s, PA_EDEVICE, "carried sums");
    HIPCHECK(s, hipStreamSynchronize(s->stream), "sync");
    return PA_OK;
}

extern "C" pa_status pa_stats_get(const pa_sim *s, pa_stats *o) {
    if (!s || !o) return PA_EINVAL;
    *o = pa_stats{};
    o->n_cells = s->cv_off.size() - 1;
    o->n_cv = (uint64_t)s->cv_off.back();
    o->n_syn = s->syn_cell.size();
    o->n_stc = 0;
    for (uint8_t k : s->syn_kind) o->n_stc += k == PA_SYN_STC;
    o->n_conn = s->conn_src.size();
    o->n_trains = s->tr_dst.size();
    o->n_probes = s->pr_what.size();
    o->n_poisson = s->po_dst.size();
    o->steps = s->step;
    o->spikes = s->sp_gid.size();
    o->epoch_steps = s->d.K;
    o->spike_ring = s->d.H;
    o->queue_events = s->queue_events;
    o->cells_per_block = batched_cells_per_block(const_cast<pa_sim *>(s));
    batched_plan_shape(const_cast<pa_sim *>(s), o->block_threads, o->solver_waves, o->exchange);
    o->advance_ms = s->advance_ms;
    o->device_bytes = s->device_bytes;
    if (s->state != 0) {
        Counters c{};
        if (hipStreamSynchronize(s->stream) == hipSuccess &&
            hipMemcpy(&c, s->d.ctr, sizeof c, hipMemcpyDeviceToHost) == hipSuccess)
            o->events = c.events;
    }
    return PA_OK;
}

extern "C" pa_status pa_kernel_timing(pa_sim *s, int32_t enable) {
    if (!s) return PA_EINVAL;
    s->timing = enable != 0;
    s->timed_ms = 0.0;
    s->timed_launches = 0;
    s->tev_used = 0;
    return PA_OK;
}

extern "C" pa_status pa_kernel_time(pa_sim *s, double *total_ms, uint64_t *launches, const char **name) {
    if (!s) return PA_EINVAL;
    if (total_ms) *total_ms = s->timed_ms;
    if (launches) *launches = s->timed_launches;
    if (name) *name = s->cfg.mode == PA_BATCHED ? (s->d.mixed ? "k_epoch<float>" : "k_epoch<double>")
                                                 : (s->d.mixed ? "k_syn<float>" : "k_syn<double>");
    return PA_OK;
}

// Accessors for the batched-form host code.
DevNet &pa_devnet(pa_sim *s) { return s->d; }
hipStream_t pa_stream(pa_sim *s) { return s->stream; }
void *pa_dev_alloc(pa_sim *s, size_t bytes) { return dev_alloc(s, bytes); }
pa_status pa_fail(pa_sim *s, pa_status st, const char *msg) { return fail(s, st, "%s", msg); }
const pa_config &pa_cfg(pa_sim *s) { return s->cfg; }
BatchedPlan *&pa_plan(pa_sim *s) { return s->plan; }

// Saves (restore = 0) or restores (restore = 1) every mutable device array,
// so that autotuning trials leave the simulation at its initial state.
pa_status pa_snapshot(pa_sim *s, int restore) {
    DevNet &d = s->d;
    std::vector<Span> spans = mutable_spans(s);
    spans.push_back({d.blk_done, (size_t)d.n_cells * 8});
    spans.push_back({d.bar_grp, 34 * 32 * 4});
    spans.push_back({d.ctr, sizeof(Counters)});
    size_t total = 0;
    for (const Span &x : spans) total += (x.n + 255) & ~size_t(255);
    if (!s->snap) {
        s->snap = dev_alloc(s, total);
        if (!s->snap) return fail(s, PA_ENOMEM, "snapshot buffer");
    }
    size_t off = 0;
    for (const Span &x : spans) {
        if (x.n) {
            void *b = (uint8_t *)s->snap + off;
            HIPCHECK(s, hipMemcpyAsync(restore ? x.p : b, restore ? b : x.p, x.n, hipMemcpyDeviceToDevice, s->stream), "snapshot");
        }
        off += (x.n + 255) & ~size_t(255);
    }
    HIPCHECK(s, hipStreamSynchronize(s->stream), "snapshot");
    return PA_OK;
}
