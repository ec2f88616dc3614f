/*
 * plasticarbor.h -- C ABI of the MI355X (gfx950) engine that advances
 * plastic networks of multi-compartment neurons step by step, after
 * "Plastic Arbor" (Luboeinski et al., arXiv 2411.16445).
 *
 * One implicit-Euler step (fixed dt) of the whole network:
 *   1. deliver queued spike events to synapses (conductance port and the
 *      delayed calcium port of the calcium-based rule, Eq. 19; two ports
 *      per connection are what the round_robin_halt selection policy of
 *      Sec. 2.2 exists for), then the post-synaptic spike hook (Sec. 2.1);
 *   2. membrane currents at V^n (ohmic current sum, Sec. 2.4: Hodgkin-Huxley
 *      soma, passive leak, conductance-based exponential synapses, clamps);
 *   3. assembly of the cable equation (Eq. 4), linearised backward Euler
 *      (the "implicit solving methods" of the discussion);
 *   4. Hines solve of every cell's tree system;
 *   5. HH gate and synaptic conductance updates at V^{n+1};
 *   6. calcium-based early phase h (Eqs. 17-18, Euler-Maruyama of Sec. 2.3
 *      with Threefry-4x64-12 + Box-Muller noise), late phase z (Eq. 20),
 *      per-cell protein p (Eq. 21) with total weight w = h + h0 z (Eq. 16);
 *   7. threshold detection and delayed event generation.
 *
 * Units everywhere: ms, mV, um, nA, uS (conductance), nF, umol/l.
 *
 * Section numbers refer to the paper: Sec. 2.1 (post-synaptic spike hook),
 * 2.2 (one connection addressing a synapse through two streams), 2.3
 * (stochastic differential equations), 2.4 (cable equation, Eq. 4, and
 * ohmic membrane currents), 3.5 (synaptic tagging and capture, Eqs. 16-21,
 * Table 5), 3.6-3.8 (networks, benchmarks).
 *
 * Conventions
 *   - Every call returns a pa_status; no C++ exception crosses the ABI.
 *     On failure pa_last_error(sim) holds a message.
 *   - Input arrays are read during the call and copied; the caller keeps
 *     ownership.  Output arrays are caller-owned host buffers, except for
 *     pa_state_read_device, which writes a caller-owned device buffer.
 *   - The library owns all device memory; it allocates it at pa_finalize
 *     through the allocator set with pa_set_allocator (default hipMalloc).
 *   - State machine: BUILD --pa_finalize--> READY.  Adding cells, synapses,
 *     connections, trains, clamps or probes after pa_finalize returns
 *     PA_ESTATE; advancing before it returns PA_ESTATE.
 *   - One host thread per simulation; different simulations are
 *     independent.  All device work of a simulation is ordered on its
 *     stream (pa_set_stream), and every call that returns data has
 *     synchronised that stream.
 */
#ifndef PLASTICARBOR_H
#define PLASTICARBOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pa_sim pa_sim;
typedef int32_t pa_status;

#define PA_OK 0
#define PA_EINVAL (-1)     /* invalid argument or network description */
#define PA_ESTATE (-2)     /* call not allowed in the current state */
#define PA_ENOMEM (-3)     /* allocation failed */
#define PA_EDEVICE (-4)    /* HIP runtime error */
#define PA_ERANGE (-5)     /* time off the dt grid, backwards, or an event in the past */
#define PA_EOVERFLOW (-6)  /* Poisson arrivals beyond their epoch queue, or the spike
                              history of one advance overflowed */
#define PA_ENUMERIC (-7)   /* a membrane voltage became non-finite */

/* precision of the run */
#define PA_FP64 0   /* every state and arithmetic in FP64 */
#define PA_MIXED 1  /* HH gates, synaptic conductance and calcium in FP32;
                       cable solve, h, z, p in FP64 */
/* execution form */
#define PA_PLAIN 0    /* one kernel per stage per step */
#define PA_BATCHED 1  /* one fused kernel per epoch of steps */

#define PA_PORT_G 1   /* conductance port: g += w (h + h0 z)/h0, or w */
#define PA_PORT_CA 2  /* calcium port: c += c_pre after t_c,delay */

#define PA_MECH_PAS 0 /* passive leak (g_pas, e_pas) */
#define PA_MECH_HH 1  /* Hodgkin-Huxley Na, K, leak */

#define PA_SYN_EXP 0  /* conductance-based exponential synapse */
#define PA_SYN_STC 1  /* exponential synapse with calcium-based early phase and
                         tagging-and-capture late phase (Sec. 3.5) */
#define PA_SYN_STDP 2 /* exponential synapse with pair-based STDP (Sec. 3.1,
                         Eqs. 6-8): weight w, traces a_pre, a_post */

typedef struct {
    double dt_ms;            /* time step, > 0 */
    double threshold_mV;     /* spike detector threshold */
    uint64_t seed;           /* key of the early-phase noise */
    int32_t precision;       /* PA_FP64 or PA_MIXED */
    int32_t mode;            /* PA_PLAIN or PA_BATCHED */
    uint32_t flags;          /* reserved, 0 */
    uint32_t cells_per_block;/* batched form: cells per workgroup; 0 = autotune */
    uint16_t block_threads;  /* batched form: 64, 128 or 256 lanes per workgroup;
                                0 = autotune */
    uint16_t solver_waves;   /* batched form: wavefronts of a workgroup that run the
                                cable solve (1 .. lanes/64 - 1; the others update
                                synapses); 0 = autotune */
    uint32_t exchange;       /* batched form: PA_EXCHANGE_AUTO, PA_EXCHANGE_KERNEL or
                                PA_EXCHANGE_RESIDENT */
} pa_config;

/* Batched form, spike exchange between epochs.  KERNEL: one launch of the
 * fused step kernel per epoch (state staged in and out of LDS every epoch;
 * spikes reach the other cells at the launch boundary).  RESIDENT: many
 * epochs per cooperative launch with every workgroup resident; the state
 * stays in LDS and the workgroups wait for each other behind a grid
 * barrier between epochs (needs all workgroups to fit on the device at
 * once).  AUTO: the faster of the two in trial epochs where RESIDENT fits. */
#define PA_EXCHANGE_AUTO 0
#define PA_EXCHANGE_KERNEL 1
#define PA_EXCHANGE_RESIDENT 2

/* Table 5 of the paper (h0 = 10 mV * 0.5 gamma_p/(gamma_p + gamma_d),
 * theta_pro = 0.5 h0, theta_tag = 0.2 h0 are given explicitly). */
typedef struct {
    double tau_c, tau_h, tau_p, tau_z;   /* ms */
    double gamma_p, gamma_d;             /* potentiation / depression rates */
    double theta_p, theta_d;             /* calcium thresholds */
    double sigma_pl;                     /* mV */
    double p_max, f_int;                 /* umol/l, l/umol */
    double t_cd;                         /* calcium delay t_c,delay, ms */
    double h0, theta_pro, theta_tag;     /* mV */
    double c_pre, c_post;                /* calcium jumps */
} pa_stc_params;

/* Pair-based STDP (Eqs. 6-8, Table 1): trace time constants (ms), trace
 * amplitudes A_pre > 0, A_post < 0 and weights (uS). */
typedef struct {
    double tau_pre, tau_post;
    double a_pre, a_post;
    double w0;      /* initial weight */
    double w_max;   /* the weight's contribution to the conductance is clipped to [0, w_max] */
} pa_stdp_params;

/* Membrane and channel constants of one cell. */
typedef struct {
    double cm;        /* uF/cm^2 */
    double ra;        /* axial resistivity, ohm cm */
    double v_init;    /* mV */
    double g_pas;     /* S/cm^2, passive CVs */
    double e_pas;     /* mV */
    double gna, gk, gl;  /* S/cm^2, HH CVs */
    double ena, ek, el;  /* mV */
} pa_cell_params;

typedef struct {
    uint64_t n_cells, n_cv, n_syn, n_stc, n_conn, n_trains, n_probes, n_poisson;
    uint64_t steps, spikes, events;
    uint32_t epoch_steps;    /* K: steps between spike exchanges */
    uint32_t spike_ring;     /* spikes each cell keeps for its targets */
    uint64_t queue_events;   /* room of the per-epoch event queues, all cells */
    uint32_t cells_per_block;
    double advance_ms;       /* wall time inside pa_advance* so far */
    uint64_t device_bytes;   /* device memory held */
    uint32_t block_threads;  /* batched form: lanes per workgroup chosen */
    uint32_t solver_waves;   /* batched form: solver wavefronts chosen */
    uint32_t exchange;       /* batched form: PA_EXCHANGE_KERNEL or PA_EXCHANGE_RESIDENT chosen */
} pa_stats;

/* Creates a simulation in the BUILD state: a network advanced by the
 * implicit step of the cable equation (Eq. 4, Sec. 2.4) with fixed dt,
 * plasticity constants of Table 5 (Sec. 3.5).  cfg and stc are copied.
 * Errors: PA_EINVAL (NULL pointer, dt <= 0, unknown precision/mode,
 * flags != 0, non-finite or non-positive time constants). */
pa_status pa_sim_create(const pa_config *cfg, const pa_stc_params *stc, pa_sim **out);

/* Releases everything; NULL-safe. */
void pa_sim_destroy(pa_sim *sim);

/* Orders all device work of the simulation on `hip_stream` (a hipStream_t,
 * e.g. a torch stream's handle).  NULL selects a stream the library
 * creates.  Allowed before pa_finalize only. */
pa_status pa_set_stream(pa_sim *sim, void *hip_stream);

/* Device memory hooks (e.g. a framework's caching allocator).  alloc
 * returns device memory of at least `bytes` bytes aligned to 256 bytes, or
 * NULL; release frees it.  Allowed before pa_finalize only. */
pa_status pa_set_allocator(pa_sim *sim, void *(*alloc)(size_t bytes, void *ctx),
                           void (*release)(void *ptr, void *ctx), void *ctx);

/* Adds n cells (Sec. 2.4: cable equation Eq. 4 on a tree of cylindrical
 * control volumes; Sec. 3.8: Hodgkin-Huxley soma, passive dendrites).
 * Cell k owns CVs cv_off[k] .. cv_off[k+1]-1 of the arrays
 * (cv_off[0] = 0).  parent holds local CV indices: parent[first] = -1 and
 * 0 <= parent[i] < i (the ordering the Hines elimination relies on).
 * Each CV is a cylinder of the given length and diameter (um) carrying
 * PA_MECH_PAS or PA_MECH_HH.  detector_cv is the local CV of the cell's
 * threshold detector.  params has n entries.  Cell ids (gids) are dense,
 * in call order; the first is written to *first_gid.  Errors: PA_EINVAL. */
pa_status pa_cells_add(pa_sim *sim, uint32_t n, const int64_t *cv_off, const int32_t *parent,
                       const double *length_um, const double *diam_um, const uint8_t *mech,
                       const int32_t *detector_cv, const pa_cell_params *params,
                       uint32_t *first_gid);

/* Adds n synapses (conductance-based exponential synapses, Sec. 3.8; with
 * PA_SYN_STC the calcium-based early phase and tagging-and-capture late
 * phase of Eqs. 16-21, Sec. 3.5): synapse k sits on local CV cv[k] of cell gid[k], kind
 * PA_SYN_EXP or PA_SYN_STC, decay time constant tau_ms[k] > 0, reversal
 * erev_mV[k].  Synapse ids are dense in call order.  Errors: PA_EINVAL. */
pa_status pa_synapses_add(pa_sim *sim, uint32_t n, const uint32_t *gid, const uint32_t *cv,
                          const uint8_t *kind, const double *tau_ms, const double *erev_mV,
                          uint32_t *first_sid);

/* Adds n connections (delayed spike delivery; the calcium port is the
 * second stream of one connection into the same synapse, Sec. 2.2, delayed
 * by t_c,delay, Eq. 19): a spike of cell src_gid[k] at t* reaches synapse
 * dst_sid[k] through the ports in ports[k] (PA_PORT_G and/or PA_PORT_CA;
 * the calcium port needs a PA_SYN_STC target) at t* + delay_ms[k] (plus
 * t_cd for the calcium port), with weight weight_uS[k] on the conductance
 * port.  delay_ms >= dt.  Connection ids are dense in call order and break
 * ties between simultaneous events.  Errors: PA_EINVAL. */
pa_status pa_connect(pa_sim *sim, uint64_t n, const uint32_t *src_gid, const uint32_t *dst_sid,
                     const uint8_t *ports, const double *weight_uS, const double *delay_ms);

/* Adds n explicit presynaptic spike trains (external input, e.g. the
 * Poisson stimulation of Sec. 3.1 and 3.5 given as arrival times): train k
 * delivers arrivals at
 * times_ms[time_off[k] .. time_off[k+1]-1] (non-decreasing, >= 0) to
 * synapse dst_sid[k] through ports[k] with weight weight_uS[k]; the
 * calcium port adds t_cd.  Trains act as sources with ids n_cells + k.
 * Errors: PA_EINVAL. */
pa_status pa_trains_add(pa_sim *sim, uint32_t n, const uint32_t *dst_sid, const uint8_t *ports,
                        const double *weight_uS, const int64_t *time_off, const double *times_ms);

/* Adds n Poisson sources (external Poisson input, Sec. 3.1 and 3.5, drawn
 * on the device from the counter-based generator of Sec. 2.3): source k
 * delivers arrivals of a homogeneous
 * Poisson process of rate_hz[k] to synapse dst_sid[k] through ports[k] with
 * weight weight_uS[k] (the calcium port adds t_cd).  Arrival j of source k
 * follows the previous one (or t = 0) after -ln(u) / rate, u the first
 * output word of Threefry-4x64-12 with counter (j, 0, 0, 0) and key (seed,
 * k, tag, 0) mapped to (0, 1); k counts Poisson sources in call order.
 * Sources act as event sources with ids n_cells + n_trains + k.  rate 0
 * gives no arrivals.  Errors: PA_EINVAL. */
pa_status pa_poisson_add(pa_sim *sim, uint32_t n, const uint32_t *dst_sid, const uint8_t *ports,
                         const double *weight_uS, const double *rate_hz);

/* Adds n current clamps (the injected current of the cable equation,
 * Eq. 4) injecting amp_nA[k] into local CV cv[k] of cell gid[k] during
 * t0 <= t_n < t0 + dur.  Errors: PA_EINVAL. */
pa_status pa_clamps_add(pa_sim *sim, uint32_t n, const uint32_t *gid, const uint32_t *cv,
                        const double *t0_ms, const double *dur_ms, const double *amp_nA);

#define PA_PROBE_V 0   /* index: global CV (cv_off of the cell + local CV) */
#define PA_PROBE_G 1   /* index: synapse id */
#define PA_PROBE_CA 2  /* index: synapse id (PA_SYN_STC; a_pre of PA_SYN_STDP) */
#define PA_PROBE_H 3   /* index: synapse id (PA_SYN_STC; w of PA_SYN_STDP) */
#define PA_PROBE_Z 4   /* index: synapse id (PA_SYN_STC; a_post of PA_SYN_STDP) */
#define PA_PROBE_P 5   /* index: cell id */
#define PA_PROBE_SPS 6 /* index: global CV (needs pa_set_diffusion) */
#define PA_PROBE_PRP 7 /* index: global CV (needs pa_set_diffusion) */

/* Switches the protein model from the per-cell sum of Eq. 21 to particle
 * diffusion over each cell's CVs (Eq. 5, Sec. 2.4; the multi-compartment
 * formulation of Sec. 3.6 with the threshold of Eq. 23).  Two species
 * diffuse by backward Euler on the finite-volume tree of the cell (sealed
 * ends; between a CV and its parent a flux D (X_j - X_i) over the two
 * half-cylinders' length / cross-section in series; CV volume pi r^2 l):
 *   SPS, released at each plastic synapse's CV by the step's change of
 *     |h - h0| (so that a cell's SPS amount is the sum of Eq. 21);
 *   PRP, decaying at rate 1 / tau_p everywhere and synthesised in the
 *     detector CV (the soma) at p_max V_tot / tau_p (amount per time) while
 *     the SPS concentration there exceeds theta_pro / V_tot (Eq. 23), so
 *     that a well-mixed cell follows Eq. 21.
 * z (Eq. 20) then takes the step-start PRP concentration of its synapse's
 * CV; the per-cell p is no longer updated.  Diffusivities in um^2/ms
 * (1e-11 m^2/s = 1e-2 um^2/ms), >= 0.  Both start at zero concentration.
 * Allowed before pa_finalize only.  Errors: PA_EINVAL, PA_ESTATE. */
pa_status pa_set_diffusion(pa_sim *sim, double d_sps_um2_per_ms, double d_prp_um2_per_ms);

/* Parameters of the PA_SYN_STDP synapses (Eqs. 6-8): a conductance-port
 * event of connection weight w_conn adds w_conn clip(w, 0, w_max) to g
 * (the weight before this spike's change), then a_pre += A_pre and
 * w += a_post; a post-synaptic spike (the hook of Sec. 2.1, at the start of
 * the step after its detection, after that step's events) adds A_post to
 * a_post and a_pre to w; both traces decay by exp(-dt/tau) every step.  The
 * state arrays and probes report w as H, a_pre as CA and a_post as Z.
 * Fast-forward leaves STDP synapses as they are (apart from their
 * conductance).  Required before pa_finalize when PA_SYN_STDP synapses
 * exist.  Errors: PA_EINVAL (time constants not positive), PA_ESTATE. */
pa_status pa_set_stdp(pa_sim *sim, const pa_stdp_params *params);

/* Adds n probes (the recorded traces of the paper's figures): probe k
 * samples quantity what[k] of element index[k] after every
 * stride_steps[k]-th completed step (stride >= 1).  Probe ids are dense in
 * call order; the first is written to *first_probe.  Errors: PA_EINVAL. */
pa_status pa_probes_add(pa_sim *sim, uint32_t n, const int32_t *what, const uint64_t *index,
                        const uint32_t *stride_steps, uint32_t *first_probe);

/* Validates, orders synapses by (cell, CV, id), builds the cable
 * invariants (Eq. 4), the table of incoming connections by target cell,
 * the spike rings and the per-epoch event queues, allocates and uploads
 * device memory, initialises the state (V = v_init, gates at steady state,
 * g = c = z = p = 0, h = h0) and, in the batched form, picks and captures
 * the launch plan.  Errors: PA_EINVAL, PA_ESTATE, PA_ENOMEM, PA_EDEVICE. */
pa_status pa_finalize(pa_sim *sim);

/* Advances to t_until_ms, which must lie on the dt grid (within 1e-9
 * relative) and not before the present time: per step, event delivery and
 * the post-synaptic hook (Sec. 2.1, Eq. 16, Eq. 19), membrane currents
 * (Sec. 2.4), the implicit cable step (Eq. 4), HH gates and synaptic decay
 * (Sec. 3.8), plasticity (Eqs. 17-21 with the noise of Sec. 2.3) and
 * threshold detection (Sec. 2.1).  Errors: PA_ESTATE, PA_ERANGE,
 * PA_EOVERFLOW, PA_ENUMERIC, PA_EDEVICE; after any of the last three the
 * simulation refuses further advances. */
pa_status pa_advance(pa_sim *sim, double t_until_ms);

/* Advances by n_steps steps.  Errors as pa_advance. */
pa_status pa_advance_steps(pa_sim *sim, uint64_t n_steps);

/* Number of spikes recorded so far. */
pa_status pa_spikes_count(const pa_sim *sim, uint64_t *n);

/* Copies up to cap spikes (gid, step of the crossing, interpolated time;
 * the threshold detector of Sec. 2.1) in (time, gid) order; *n receives
 * the number copied.  Any of the three arrays may be NULL. */
pa_status pa_spikes_read(const pa_sim *sim, uint32_t *gid, uint64_t *step, double *t_ms,
                         uint64_t cap, uint64_t *n);

/* Number of samples probe_id has recorded so far.  Errors: PA_EINVAL. */
pa_status pa_probe_count(const pa_sim *sim, uint32_t probe_id, uint64_t *n_samples);

/* Copies up to cap samples of probe probe_id, oldest first.  Errors:
 * PA_EINVAL. */
pa_status pa_probe_read(const pa_sim *sim, uint32_t probe_id, double *out, uint64_t cap, uint64_t *n);

#define PA_STATE_V 0        /* n_cv doubles, CV order of pa_cells_add */
#define PA_STATE_M 1        /* one double per HH CV, in CV order */
#define PA_STATE_HHH 2
#define PA_STATE_N 3
#define PA_STATE_G 4        /* n_syn doubles, synapse id order */
#define PA_STATE_CA 5
#define PA_STATE_H 6
#define PA_STATE_Z 7
#define PA_STATE_P 8        /* n_cells doubles */
#define PA_STATE_EVCOUNT 9  /* 2 uint64 per synapse: delivered events per port */
#define PA_STATE_EVSTEPSUM 10 /* 2 uint64 per synapse: sum of delivery steps */
#define PA_STATE_SPS 11     /* n_cv doubles: SPS concentration (needs pa_set_diffusion) */
#define PA_STATE_PRP 12     /* n_cv doubles: PRP concentration (needs pa_set_diffusion) */

/* Copies a state array to a host buffer of n elements (count must match).
 * FP32 state of the mixed form is widened.  READY state only. */
pa_status pa_state_read(pa_sim *sim, int32_t what, void *out, uint64_t n);

/* The same into a caller-owned device buffer `dev_out` (e.g. a framework
 * tensor's storage) of n elements: doubles for codes 0-8 (FP32 state of
 * the mixed form widened), uint64 pairs for 9-10, in the same order as
 * pa_state_read.  Enqueued on the simulation's stream; the call returns
 * after the copy has completed.  Errors: PA_EINVAL, PA_ESTATE, PA_ENOMEM
 * (element counts above 2^32), PA_EDEVICE. */
pa_status pa_state_read_device(pa_sim *sim, int32_t what, void *dev_out, uint64_t n);

/* Overwrites a state array (codes 0-8) from a host buffer; for setting up
 * test states.  READY state only. */
pa_status pa_state_write(pa_sim *sim, int32_t what, const void *in, uint64_t n);

/* Fast-forward (the long steps of slow network dynamics of the 8-h
 * paradigm, Sec. 3.5): n_long steps of length dt_long_ms (a whole multiple
 * of dt) that advance only h, z and p, with spiking and calcium off: per
 * long step, from step-start values, h += (dt_long/tau_h) 0.1 (h0 - h)
 * (Eq. 17 without calcium), z by Eq. 20 and p by Eq. 21 with S = sum
 * |h - h0|; synaptic conductances and calcium decay exactly over each long
 * step; membrane voltages and gates stay as they are.  Everything in
 * flight is dropped: spikes before the new time cause no events, the
 * post-synaptic flags clear, explicit train arrivals before the new time
 * are skipped, and a Poisson source whose next arrival falls before it
 * draws that arrival again (index + 1) as the new time plus an interval.
 * Time moves to t + n_long dt_long.  Needs the per-cell protein model.
 * Errors: PA_EINVAL (dt_long not a whole positive multiple of dt, particle
 * diffusion on), PA_ESTATE, PA_ERANGE, PA_ENOMEM, PA_EDEVICE. */
pa_status pa_fast_forward(pa_sim *sim, uint64_t n_long, double dt_long_ms);

/* Device state dump (the state saving of Sec. 3.5, without a host round
 * trip): every mutable array of the simulation (voltages, gates,
 * conductances, calcium, h, z, p, species, post flags, spike rings,
 * delivery statistics, train cursors, Poisson streams) and the step, in
 * one buffer of pa_state_size bytes.  buf may be a device pointer (e.g. a
 * framework tensor's storage) or host memory.  pa_state_load restores a
 * dump into a simulation of the same network, precision and protein model
 * (checked against the dump's header) and sets its time to the dump's;
 * spikes and probe samples already read out are not part of the state.
 * Errors: PA_EINVAL (buffer too small, dump of another shape), PA_ESTATE,
 * PA_EDEVICE. */
pa_status pa_state_size(pa_sim *sim, uint64_t *bytes);
pa_status pa_state_save(pa_sim *sim, void *buf, uint64_t bytes);
pa_status pa_state_load(pa_sim *sim, const void *buf, uint64_t bytes);

/* Sizes and counters. */
pa_status pa_stats_get(const pa_sim *sim, pa_stats *out);

/* Batched form: choose the plan again (workgroup shape, cells per
 * workgroup, solver wavefronts, spike exchange; within the limits the
 * configuration fixes) by timing trial epochs from the present state, which
 * is restored after each trial, as pa_finalize does from the initial
 * state.  The work of a step depends on the network's regime (a network at
 * rest draws no weight noise; one whose synapses carry calcium above a
 * threshold draws it on most of them every step), so a plan chosen at rest
 * can be slow later.  No step is advanced and no spike is recorded.  The
 * replaced plan's block table (a few bytes per workgroup) stays allocated
 * until pa_sim_destroy.  Results may change in the last bits of the mixed
 * form's FP32 arithmetic with the plan; the FP64 batched form gives the
 * same bits under every plan.
 * Errors: PA_EINVAL (plain form), PA_ESTATE (not finalized, or failed),
 * PA_ENOMEM, PA_EDEVICE; after an error the simulation is failed. */
pa_status pa_retune(pa_sim *sim);

/* Per-launch timing of the dominant kernel (the per-step synapse and
 * plasticity kernel in the plain form, the fused epoch kernel in the
 * batched form) with HIP events on the simulation's stream.  When enabled,
 * pa_kernel_time reports the summed duration and the launch count since
 * the last enable. */
pa_status pa_kernel_timing(pa_sim *sim, int32_t enable);
pa_status pa_kernel_time(pa_sim *sim, double *total_ms, uint64_t *launches, const char **name);

/* Batched Hines solve (Hines 1989) of caller-given tree systems on the
 * device, outside any simulation: the linear system of one implicit step
 * of the cable equation (Eq. 4, Sec. 2.4) for n_cells cells at once.  All
 * array arguments are device pointers owned by the caller:
 *   cv_off  int64[n_cells+1]: cell k owns rows cv_off[k] .. cv_off[k+1]-1,
 *           0 <= cv_off[k] <= cv_off[k+1] <= n_cv;
 *   parent  int32[n_cv]: cell-local parent row, -1 for a cell's first row,
 *           else 0 <= parent[i] < i;
 *   diag    double[n_cv]: diagonal entries;
 *   off     double[n_cv]: off[i] is the symmetric entry coupling row i to
 *           its parent (ignored for a cell's first row);
 *   rhs     double[n_cv]: right-hand side;
 *   x       double[n_cv]: the solution (written).
 * diag, off and rhs are not modified.  The elimination runs from a cell's
 * last row towards its root, then substitution from the root, in the
 * sequential algorithm's order (IEEE FP64, no fused multiply-add).  A cell
 * whose range or parents break the rules above gets NaN in its rows of x;
 * where a decreasing cv_off makes two cells' ranges overlap, the shared
 * rows are written by both and their contents are unspecified.
 * Work is enqueued on hip_stream (NULL: the null stream); the call returns
 * after it has completed.  The elimination workspace (16 bytes per row) is
 * allocated with hipMalloc for the call.  Errors: PA_EINVAL (NULL array
 * with n_cells > 0), PA_ENOMEM, PA_EDEVICE. */
pa_status pa_tree_solve(uint32_t n_cells, uint64_t n_cv, const int64_t *cv_off, const int32_t *parent,
                        const double *diag, const double *off, const double *rhs, double *x,
                        void *hip_stream);

/* The same solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops): it allocates nothing, takes its
 * workspace from a fixed per-device array of the library (16 MiB, so
 * n_cv <= 1048576), does not synchronise and returns once the work is
 * enqueued.  Calls that overlap on one device share that workspace and
 * race: order them on one stream.  Errors: PA_EINVAL, PA_ERANGE
 * (n_cv > 1048576), PA_EDEVICE. */
pa_status pa_tree_solve_noalloc(uint32_t n_cells, uint64_t n_cv, const int64_t *cv_off,
                                const int32_t *parent, const double *diag, const double *off,
                                const double *rhs, double *x, void *hip_stream);

/* Parameters of the calcium-based rule of Graupner and Brunel (Sec. 3.3,
 * Eqs. 10-12, Table 3): time constants and the calcium delay in ms, the
 * weight without unit. */
typedef struct {
    double tau_w, w_star, gamma_p, gamma_d, theta_p, theta_d, sigma;
    double tau_c, c_pre, c_post, t_cd;
} pa_gb_params;

/* Batched single-synapse trials of that rule under the pairing protocol of
 * its DP curve (Sec. 3.3, Fig. 2f/j): n_pairs presynaptic spikes, one every
 * period_ms from t0_ms, each adding c_pre to the calcium t_cd later
 * (delivered at the step floor(t / dt)); postsynaptic spikes imposed
 * delay_ms[i] after each presynaptic one, adding c_post.  Per step, after
 * that step's jumps (presynaptic first), the Euler-Maruyama step of Eq. 10
 * from the step-start calcium,
 *   w += (dt/tau_w)(-w(1-w)(w_* - w) + gamma_p (1-w) Th_p - gamma_d w Th_d)
 *        + sigma sqrt((Th_p + Th_d) dt / tau_w) N,
 * Th_x = [c > theta_x], N the standard normal of trial i at step n (the
 * counter-based generator of the early-phase noise keyed by (seed, i)), then
 * c *= exp(-dt / tau_c) (Eq. 12).  The run covers floor((t0 + n_pairs
 * period) / dt) steps.  delay_ms, w0 (inputs) and w_final, c_final (the
 * weight and calcium at the end; c_final may be NULL) are device arrays of
 * n_trials doubles owned by the caller.  Work runs on hip_stream (NULL: the
 * null stream); the call returns after it has completed.  Errors:
 * PA_EINVAL, PA_ERANGE, PA_EDEVICE. */
pa_status pa_gb_trials(const pa_gb_params *params, double dt_ms, uint64_t n_trials, const double *delay_ms,
                       const double *w0, uint32_t n_pairs, double period_ms, double t0_ms, uint64_t seed,
                       double *w_final, double *c_final, void *hip_stream);

const char *pa_last_error(const pa_sim *sim);
const char *pa_status_str(pa_status status);

#ifdef __cplusplus
}
#endif
#endif /* PLASTICARBOR_H */
