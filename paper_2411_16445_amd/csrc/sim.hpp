// Internal layout of a finalized simulation on the device.
//
// Structure-of-arrays, indices in uint32 (a single MI355X holds < 2^32 CVs,
// synapses and connections of any network that fits its 288 GB).  Synapses
// are stored sorted by (cell, CV, id) so that each CV's synapses and each
// cell's synapses are contiguous; connections are stored as a table by
// target cell.  Every cell keeps its last H spikes in a ring; at the start
// of an epoch each target cell gathers from its incoming connections the
// events due in the epoch into a queue of its own, counted and sorted per
// delivery step (no event is stored between epochs).
#pragma once

#include <cstddef>
#include <cstdint>

namespace pa {

struct Event {
    double t;       // delivery time t_e (ms): sort key 1
    double w;       // weight of the conductance port (uS)
    uint32_t syn;   // sorted synapse index
    uint32_t src;   // source id: cell gid, or n_cells + train index: sort key 2
    uint32_t conn;  // connection id (0 for trains): sort key 3
    uint32_t port;  // 1 conductance, 2 calcium: sort key 4
};
static_assert(sizeof(Event) == 32, "event record is 32 bytes");

// Error flags raised on the device, read back after every advance.
//   QUEUE: a cell's events of one epoch exceeded its queue (possible only
//     through device Poisson sources far above their rate's bound);
//   LATE: an event due before the step of the spike that caused it;
//   NONFINITE: a membrane voltage became non-finite;
//   BARRIER: the grid barrier of the resident form gave up;
//   HISTORY: the spike history of one advance overflowed.
enum : uint32_t {
    FLAG_QUEUE = 1u, FLAG_LATE = 2u, FLAG_NONFINITE = 4u, FLAG_BARRIER = 8u, FLAG_HISTORY = 16u
};

struct Counters {
    uint64_t step;      // first step of the current epoch (advanced by the epoch close)
    uint32_t blocks_done;  // workgroups of a single-epoch launch that finished
    uint32_t flags;     // FLAG_*
    uint64_t hist_n;    // spikes in the history buffer
    uint64_t events;    // events delivered
    uint32_t bad_cell;  // first cell that raised a flag
    uint32_t pad;
};

// One entry of a cell's spike ring: the crossing time, and its step and
// index in the cell's spike sequence (the index tells a reader whether the
// entry already holds the spike it looks for).
struct SpikeRec {
    double t;
    uint32_t step;
    uint32_t idx;
};
static_assert(sizeof(SpikeRec) == 16, "spike record is 16 bytes");

struct Stc {
    double tau_c, tau_h, tau_p, tau_z, gamma_p, gamma_d, theta_p, theta_d;
    double sigma_pl, p_max, f_int, t_cd, h0, theta_pro, theta_tag, c_pre, c_post;
};

// Pair-based STDP (synapse kind 2): trace jumps, weight clip and the
// traces' decay factors per step.
struct StdpK {
    double a_pre, a_post, w_max, r_pre, r_post;
    float r_pre_f;
};

// Everything a kernel needs, passed by value.
struct DevNet {
    uint32_t n_cells, n_cv, n_syn, n_hh, n_trains, n_probes;
    uint32_t K;          // steps per epoch
    uint32_t H;          // spike ring entries per cell
    uint32_t mixed;      // gates, g and c stored in FP32
    double dt, theta;
    uint64_t seed;
    Stc stc;
    StdpK stdp;
    double r_c;          // exp(-dt / tau_c)
    float r_c_f;

    // cells
    const uint32_t *cv_off;      // n_cells + 1
    const uint32_t *det_cv;      // global detector CV
    const uint32_t *syn_off;     // n_cells + 1, into sorted synapses
    const uint32_t *hh_off;      // n_cells + 1, into the HH list
    double *p, *S, *vdet_old;
    uint8_t *post;

    // CVs
    const int32_t *parent;       // global parent, -1 at roots
    const uint16_t *run;         // consecutive nodes ending here whose parent is their predecessor
    // branch segments: maximal runs [a, b] in which every node after a has
    // its predecessor as parent and only child; per cell contiguous
    uint32_t n_seg;
    const uint32_t *seg_off;     // n_cells + 1
    const uint32_t *seg_a, *seg_b;  // global CV of head and bottom node
    const uint8_t *seg_lvl;      // depth in the segment tree (root segment 0)
    const uint32_t *kid_off;     // n_seg + 1, into kids
    const uint32_t *kids;        // child segments of each segment's bottom node, descending head
    const double *cdt, *d0, *gpas_e, *axial;
    const int32_t *hh_of;        // HH slot or -1
    const uint32_t *cv_syn_off;  // n_cv + 1
    const double *cv_dec;        // per CV: the decay factor its synapses share (1 if none)
    uint32_t cv_dec_uniform;     // every CV's synapses share one decay factor
    // batched mixed form with a shared decay factor per CV: summed synaptic
    // conductance and conductance x reversal potential of each CV, decayed
    // to the next step and still without its events (state, n_cv each)
    double *gsum, *gesum;
    const uint32_t *cv_cl_off;   // n_cv + 1, into clamps sorted by (CV, id)
    double *V, *I, *G, *D, *b;

    // HH
    const uint32_t *hh_cv;
    const double *hh_scale;      // 1e-2 * area
    const double *hh_par;        // 6 per HH CV: gna gk gl ena ek el
    void *gm, *gh, *gn;          // double or float

    // synapses, sorted
    const uint32_t *syn_cell, *syn_cv;
    const uint8_t *syn_kind;
    const double *syn_erev, *syn_decay;
    const float *syn_decay_f;
    const uint32_t *syn_sid;
    void *g, *c;                 // double or float
    double *h, *z;
    unsigned long long *ev_cnt, *ev_sum;  // 2 per synapse

    // incoming connections by target cell (in connection id order)
    const uint64_t *in_off;      // n_cells + 1
    const uint32_t *in_src, *in_syn, *in_cid;
    const uint32_t *in_lag;      // steps back from an epoch's first step to the oldest spike that can matter
    const uint8_t *in_ports;
    const double *in_w, *in_d;

    // spike rings: the last H spikes of each cell, entry k of cell c at
    // c * H + k mod H; spk_n counts the cell's spikes, spk_last holds the
    // step of its last spike plus one (0 before the first)
    SpikeRec *spk;
    uint32_t *spk_n, *spk_last;

    // trains
    const uint32_t *tr_syn, *tr_cell;
    const uint8_t *tr_ports;
    const double *tr_w, *tr_t;
    const uint64_t *tr_off;
    uint64_t *tr_cur;            // 2 per train: conductance and calcium cursors
    const uint32_t *tr_cell_off, *tr_by_cell;   // trains grouped by target cell
    const uint32_t *po_cell_off, *po_by_cell;   // Poisson sources grouped by target cell

    // Poisson sources
    uint32_t n_pois;
    const uint32_t *pois_syn, *pois_cell;
    const uint8_t *pois_ports;
    const double *pois_w, *pois_rate;
    const uint32_t *pois_cap;    // most arrivals per port a source may bring into one epoch
    double *pois_t;              // 2 per source (conductance, calcium stream): next arrival time
    uint64_t *pois_j;            // and its index

    // clamps, sorted by (CV, id)
    const double *cl_t0, *cl_dur, *cl_amp;

    // per-epoch event queues: cell c's events of the epoch in
    // q_ev[q_off[c] .. q_off[c + 1]) (room for the most its incoming
    // connections and sources can bring in one epoch); per (cell, step of
    // the epoch) slot its count and offset into the cell's queue
    const uint64_t *q_off;       // n_cells + 1
    Event *q_ev;
    uint32_t *ev_n, *ev_off;     // n_cells * K each (plain form)
    uint64_t *blk_done;          // n_cells: per workgroup, grid barriers passed (multi-epoch kernel)
    uint32_t *bar_grp;           // grid barrier: 32 group counters, top counter, release word (128 bytes apart)

    // spike history of the present advance
    uint32_t *hist_gid;          // capacity hist_cap
    uint64_t *hist_step;
    double *hist_t;
    uint64_t hist_cap;
    Counters *ctr;

    // particle diffusion (Eq. 5) of the signal triggering protein synthesis
    // (SPS) and of the protein (PRP) over each cell's CVs, in place of the
    // per-cell trigger sum and p (dif = 0: off).  Both species' tree
    // systems are constant, so their elimination is done once on the host:
    // per CV the coupling to the parent (u), the elimination factor
    // u / D' and the eliminated diagonal D'; a step only sweeps the
    // right-hand side.
    uint32_t dif;
    const double *dvol;                       // CV volume, um^3
    const double *sps_u, *sps_f, *sps_dp;
    const double *prp_u, *prp_f, *prp_dp;
    const double *dif_thr, *dif_pv;           // per cell: theta_pro / V_tot, p_max V_tot
    double *sps, *prp;                        // per CV concentrations (state)
    double *dlt;                              // per synapse: change of |h - h0| in the step (plain form)

    // probes: probe k samples after every pr_stride[k]-th step into its
    // own region of pr_buf starting at pr_off[k]
    const int32_t *pr_what;
    const uint64_t *pr_idx;      // internal index (sorted synapse, CV, cell)
    const uint32_t *pr_stride;
    const uint64_t *pr_off;
    double *pr_buf;
};

// Launchers (kernels.hip).  All enqueue on `stream` and return a HIP error
// code (0 on success).
int launch_init(const DevNet &d, void *stream);
// Plain form: the events of the epoch [n0, n0 + nsteps) into the per-cell
// queues, then one step.
int launch_gather(const DevNet &d, uint64_t n0, uint32_t nsteps, void *stream);
int launch_step_plain(const DevNet &d, uint64_t n, uint64_t n0, void *stream, void *ev_begin, void *ev_end);
// Samples the probes due after step n (those whose stride divides n);
// `first` is the first step of the present drain interval.
int launch_probe(const DevNet &d, uint64_t n, uint64_t first, void *stream);
// Fused epochs: workgroup b owns cells blk[b] .. blk[b+1]-1; the first
// solver_waves wavefronts of a multi-wavefront workgroup share its cable
// solves.  resident = 0: one epoch of nsteps <= K steps, its first step
// read from Counters::step (so that a captured graph of epochs can be
// replayed) and advanced by the last workgroup; resident = 1: nsteps steps
// in epochs of K (the last one shorter) in one cooperative launch, the
// workgroups waiting for each other between epochs.
int launch_epoch_fused(const DevNet &d, uint32_t nsteps, uint32_t resident, const uint32_t *blk, uint32_t n_blocks,
                       size_t lds_bytes, uint32_t block_threads, uint32_t solver_waves, void *stream);
// Workgroups of the fused kernel that can be resident at once (0 if the
// device does not support cooperative launches).
uint32_t epoch_fused_capacity(bool mixed, uint32_t block_threads, size_t lds_bytes);
// Recomputes gsum and gesum from the synapse conductances (after they were
// written from the host).
int launch_carried_sums(const DevNet &d, void *stream);
int launch_fill_u32(uint32_t *p, uint32_t v, size_t n, void *stream);
// Fast-forward: n_long long steps of the slow plasticity variables (gdec:
// per sorted synapse the conductance decay over a long step, rc the
// calcium's), clearing post flags and spike rings; Poisson sources restart
// from step n_new.
int launch_fast_forward(const DevNet &d, uint64_t n_long, double dt_long, const double *gdec, double rc,
                        uint64_t n_new, void *stream);
// Copies n elements of a state array (words 64-bit words each, or FP32
// widened to FP64) to dst, element q to position perm[q] (perm may be null).
int launch_state_out(const void *src, uint32_t words, bool narrow, const uint32_t *perm, uint64_t n, void *dst,
                     void *stream);

}  // namespace pa
