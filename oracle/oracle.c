/*
 * Plain FP64 CPU oracle for one implicit-Euler step of a plastic network of
 * multi-compartment neurons (Plastic Arbor, arXiv 2411.16445).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP library is checked against.  It is called only by
 * the test-suite, by the smoke check and by the CPU-baseline leg of the
 * benchmark; the product path never links, loads or executes it, and it
 * shares no source, header or helper with the HIP library.
 *
 * What one step n -> n+1 (t_n = n dt) computes, in this order:
 *  1. deliver every queued event whose delivery step is n, ordered by
 *     (t_e, source, connection, port): conductance port g += w (h + h0 z)/h0
 *     for tagging-and-capture synapses (total weight, Eq. 16, normalised to
 *     its baseline) or g += w for plain exponential synapses; calcium port
 *     c += c_pre (Eq. 19).  Then the post-synaptic hook: every synapse of a
 *     cell that fired in step n-1 gets c += c_post (Sec. 2.1, Eq. 19).
 *  2. membrane current I and conductance G = dI/dV at V^n per CV, summed in
 *     a fixed order: Hodgkin-Huxley, synapses by (CV, id), clamps (the
 *     ohmic current sum of Sec. 2.4).
 *  3. assembly of the cable system, linearised backward Euler on the
 *     finite-volume discretisation of the cable equation (Eq. 4),
 *  4. Hines elimination over the tree (descending index, then forward
 *     substitution),
 *  5. HH gates by exact exponential integration at V^{n+1}; exponential
 *     decay of every synaptic conductance,
 *  6. plasticity (Eqs. 17, 18, 20, 21): per cell S = sum |h - h0| over its
 *     tagging synapses from step-start h; Euler-Maruyama step of h (Sec. 2.3)
 *     with Threefry-4x64-12 + Box-Muller noise; z; calcium decay; then p,
 *     With particle diffusion switched on (prp_model 1, Sec. 2.4 Eq. 5 and
 *     Sec. 3.6 Eq. 23) the per-cell sum and p are replaced by two species
 *     diffusing over the cell's CVs: a signal triggering protein synthesis
 *     (SPS), released at each synapse's CV by the change of |h - h0|, and
 *     the protein (PRP), synthesised at the soma while the SPS
 *     concentration there exceeds theta_pro / V_tot and decaying everywhere;
 *     z then takes the PRP concentration of its synapse's CV.
 *     Pair-based STDP synapses (kind 2, Eqs. 6-8): a conductance-port event
 *     adds w_conn x clip(w, 0, w_max) to g, then a_pre += A_pre and
 *     w += a_post; the post-synaptic hook adds A_post to a_post and a_pre
 *     to w; both traces decay exactly in step 6.
 *  7. threshold detection V^n < theta <= V^{n+1}, linear interpolation of
 *     the crossing time, and one queued event per outgoing connection and
 *     port (delay d, calcium port a further t_c,delay later), delivered at
 *     step floor(t_e / dt).
 *  External drive: explicit arrival trains, and Poisson sources whose
 *  inter-arrival times come from a counter-based generator.
 *
 * The event queue is a single binary min-heap; there are no epochs.
 * Built with -fopenmp (the timing variant only), the loops over CVs, cells
 * and synapses whose iterations are independent run on several threads;
 * every value is computed by the same expressions in the same order, so
 * both builds give the same bits.
 * Functions whose result no test pins against an independent fact are
 * marked "parity unpinned" below.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------ input layout */
typedef struct {
    double dt, theta;
    uint64_t seed;
    /* STC parameters, Table 5 */
    double tau_c, tau_h, tau_p, tau_z, gamma_p, gamma_d, theta_p, theta_d;
    double sigma_pl, p_max, f_int, t_cd, h0, theta_pro, theta_tag, c_pre, c_post;

    int64_t n_cells;
    const int64_t *cv_off;      /* n_cells + 1 */
    const int32_t *parent;      /* local index, -1 for the root */
    const double *length, *diam;
    const uint8_t *mech;        /* 0 passive, 1 HH */
    const int32_t *detector;    /* local CV */
    const double *cell_params;  /* n_cells x 11 */

    int64_t n_syn;
    const int32_t *syn_cell, *syn_cv;
    const uint8_t *syn_kind;
    const double *syn_tau, *syn_erev;

    int64_t n_conn;
    const int32_t *conn_src, *conn_dst;
    const uint8_t *conn_ports;
    const double *conn_w, *conn_d;

    int64_t n_trains;
    const int32_t *train_dst;
    const uint8_t *train_ports;
    const double *train_w;
    const int64_t *train_off;
    const double *train_times;

    int64_t n_clamps;
    const int32_t *clamp_cell, *clamp_cv;
    const double *clamp_t0, *clamp_dur, *clamp_amp;

    int64_t n_pois;               /* Poisson sources drawn from the noise key */
    const int32_t *pois_dst;
    const uint8_t *pois_ports;
    const double *pois_w, *pois_rate;

    /* protein model: 0 the per-cell sum of Eq. 21; 1 SPS / PRP diffusion
       (Eq. 5) with diffusivities in um^2/ms */
    int64_t prp_model;
    double d_sps, d_prp;

    /* pair-based STDP synapses (kind 2; Eqs. 6-8, Table 1): trace time
       constants (ms), trace amplitudes and weights (uS) */
    double tau_pre, tau_post, a_pre_amp, a_post_amp, w0, w_max;
} orc_net;

/* ------------------------------------------------------------ event heap */
typedef struct {
    int64_t step;
    double t;
    int64_t src, conn;
    int32_t port;   /* 1 conductance, 2 calcium */
    int32_t syn;
    double w;
} orc_event;

static int ev_less(const orc_event *a, const orc_event *b) {
    if (a->step != b->step) return a->step < b->step;
    if (a->t != b->t) return a->t < b->t;
    if (a->src != b->src) return a->src < b->src;
    if (a->conn != b->conn) return a->conn < b->conn;
    return a->port < b->port;
}

typedef struct {
    orc_event *v;
    int64_t n, cap;
} heap;

static int heap_push(heap *h, orc_event e) {
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        orc_event *nv = (orc_event *)realloc(h->v, (size_t)nc * sizeof(orc_event));
        if (!nv) return -1;
        h->v = nv;
        h->cap = nc;
    }
    int64_t i = h->n++;
    h->v[i] = e;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!ev_less(&h->v[i], &h->v[p])) break;
        orc_event t = h->v[i]; h->v[i] = h->v[p]; h->v[p] = t;
        i = p;
    }
    return 0;
}

static orc_event heap_pop(heap *h) {
    orc_event top = h->v[0];
    h->v[0] = h->v[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && ev_less(&h->v[l], &h->v[m])) m = l;
        if (r < h->n && ev_less(&h->v[r], &h->v[m])) m = r;
        if (m == i) break;
        orc_event t = h->v[i]; h->v[i] = h->v[m]; h->v[m] = t;
        i = m;
    }
    return top;
}

/* ------------------------------------------------------------ Threefry */
/* Threefry-4x64 with 12 rounds (Salmon et al. 2011): the Threefish-256 round
 * function (two add/rotate/xor mixes, then the word permutation that swaps
 * words 1 and 3) with a key injection every four rounds; key-schedule parity
 * constant and rotation table of Threefish-256.  Parity unpinned against the
 * original library (no known-answer vectors available); the tests check its
 * uniformity and independence statistically. */
static uint64_t rotl64(uint64_t x, int r) { return (x << r) | (x >> (64 - r)); }

void orc_threefry4x64_12(const uint64_t ctr[4], const uint64_t key[4], uint64_t out[4]) {
    static const int rot[8][2] = {{14, 16}, {52, 57}, {23, 40}, {5, 37},
                                  {25, 33}, {46, 12}, {58, 22}, {32, 32}};
    uint64_t ks[5];
    ks[4] = 0x1BD11BDAA9FC1A22ULL;
    for (int i = 0; i < 4; i++) { ks[i] = key[i]; ks[4] ^= key[i]; }
    uint64_t x0 = ctr[0] + ks[0], x1 = ctr[1] + ks[1], x2 = ctr[2] + ks[2], x3 = ctr[3] + ks[3];
    for (int r = 0; r < 12; r++) {
        x0 += x1; x1 = rotl64(x1, rot[r % 8][0]); x1 ^= x0;
        x2 += x3; x3 = rotl64(x3, rot[r % 8][1]); x3 ^= x2;
        uint64_t t = x1; x1 = x3; x3 = t;
        if (r % 4 == 3) {
            uint64_t s = (uint64_t)(r + 1) / 4;
            x0 += ks[s % 5]; x1 += ks[(s + 1) % 5]; x2 += ks[(s + 2) % 5]; x3 += ks[(s + 3) % 5] + s;
        }
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

#define ORC_NOISE_TAG 0x5354432d6e6f6973ULL /* domain tag of the early-phase noise */
#define ORC_POIS_TAG 0x706f6973736f6e21ULL  /* domain tag of the Poisson sources */

/* uniform in (0,1): top 53 bits, offset by half an ulp so 0 never occurs */
static double to_unit(uint64_t x) { return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

/* Standard normal of synapse `sid` at step n: one Threefry call per four
 * steps (counter n/4), Box-Muller on output pairs (0,1) and (2,3), cosine
 * branch for even n mod 4, sine for odd. */
double orc_normal(uint64_t seed, uint64_t sid, uint64_t n) {
    uint64_t key[4] = {seed, sid, ORC_NOISE_TAG, 0};
    uint64_t ctr[4] = {n >> 2, 0, 0, 0};
    uint64_t x[4];
    orc_threefry4x64_12(ctr, key, x);
    int lane = (int)(n & 3);
    int pair = lane >> 1;
    double ua = to_unit(x[2 * pair]), ub = to_unit(x[2 * pair + 1]);
    double r = sqrt(-2.0 * log(ua));
    double ang = 6.283185307179586 * ub;
    return (lane & 1) ? r * sin(ang) : r * cos(ang);
}

/* Inter-arrival time (ms) number j of Poisson source k at rate (Hz):
 * -ln(u) / rate with u the first word of Threefry(counter j, key (seed, k,
 * tag, 0)) mapped to (0,1).  Arrival j is the sum of intervals 0..j. */
double orc_poisson_isi(uint64_t seed, uint64_t k, uint64_t j, double rate_hz) {
    uint64_t key[4] = {seed, k, ORC_POIS_TAG, 0};
    uint64_t ctr[4] = {j, 0, 0, 0};
    uint64_t x[4];
    orc_threefry4x64_12(ctr, key, x);
    return -log(to_unit(x[0])) * (1000.0 / rate_hz);
}

/* ------------------------------------------------------------ HH rates */
/* x / (exp(x) - 1), equal to 1 at x = 0 */
static double exprelr(double x) { return (x == 0.0) ? 1.0 : x / expm1(x); }

/* Hodgkin-Huxley 1952 rates (ms^-1), resting potential shifted to -65 mV */
void orc_hh_rates(double v, double r[6]) {
    r[0] = exprelr(-(v + 40.0) / 10.0);              /* alpha_m */
    r[1] = 4.0 * exp(-(v + 65.0) / 18.0);            /* beta_m  */
    r[2] = 0.07 * exp(-(v + 65.0) / 20.0);           /* alpha_h */
    r[3] = 1.0 / (exp(-(v + 35.0) / 10.0) + 1.0);    /* beta_h  */
    r[4] = 0.1 * exprelr(-(v + 55.0) / 10.0);        /* alpha_n */
    r[5] = 0.125 * exp(-(v + 65.0) / 80.0);          /* beta_n  */
}

/* ------------------------------------------------------------ state */
typedef struct {
    orc_net net;       /* shallow copy; arrays owned by the caller */
    int64_t n_cv;
    int64_t step;
    char err[256];
    /* per CV */
    double *V, *Vold, *I, *G, *D, *b;
    double *cdt, *gpas, *gpas_e, *axial, *d0, *scale;
    int64_t *gparent;  /* global parent CV or -1 */
    int64_t *hh_of;    /* HH gate slot or -1 */
    int64_t *cv_cell;  /* owning cell of each CV */
    int64_t n_hh;
    double *gm, *gh, *gn;
    /* per synapse */
    double *g, *c, *h, *z, *decay;
    int64_t *syn_order; /* synapses sorted by (global CV, id) */
    int64_t *cv_syn_off; /* n_cv + 1 into syn_order */
    uint64_t *ev_count, *ev_stepsum; /* per synapse x 2 ports */
    /* per cell */
    double *p, *S;
    uint8_t *post;
    int64_t *out_off, *out_conn; /* outgoing connections per cell */
    /* particle diffusion: CV volume (um^3), the geometric factor of the
       flux between a CV and its parent (um), species concentrations, the
       soma CV and total volume of each cell, per-synapse change of
       |h - h0| in the step, per-CV release, elimination scratch */
    double *vol, *dgeo, *sps, *prp, *dlt, *src, *Dx, *bx, *vtot;
    int64_t *soma;
    /* Poisson sources: next arrival time and its index */
    double *pois_t;
    int64_t *pois_j;
    /* spikes */
    int64_t n_spikes, cap_spikes;
    int64_t *sp_gid, *sp_step;
    double *sp_t;
    heap q;
    double r_c, r_pre, r_post;
} orc;

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }

static int cmp_i64_pair(const void *a, const void *b) {
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}

void orc_destroy(orc *o);

/* Builds the oracle state from a network description; returns NULL and
 * writes a message into err on invalid input. */
orc *orc_create(const orc_net *net, char *err, int errlen) {
    orc *o = (orc *)calloc(1, sizeof(orc));
    if (!o) return NULL;
    o->net = *net;
    const orc_net *N = &o->net;
#define FAIL(...) do { snprintf(err, (size_t)errlen, __VA_ARGS__); orc_destroy(o); return NULL; } while (0)
    if (!(N->dt > 0)) FAIL("dt must be positive");
    int64_t nc = N->n_cells;
    o->n_cv = N->cv_off[nc];
    int64_t ncv = o->n_cv;
    o->V = xcalloc(ncv, 8); o->Vold = xcalloc(ncv, 8); o->I = xcalloc(ncv, 8);
    o->G = xcalloc(ncv, 8); o->D = xcalloc(ncv, 8); o->b = xcalloc(ncv, 8);
    o->cdt = xcalloc(ncv, 8); o->gpas = xcalloc(ncv, 8); o->gpas_e = xcalloc(ncv, 8);
    o->axial = xcalloc(ncv, 8); o->d0 = xcalloc(ncv, 8); o->scale = xcalloc(ncv, 8);
    o->gparent = xcalloc(ncv, 8); o->hh_of = xcalloc(ncv, 8); o->cv_cell = xcalloc(ncv, 8);
    o->vol = xcalloc(ncv, 8); o->dgeo = xcalloc(ncv, 8); o->sps = xcalloc(ncv, 8); o->prp = xcalloc(ncv, 8);
    o->src = xcalloc(ncv, 8); o->Dx = xcalloc(ncv, 8); o->bx = xcalloc(ncv, 8);
    o->vtot = xcalloc(nc, 8); o->soma = xcalloc(nc, 8);
    if (N->prp_model != 0 && N->prp_model != 1) FAIL("prp_model must be 0 or 1");
    if (N->prp_model == 1 && !(N->d_sps >= 0 && N->d_prp >= 0)) FAIL("diffusivities must be >= 0");
    int has_stdp = 0;
    for (int64_t s = 0; s < N->n_syn; s++) has_stdp |= N->syn_kind[s] == 2;
    if (has_stdp && !(N->tau_pre > 0 && N->tau_post > 0 && N->w_max >= 0)) FAIL("STDP time constants must be positive");
    const double pi = 3.14159265358979323846;
    int64_t nhh = 0;
    for (int64_t c = 0; c < nc; c++) {
        const double *P = N->cell_params + 11 * c;
        int64_t b0 = N->cv_off[c], b1 = N->cv_off[c + 1];
        if (b1 <= b0) FAIL("cell %lld has no CV", (long long)c);
        if (N->detector[c] < 0 || N->detector[c] >= b1 - b0) FAIL("bad detector CV");
        for (int64_t i = b0; i < b1; i++) {
            int32_t pl = N->parent[i];
            if (i == b0 ? pl != -1 : (pl < 0 || pl >= i - b0)) FAIL("cell %lld: parent must satisfy parent[0]=-1, 0<=parent[i]<i", (long long)c);
            if (!(N->length[i] > 0) || !(N->diam[i] > 0)) FAIL("non-positive CV geometry");
            o->gparent[i] = (i == b0) ? -1 : b0 + pl;
            o->cv_cell[i] = c;
            /* finite-volume CV: a cylinder, lateral area only */
            double area = pi * N->diam[i] * N->length[i];          /* um^2 */
            o->cdt[i] = (1e-5 * P[0] * area) / N->dt;              /* C/dt, nF/ms = uS */
            if (N->mech[i] == 1) {
                o->hh_of[i] = nhh++;
                o->scale[i] = 1e-2 * area;                          /* S/cm^2 -> uS */
                o->gpas[i] = 0.0;
                o->gpas_e[i] = 0.0;
            } else {
                o->hh_of[i] = -1;
                o->scale[i] = 0.0;
                o->gpas[i] = 1e-2 * P[3] * area;
                o->gpas_e[i] = o->gpas[i] * P[4];
            }
            o->V[i] = P[2];
        }
        for (int64_t i = b0 + 1; i < b1; i++) {
            int64_t k = o->gparent[i];
            double ri = 0.5 * N->diam[i], rk = 0.5 * N->diam[k];
            /* series resistance of the two half-cylinders between the nodes */
            double rsum = N->length[i] / (2.0 * pi * ri * ri) + N->length[k] / (2.0 * pi * rk * rk);
            o->axial[i] = 1e2 / (P[1] * rsum);                     /* uS */
            /* the same half-cylinder series form for a diffusive flux:
               cross-section over length, summed as resistances */
            o->dgeo[i] = 1.0 / rsum;                                /* um */
        }
        for (int64_t i = b0; i < b1; i++) {
            double r = 0.5 * N->diam[i];
            o->vol[i] = pi * r * r * N->length[i];                  /* um^3 */
            o->vtot[c] += o->vol[i];
        }
        o->soma[c] = b0 + N->detector[c];
    }
    /* diagonal invariant: C/dt + g_pas + (own axial + children's axial) */
    double *axsum = xcalloc(ncv, 8);
    for (int64_t i = 0; i < ncv; i++) axsum[i] = o->axial[i];
    for (int64_t i = 0; i < ncv; i++) if (o->gparent[i] >= 0) axsum[o->gparent[i]] += o->axial[i];
    for (int64_t i = 0; i < ncv; i++) o->d0[i] = (o->cdt[i] + o->gpas[i]) + axsum[i];
    free(axsum);
    o->n_hh = nhh;
    o->gm = xcalloc(nhh, 8); o->gh = xcalloc(nhh, 8); o->gn = xcalloc(nhh, 8);
    for (int64_t i = 0; i < ncv; i++) {
        if (o->hh_of[i] < 0) continue;
        double r[6];
        orc_hh_rates(o->V[i], r);
        int64_t k = o->hh_of[i];
        o->gm[k] = r[0] / (r[0] + r[1]);
        o->gh[k] = r[2] / (r[2] + r[3]);
        o->gn[k] = r[4] / (r[4] + r[5]);
    }
    /* synapses */
    int64_t ns = N->n_syn;
    o->g = xcalloc(ns, 8); o->c = xcalloc(ns, 8); o->h = xcalloc(ns, 8); o->z = xcalloc(ns, 8);
    o->decay = xcalloc(ns, 8); o->dlt = xcalloc(ns, 8);
    o->ev_count = xcalloc(2 * ns, 8); o->ev_stepsum = xcalloc(2 * ns, 8);
    int64_t *pairs = xcalloc(2 * ns, 8);
    for (int64_t s = 0; s < ns; s++) {
        int32_t cell = N->syn_cell[s];
        if (cell < 0 || cell >= nc) FAIL("synapse %lld: bad cell", (long long)s);
        if (N->syn_cv[s] < 0 || N->syn_cv[s] >= N->cv_off[cell + 1] - N->cv_off[cell]) FAIL("synapse %lld: bad CV", (long long)s);
        if (!(N->syn_tau[s] > 0)) FAIL("synapse %lld: tau must be positive", (long long)s);
        if (N->syn_kind[s] > 2) FAIL("synapse %lld: bad kind", (long long)s);
        o->decay[s] = exp(-N->dt / N->syn_tau[s]);
        /* h holds the early-phase weight of a tagging-and-capture synapse
           and the weight w of an STDP synapse (whose traces a_pre, a_post
           live in c and z) */
        o->h[s] = (N->syn_kind[s] == 1) ? N->h0 : ((N->syn_kind[s] == 2) ? N->w0 : 0.0);
        pairs[2 * s] = N->cv_off[cell] + N->syn_cv[s];
        pairs[2 * s + 1] = s;
    }
    qsort(pairs, (size_t)ns, 16, cmp_i64_pair);
    o->syn_order = xcalloc(ns, 8);
    o->cv_syn_off = xcalloc(ncv + 1, 8);
    for (int64_t k = 0; k < ns; k++) { o->syn_order[k] = pairs[2 * k + 1]; o->cv_syn_off[pairs[2 * k] + 1]++; }
    for (int64_t i = 0; i < ncv; i++) o->cv_syn_off[i + 1] += o->cv_syn_off[i];
    free(pairs);
    /* cells */
    o->p = xcalloc(nc, 8); o->S = xcalloc(nc, 8); o->post = xcalloc(nc, 1);
    o->out_off = xcalloc(nc + 1, 8); o->out_conn = xcalloc(N->n_conn, 8);
    for (int64_t k = 0; k < N->n_conn; k++) {
        if (N->conn_src[k] < 0 || N->conn_src[k] >= nc) FAIL("connection %lld: bad source", (long long)k);
        if (N->conn_dst[k] < 0 || N->conn_dst[k] >= ns) FAIL("connection %lld: bad target", (long long)k);
        if ((N->conn_ports[k] & 2) && N->syn_kind[N->conn_dst[k]] != 1) FAIL("calcium port needs a plasticity synapse");
        if (N->conn_ports[k] == 0 || N->conn_ports[k] > 3) FAIL("bad ports");
        if (!(N->conn_d[k] >= N->dt)) FAIL("connection %lld: delay below dt", (long long)k);
        o->out_off[N->conn_src[k] + 1]++;
    }
    for (int64_t c = 0; c < nc; c++) o->out_off[c + 1] += o->out_off[c];
    int64_t *fill = xcalloc(nc, 8);
    for (int64_t k = 0; k < N->n_conn; k++) {
        int64_t sc = N->conn_src[k];
        o->out_conn[o->out_off[sc] + fill[sc]++] = k;
    }
    free(fill);
    o->r_c = exp(-N->dt / N->tau_c);
    o->r_pre = has_stdp ? exp(-N->dt / N->tau_pre) : 1.0;
    o->r_post = has_stdp ? exp(-N->dt / N->tau_post) : 1.0;
    /* explicit presynaptic trains enter the queue up front */
    for (int64_t tr = 0; tr < N->n_trains; tr++) {
        int32_t s = N->train_dst[tr];
        if (s < 0 || s >= ns) FAIL("train %lld: bad target", (long long)tr);
        if ((N->train_ports[tr] & 2) && N->syn_kind[s] != 1) FAIL("calcium port needs a plasticity synapse");
        for (int64_t j = N->train_off[tr]; j < N->train_off[tr + 1]; j++) {
            double t = N->train_times[j];
            if (!(t >= 0)) FAIL("negative train time");
            orc_event e = {0};
            e.src = nc + tr; e.conn = 0; e.syn = s; e.w = N->train_w[tr];
            if (N->train_ports[tr] & 1) {
                e.t = t; e.step = (int64_t)floor(e.t / N->dt); e.port = 1;
                if (heap_push(&o->q, e)) FAIL("out of memory");
            }
            if (N->train_ports[tr] & 2) {
                e.t = t + N->t_cd; e.step = (int64_t)floor(e.t / N->dt); e.port = 2;
                if (heap_push(&o->q, e)) FAIL("out of memory");
            }
        }
    }
    for (int64_t k = 0; k < N->n_clamps; k++) {
        int32_t cell = N->clamp_cell[k];
        if (cell < 0 || cell >= nc || N->clamp_cv[k] < 0 || N->clamp_cv[k] >= N->cv_off[cell + 1] - N->cv_off[cell]) FAIL("bad clamp");
    }
    o->pois_t = xcalloc(N->n_pois, 8);
    o->pois_j = xcalloc(N->n_pois, 8);
    for (int64_t k = 0; k < N->n_pois; k++) {
        int32_t s = N->pois_dst[k];
        if (s < 0 || s >= ns) FAIL("Poisson source %lld: bad target", (long long)k);
        if ((N->pois_ports[k] & 2) && N->syn_kind[s] != 1) FAIL("calcium port needs a plasticity synapse");
        if (!(N->pois_rate[k] >= 0)) FAIL("negative rate");
        o->pois_t[k] = N->pois_rate[k] > 0 ? orc_poisson_isi(N->seed, (uint64_t)k, 0, N->pois_rate[k]) : INFINITY;
    }
#undef FAIL
    return o;
}

static int record_spike(orc *o, int64_t gid, int64_t step, double t) {
    if (o->n_spikes == o->cap_spikes) {
        int64_t nc = o->cap_spikes ? 2 * o->cap_spikes : 1024;
        int64_t *a = realloc(o->sp_gid, (size_t)nc * 8), *b;
        if (!a) return -1;
        o->sp_gid = a;
        b = realloc(o->sp_step, (size_t)nc * 8);
        if (!b) return -1;
        o->sp_step = b;
        double *t2 = realloc(o->sp_t, (size_t)nc * 8);
        if (!t2) return -1;
        o->sp_t = t2;
        o->cap_spikes = nc;
    }
    o->sp_gid[o->n_spikes] = gid; o->sp_step[o->n_spikes] = step; o->sp_t[o->n_spikes] = t;
    o->n_spikes++;
    return 0;
}

/* Membrane current I (nA, outward positive) and its voltage derivative G
 * (uS) per CV at the present voltage: HH first, then synapses in (CV, id)
 * order, then the clamps active at time tn. */
static void currents(orc *o, double tn) {
    const orc_net *N = &o->net;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < o->n_cv; i++) {
        double I = 0.0, G = 0.0, v = o->V[i];
        if (o->hh_of[i] >= 0) {
            int64_t k = o->hh_of[i];
            const double *P = N->cell_params + 11 * o->cv_cell[i];
            double gna = P[5] * o->gm[k] * o->gm[k] * o->gm[k] * o->gh[k];
            double gk = P[6] * o->gn[k] * o->gn[k] * o->gn[k] * o->gn[k];
            double idens = gna * (v - P[8]) + gk * (v - P[9]) + P[7] * (v - P[10]);
            I = o->scale[i] * idens;
            G = o->scale[i] * (gna + gk + P[7]);
        }
        for (int64_t q = o->cv_syn_off[i]; q < o->cv_syn_off[i + 1]; q++) {
            int64_t s = o->syn_order[q];
            I += o->g[s] * (v - N->syn_erev[s]);
            G += o->g[s];
        }
        o->I[i] = I;
        o->G[i] = G;
    }
    for (int64_t k = 0; k < N->n_clamps; k++) {
        if (N->clamp_t0[k] <= tn && tn < N->clamp_t0[k] + N->clamp_dur[k])
            o->I[N->cv_off[N->clamp_cell[k]] + N->clamp_cv[k]] -= N->clamp_amp[k];
    }
}

/* One backward-Euler step of the diffusion equation (Eq. 5) of one species
 * over the CVs b0..b1-1 of a cell, in amounts: (V_i + dt sum_j a_ij) X_i -
 * dt sum_j a_ij X_j = bx_i, a_ij = D x (cross-section / length) of the
 * CV-parent pair, sealed ends; solved by the same elimination as the cable
 * system.  bx holds the right-hand side on entry; X receives the
 * concentrations. */
static void diffuse_cell(orc *o, int64_t b0, int64_t b1, double dcoef, double *X) {
    const double dt = o->net.dt;
    for (int64_t i = b0; i < b1; i++) o->Dx[i] = o->vol[i];
    for (int64_t i = b0 + 1; i < b1; i++) {
        double a = dt * (dcoef * o->dgeo[i]);
        o->Dx[i] += a;
        o->Dx[o->gparent[i]] += a;
    }
    for (int64_t i = b1 - 1; i > b0; i--) {
        int64_t p = o->gparent[i];
        double u = -(dt * (dcoef * o->dgeo[i]));
        double f = u / o->Dx[i];
        o->Dx[p] -= f * u;
        o->bx[p] -= f * o->bx[i];
    }
    X[b0] = o->bx[b0] / o->Dx[b0];
    for (int64_t i = b0 + 1; i < b1; i++) {
        double u = -(dt * (dcoef * o->dgeo[i]));
        X[i] = (o->bx[i] - u * X[o->gparent[i]]) / o->Dx[i];
    }
}

/* One step n -> n+1.  Returns 0, or -1 with a message. */
static int orc_step(orc *o) {
    const orc_net *N = &o->net;
    const int64_t n = o->step, nc = N->n_cells, ncv = o->n_cv;
    const double dt = N->dt, tn = (double)n * dt, h0 = N->h0;

    /* Poisson arrivals due in this step enter the queue (their calcium
       events later) */
    for (int64_t k = 0; k < N->n_pois; k++) {
        while (floor(o->pois_t[k] / dt) <= (double)n) {
            double t = o->pois_t[k];
            orc_event e = {0};
            e.src = nc + N->n_trains + k; e.conn = 0; e.syn = N->pois_dst[k]; e.w = N->pois_w[k];
            if (N->pois_ports[k] & 1) {
                e.t = t; e.step = (int64_t)floor(t / dt); e.port = 1;
                if (heap_push(&o->q, e)) { snprintf(o->err, sizeof o->err, "out of memory"); return -1; }
            }
            if (N->pois_ports[k] & 2) {
                e.t = t + N->t_cd; e.step = (int64_t)floor(e.t / dt); e.port = 2;
                if (heap_push(&o->q, e)) { snprintf(o->err, sizeof o->err, "out of memory"); return -1; }
            }
            o->pois_j[k] += 1;
            o->pois_t[k] = t + orc_poisson_isi(N->seed, (uint64_t)k, (uint64_t)o->pois_j[k], N->pois_rate[k]);
        }
    }

    /* 1. event delivery, then the post-synaptic hook */
    while (o->q.n > 0 && o->q.v[0].step <= n) {
        orc_event e = heap_pop(&o->q);
        if (e.step < n) { snprintf(o->err, sizeof o->err, "event for step %lld found at step %lld", (long long)e.step, (long long)n); return -1; }
        int32_t s = e.syn;
        if (e.port == 1) {
            if (N->syn_kind[s] == 1) {
                o->g[s] += e.w * ((o->h[s] + h0 * o->z[s]) / h0);
            } else if (N->syn_kind[s] == 2) {
                /* STDP (Eqs. 6-8): the spike transmits the present weight,
                   clipped to [0, w_max]; then a_pre += A_pre, w += a_post */
                double w = o->h[s];
                double wc = w < 0.0 ? 0.0 : (w > N->w_max ? N->w_max : w);
                o->g[s] += e.w * wc;
                o->c[s] += N->a_pre_amp;
                o->h[s] = w + o->z[s];
            } else {
                o->g[s] += e.w;
            }
        } else {
            o->c[s] += N->c_pre;
        }
        o->ev_count[2 * s + e.port - 1] += 1;
        o->ev_stepsum[2 * s + e.port - 1] += (uint64_t)n;
    }
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N->n_syn; s++) {
        if (!o->post[N->syn_cell[s]]) continue;
        if (N->syn_kind[s] == 1) {
            o->c[s] += N->c_post;
        } else if (N->syn_kind[s] == 2) {
            /* STDP post-synaptic spike: a_post += A_post, w += a_pre */
            o->z[s] += N->a_post_amp;
            o->h[s] += o->c[s];
        }
    }
    memset(o->post, 0, (size_t)nc);

    /* 2. currents and conductances at V^n */
    currents(o, tn);

    /* 3. assembly and 4. Hines solve, cell by cell */
    for (int64_t i = 0; i < ncv; i++) o->Vold[i] = o->V[i];
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t cell = 0; cell < nc; cell++) {
        int64_t b0 = N->cv_off[cell], b1 = N->cv_off[cell + 1];
        for (int64_t i = b0; i < b1; i++) {
            double v = o->V[i];
            o->D[i] = o->d0[i] + o->G[i];
            o->b[i] = ((o->cdt[i] * v + o->gpas_e[i]) - o->I[i]) + o->G[i] * v;
        }
        for (int64_t i = b1 - 1; i > b0; i--) {
            int64_t p = o->gparent[i];
            double u = -o->axial[i];
            double f = u / o->D[i];
            o->D[p] -= f * u;
            o->b[p] -= f * o->b[i];
        }
        o->V[b0] = o->b[b0] / o->D[b0];
        for (int64_t i = b0 + 1; i < b1; i++) {
            double u = -o->axial[i];
            o->V[i] = (o->b[i] - u * o->V[o->gparent[i]]) / o->D[i];
        }
    }

    /* 5. gates at V^{n+1}; synaptic conductance decay */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ncv; i++) {
        if (o->hh_of[i] < 0) continue;
        int64_t k = o->hh_of[i];
        double r[6];
        orc_hh_rates(o->V[i], r);
        double *x[3] = {&o->gm[k], &o->gh[k], &o->gn[k]};
        for (int j = 0; j < 3; j++) {
            double a = r[2 * j], bb = r[2 * j + 1];
            double xinf = a / (a + bb);
            *x[j] = xinf + (*x[j] - xinf) * exp(-dt * (a + bb));
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N->n_syn; s++) o->g[s] *= o->decay[s];

    /* 6. plasticity: S from step-start h; h, z from step-start h, z, p, c.
       With particle diffusion the trigger is the step-start SPS
       concentration at the soma against theta_pro / V_tot (Eq. 23), and z
       takes the step-start PRP concentration of its synapse's CV. */
    const int diffuse = N->prp_model == 1;
    if (!diffuse) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t cell = 0; cell < nc; cell++) {
            double S = 0.0;
            for (int64_t i = N->cv_off[cell]; i < N->cv_off[cell + 1]; i++)
                for (int64_t q = o->cv_syn_off[i]; q < o->cv_syn_off[i + 1]; q++) {
                    int64_t s = o->syn_order[q];
                    if (N->syn_kind[s] == 1) S += fabs(o->h[s] - h0);
                }
            o->S[cell] = S;
        }
    } else {
        for (int64_t cell = 0; cell < nc; cell++)
            o->S[cell] = (o->sps[o->soma[cell]] - N->theta_pro / o->vtot[cell] > 0.0) ? 1.0 : 0.0;
    }
    const double ah = dt / N->tau_h, az = dt / N->tau_z;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N->n_syn; s++) {
        if (N->syn_kind[s] == 2) {
            /* STDP traces decay exactly over the step (Eqs. 6, 7) */
            o->c[s] *= o->r_pre;
            o->z[s] *= o->r_post;
            continue;
        }
        if (N->syn_kind[s] != 1) continue;
        int32_t cell = N->syn_cell[s];
        double c = o->c[s], h = o->h[s], z = o->z[s];
        double p = diffuse ? o->prp[N->cv_off[cell] + N->syn_cv[s]] : o->p[cell];
        double thp = (c - N->theta_p > 0.0) ? 1.0 : 0.0;
        double thd = (c - N->theta_d > 0.0) ? 1.0 : 0.0;
        double drift = 0.1 * (h0 - h) + N->gamma_p * (10.0 - h) * thp - N->gamma_d * h * thd;
        double hn = h + ah * drift;
        if (thp + thd > 0.0)
            hn += N->sigma_pl * sqrt((thp + thd) * ah) * orc_normal(N->seed, (uint64_t)s, (uint64_t)n);
        double tagp = ((h - h0) - N->theta_tag > 0.0) ? 1.0 : 0.0;
        double tagd = ((h0 - h) - N->theta_tag > 0.0) ? 1.0 : 0.0;
        double zn = z + az * p * N->f_int * ((1.0 - z) * tagp - (z + 0.5) * tagd);
        o->dlt[s] = fabs(hn - h0) - fabs(h - h0);
        o->h[s] = hn;
        o->z[s] = zn;
        o->c[s] = c * o->r_c;
    }
    const double ap = dt / N->tau_p;
    if (!diffuse) {
#pragma omp parallel for schedule(static)
        for (int64_t cell = 0; cell < nc; cell++) {
            double trig = (o->S[cell] - N->theta_pro > 0.0) ? 1.0 : 0.0;
            o->p[cell] = o->p[cell] + ap * (-o->p[cell] + N->p_max * trig);
        }
    } else {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t cell = 0; cell < nc; cell++) {
            int64_t b0 = N->cv_off[cell], b1 = N->cv_off[cell + 1];
            /* SPS released in the step per CV: the change of |h - h0| of its
               plastic synapses, in (CV, id) order */
            for (int64_t i = b0; i < b1; i++) {
                double r = 0.0;
                for (int64_t q = o->cv_syn_off[i]; q < o->cv_syn_off[i + 1]; q++) {
                    int64_t s = o->syn_order[q];
                    if (N->syn_kind[s] == 1) r += o->dlt[s];
                }
                o->src[i] = r;
            }
            for (int64_t i = b0; i < b1; i++) o->bx[i] = o->vol[i] * o->sps[i] + o->src[i];
            diffuse_cell(o, b0, b1, N->d_sps, o->sps);
            /* PRP: decay in every CV; synthesis at the soma while triggered,
               scaled so that the well-mixed cell follows Eq. 21 */
            for (int64_t i = b0; i < b1; i++) {
                double x = o->prp[i];
                o->bx[i] = o->vol[i] * (x + ap * (-x));
            }
            o->bx[o->soma[cell]] += ap * (N->p_max * o->vtot[cell]) * o->S[cell];
            diffuse_cell(o, b0, b1, N->d_prp, o->prp);
        }
    }

    /* 7. threshold detection and event generation */
    for (int64_t cell = 0; cell < nc; cell++) {
        int64_t d = N->cv_off[cell] + N->detector[cell];
        double v0 = o->Vold[d], v1 = o->V[d];
        if (!(v0 < N->theta && v1 >= N->theta)) continue;
        double ts = tn + dt * ((N->theta - v0) / (v1 - v0));
        if (record_spike(o, cell, n, ts)) { snprintf(o->err, sizeof o->err, "out of memory"); return -1; }
        o->post[cell] = 1;
        for (int64_t q = o->out_off[cell]; q < o->out_off[cell + 1]; q++) {
            int64_t k = o->out_conn[q];
            orc_event e = {0};
            e.src = cell; e.conn = k; e.syn = N->conn_dst[k]; e.w = N->conn_w[k];
            double te = ts + N->conn_d[k];
            if (N->conn_ports[k] & 1) {
                e.t = te; e.step = (int64_t)floor(te / dt); e.port = 1;
                if (e.step <= n) { snprintf(o->err, sizeof o->err, "event scheduled in the past"); return -1; }
                if (heap_push(&o->q, e)) { snprintf(o->err, sizeof o->err, "out of memory"); return -1; }
            }
            if (N->conn_ports[k] & 2) {
                e.t = te + N->t_cd; e.step = (int64_t)floor(e.t / dt); e.port = 2;
                if (e.step <= n) { snprintf(o->err, sizeof o->err, "event scheduled in the past"); return -1; }
                if (heap_push(&o->q, e)) { snprintf(o->err, sizeof o->err, "out of memory"); return -1; }
            }
        }
    }
    for (int64_t i = 0; i < ncv; i++) {
        if (!isfinite(o->V[i])) { snprintf(o->err, sizeof o->err, "non-finite voltage at CV %lld, step %lld", (long long)i, (long long)n); return -1; }
    }
    o->step = n + 1;
    return 0;
}

/* Fast-forward (Sec. 3.5, the phases of slow network dynamics in the 8-h
 * paradigm): n_long steps of length dt_long (a whole multiple of dt) that
 * advance only the slow plasticity variables, with spiking and calcium
 * dynamics off.  Per long step, from step-start values and with the
 * calcium thresholds not crossed (no early-phase drive, no noise):
 *   h <- h + (dt_long / tau_h) 0.1 (h0 - h)                     (Eq. 17)
 *   z <- z + (dt_long / tau_z) p f_int [(1 - z) tag+ - (z + 0.5) tag-]  (Eq. 20)
 *   p <- p + (dt_long / tau_p) (-p + p_max [S - theta_pro > 0])       (Eq. 21)
 * with S = sum |h - h0| over the cell's plastic synapses (step-start h);
 * calcium and synaptic conductances decay exactly over each long step;
 * membrane voltages and gates stay as they are.  Everything in flight is
 * dropped: spikes before the new time cause no events, post-synaptic flags
 * clear, explicit train arrivals before the new time are skipped, and a
 * Poisson source whose next arrival falls before it draws that arrival
 * again (index + 1) as the new time plus an interval (the process is
 * memoryless).  Time moves to t + n_long dt_long.  The per-cell protein
 * model only.  Returns 0, or -1 with a message. */
int orc_fast_forward(orc *o, int64_t n_long, double dt_long) {
    const orc_net *N = &o->net;
    const int64_t nc = N->n_cells;
    const double dt = N->dt, h0 = N->h0;
    if (N->prp_model != 0) { snprintf(o->err, sizeof o->err, "fast-forward needs the per-cell protein model"); return -1; }
    double q = dt_long / dt;
    int64_t ratio = (int64_t)floor(q + 0.5);
    if (n_long < 0 || ratio < 1 || fabs((double)ratio * dt - dt_long) > 1e-9 * dt_long) {
        snprintf(o->err, sizeof o->err, "dt_long must be a positive whole multiple of dt"); return -1;
    }
    const double ah = dt_long / N->tau_h, az = dt_long / N->tau_z, ap = dt_long / N->tau_p;
    const double rc = exp(-dt_long / N->tau_c);
    for (int64_t k = 0; k < n_long; k++) {
        for (int64_t cell = 0; cell < nc; cell++) {
            double S = 0.0;
            for (int64_t i = N->cv_off[cell]; i < N->cv_off[cell + 1]; i++)
                for (int64_t qq = o->cv_syn_off[i]; qq < o->cv_syn_off[i + 1]; qq++) {
                    int64_t s = o->syn_order[qq];
                    if (N->syn_kind[s] == 1) S += fabs(o->h[s] - h0);
                }
            o->S[cell] = S;
        }
        for (int64_t s = 0; s < N->n_syn; s++) {
            o->g[s] *= exp(-dt_long / N->syn_tau[s]);
            if (N->syn_kind[s] != 1) continue;
            double h = o->h[s], z = o->z[s], p = o->p[N->syn_cell[s]];
            double tagp = ((h - h0) - N->theta_tag > 0.0) ? 1.0 : 0.0;
            double tagd = ((h0 - h) - N->theta_tag > 0.0) ? 1.0 : 0.0;
            o->h[s] = h + ah * (0.1 * (h0 - h));
            o->z[s] = z + az * p * N->f_int * ((1.0 - z) * tagp - (z + 0.5) * tagd);
            o->c[s] *= rc;
        }
        for (int64_t cell = 0; cell < nc; cell++) {
            double trig = (o->S[cell] - N->theta_pro > 0.0) ? 1.0 : 0.0;
            o->p[cell] = o->p[cell] + ap * (-o->p[cell] + N->p_max * trig);
        }
    }
    const int64_t n_new = o->step + n_long * ratio;
    const double t_new = (double)n_new * dt;
    memset(o->post, 0, (size_t)nc);
    /* drop every queued event, then queue the train arrivals from the new
       time on again */
    o->q.n = 0;
    for (int64_t tr = 0; tr < N->n_trains; tr++) {
        for (int64_t j = N->train_off[tr]; j < N->train_off[tr + 1]; j++) {
            double t = N->train_times[j];
            if (floor(t / dt) < (double)n_new) continue;
            orc_event e = {0};
            e.src = nc + tr; e.conn = 0; e.syn = N->train_dst[tr]; e.w = N->train_w[tr];
            if (N->train_ports[tr] & 1) {
                e.t = t; e.step = (int64_t)floor(e.t / dt); e.port = 1;
                if (heap_push(&o->q, e)) { snprintf(o->err, sizeof o->err, "out of memory"); return -1; }
            }
            if (N->train_ports[tr] & 2) {
                e.t = t + N->t_cd; e.step = (int64_t)floor(e.t / dt); e.port = 2;
                if (heap_push(&o->q, e)) { snprintf(o->err, sizeof o->err, "out of memory"); return -1; }
            }
        }
    }
    for (int64_t k = 0; k < N->n_pois; k++) {
        if (N->pois_rate[k] > 0 && floor(o->pois_t[k] / dt) < (double)n_new) {
            o->pois_j[k] += 1;
            o->pois_t[k] = t_new + orc_poisson_isi(N->seed, (uint64_t)k, (uint64_t)o->pois_j[k], N->pois_rate[k]);
        }
    }
    o->step = n_new;
    return 0;
}

int orc_run(orc *o, int64_t n_steps) {
    for (int64_t k = 0; k < n_steps; k++)
        if (orc_step(o)) return -1;
    return 0;
}

const char *orc_error(const orc *o) { return o->err; }
int64_t orc_step_count(const orc *o) { return o->step; }
int64_t orc_n_cv(const orc *o) { return o->n_cv; }
int64_t orc_n_hh(const orc *o) { return o->n_hh; }
int64_t orc_spike_count(const orc *o) { return o->n_spikes; }

void orc_spikes(const orc *o, int64_t *gid, int64_t *step, double *t) {
    for (int64_t k = 0; k < o->n_spikes; k++) { gid[k] = o->sp_gid[k]; step[k] = o->sp_step[k]; t[k] = o->sp_t[k]; }
}

/* what: 0 V, 1 m, 2 h(HH), 3 n, 4 g, 5 c, 6 h(weight), 7 z, 8 p,
 *       9 delivered-event counts (2 per synapse), 10 step sums (2 per synapse),
 *       11 SPS concentration, 12 PRP concentration (per CV) */
int orc_read(const orc *o, int what, void *out) {
    const orc_net *N = &o->net;
    size_t nh = (size_t)o->n_hh, ns = (size_t)N->n_syn;
    switch (what) {
    case 0: memcpy(out, o->V, (size_t)o->n_cv * 8); return 0;
    case 1: memcpy(out, o->gm, nh * 8); return 0;
    case 2: memcpy(out, o->gh, nh * 8); return 0;
    case 3: memcpy(out, o->gn, nh * 8); return 0;
    case 4: memcpy(out, o->g, ns * 8); return 0;
    case 5: memcpy(out, o->c, ns * 8); return 0;
    case 6: memcpy(out, o->h, ns * 8); return 0;
    case 7: memcpy(out, o->z, ns * 8); return 0;
    case 8: memcpy(out, o->p, (size_t)N->n_cells * 8); return 0;
    case 9: memcpy(out, o->ev_count, 2 * ns * 8); return 0;
    case 10: memcpy(out, o->ev_stepsum, 2 * ns * 8); return 0;
    case 11: memcpy(out, o->sps, (size_t)o->n_cv * 8); return 0;
    case 12: memcpy(out, o->prp, (size_t)o->n_cv * 8); return 0;
    default: return -1;
    }
}

/* Test hooks: overwrite a state array (same codes as orc_read, 0-8, 11, 12). */
int orc_write(orc *o, int what, const double *in) {
    const orc_net *N = &o->net;
    size_t nh = (size_t)o->n_hh, ns = (size_t)N->n_syn;
    switch (what) {
    case 0: memcpy(o->V, in, (size_t)o->n_cv * 8); return 0;
    case 1: memcpy(o->gm, in, nh * 8); return 0;
    case 2: memcpy(o->gh, in, nh * 8); return 0;
    case 3: memcpy(o->gn, in, nh * 8); return 0;
    case 4: memcpy(o->g, in, ns * 8); return 0;
    case 5: memcpy(o->c, in, ns * 8); return 0;
    case 6: memcpy(o->h, in, ns * 8); return 0;
    case 7: memcpy(o->z, in, ns * 8); return 0;
    case 8: memcpy(o->p, in, (size_t)N->n_cells * 8); return 0;
    case 11: memcpy(o->sps, in, (size_t)o->n_cv * 8); return 0;
    case 12: memcpy(o->prp, in, (size_t)o->n_cv * 8); return 0;
    default: return -1;
    }
}

/* The assembled system of the current state, for the dense-solve check:
 * diagonal, off-diagonal (to parent) and right-hand side after the step's
 * currents are computed, without advancing time.  Fills D, U, b (n_cv). */
int orc_assemble(orc *o, double *Dout, double *Uout, double *bout) {
    currents(o, (double)o->step * o->net.dt);
    for (int64_t i = 0; i < o->n_cv; i++) {
        double v = o->V[i];
        Dout[i] = o->d0[i] + o->G[i];
        bout[i] = ((o->cdt[i] * v + o->gpas_e[i]) - o->I[i]) + o->G[i] * v;
        Uout[i] = -o->axial[i];
    }
    return 0;
}

/* Stand-alone Hines solve of a given tree system (parent[i] < i, parent[0]
 * = -1): the same elimination as the step, exposed for the dense LU check.
 * D and b are overwritten; the solution goes to x. */
void orc_hines(int64_t n, const int64_t *parent, const double *U, double *D, double *b, double *x) {
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t p = parent[i];
        double f = U[i] / D[i];
        D[p] -= f * U[i];
        b[p] -= f * b[i];
    }
    x[0] = b[0] / D[0];
    for (int64_t i = 1; i < n; i++) x[i] = (b[i] - U[i] * x[parent[i]]) / D[i];
}

/* ------------------------------------------------------------ Graupner-Brunel */
/* The calcium-based rule of Graupner and Brunel (Sec. 3.3, Eqs. 10-12,
 * Table 3) on independent single synapses under the pairing protocol of
 * the DP curve: n_pairs presynaptic spikes, one every period_ms from t0_ms;
 * each adds c_pre to the calcium t_cd later (delivered at the step
 * floor(t / dt)), and a postsynaptic spike delay_ms[i] after it adds c_post
 * (the postsynaptic spikes are imposed, as in the protocol).  Per step n,
 * after that step's jumps (presynaptic first): with Theta_p = [c > theta_p]
 * and Theta_d = [c > theta_d] from the step-start calcium, the
 * Euler-Maruyama step of Eq. 10,
 *   w <- w + (dt / tau_w) (-w (1 - w) (w_* - w) + gamma_p (1 - w) Theta_p
 *                          - gamma_d w Theta_d)
 *          + sigma sqrt((Theta_p + Theta_d) dt / tau_w) N_n   (Eq. 11),
 * N_n the standard normal of trial first_id + i at step n (the generator of
 * the early-phase noise keyed by the trial), then c <- c exp(-dt / tau_c)
 * (Eq. 12).  The run covers the steps of n_pairs periods from t0.  Writes
 * the final weight and calcium of every trial. */
typedef struct {
    double tau_w, w_star, gamma_p, gamma_d, theta_p, theta_d, sigma, tau_c, c_pre, c_post, t_cd;
} orc_gb;

int orc_gb_trials(const orc_gb *P, double dt, int64_t n_trials, const double *delay_ms, const double *w0,
                  int64_t n_pairs, double period_ms, double t0_ms, uint64_t seed, uint64_t first_id,
                  double *w_out, double *c_out) {
    if (!(dt > 0) || !(P->tau_w > 0) || !(P->tau_c > 0) || n_pairs < 0) return -1;
    const int64_t n_end = (int64_t)floor((t0_ms + (double)n_pairs * period_ms) / dt);
    const double ah = dt / P->tau_w, rc = exp(-dt / P->tau_c);
    for (int64_t i = 0; i < n_trials; i++) {
        double w = w0[i], c = 0.0;
        int64_t kp = 0, kq = 0;
        for (int64_t n = 0; n < n_end; n++) {
            while (kp < n_pairs && floor((t0_ms + (double)kp * period_ms + P->t_cd) / dt) <= (double)n) {
                c += P->c_pre;
                kp++;
            }
            while (kq < n_pairs && floor((t0_ms + (double)kq * period_ms + delay_ms[i]) / dt) <= (double)n) {
                c += P->c_post;
                kq++;
            }
            double thp = (c - P->theta_p > 0.0) ? 1.0 : 0.0;
            double thd = (c - P->theta_d > 0.0) ? 1.0 : 0.0;
            double drift = -w * (1.0 - w) * (P->w_star - w) + P->gamma_p * (1.0 - w) * thp - P->gamma_d * w * thd;
            double wn = w + ah * drift;
            if (thp + thd > 0.0)
                wn += P->sigma * sqrt((thp + thd) * ah) * orc_normal(seed, first_id + (uint64_t)i, (uint64_t)n);
            w = wn;
            c = c * rc;
        }
        w_out[i] = w;
        if (c_out) c_out[i] = c;
    }
    return 0;
}

void orc_destroy(orc *o) {
    if (!o) return;
    void *ptrs[] = {o->V, o->Vold, o->I, o->G, o->D, o->b, o->cdt, o->gpas, o->gpas_e, o->axial,
                    o->d0, o->scale, o->gparent, o->hh_of, o->cv_cell, o->gm, o->gh, o->gn, o->g, o->c, o->h,
                    o->z, o->decay, o->syn_order, o->cv_syn_off, o->ev_count, o->ev_stepsum, o->p,
                    o->S, o->post, o->vol, o->dgeo, o->sps, o->prp, o->dlt, o->src, o->Dx, o->bx,
                    o->vtot, o->soma, o->out_off, o->out_conn, o->sp_gid, o->sp_step, o->sp_t, o->q.v,
                    o->pois_t, o->pois_j};
    for (size_t k = 0; k < sizeof ptrs / sizeof ptrs[0]; k++) free(ptrs[k]);
    free(o);
}
