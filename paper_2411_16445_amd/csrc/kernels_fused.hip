// Batched form: one fused kernel per epoch.
//
// Cells only interact through spike events, and an event is delivered at
// least one epoch (K steps, K dt below the smallest delay) after the spike
// that caused it.  Within an epoch every cell therefore evolves on its own:
// a workgroup owns a packed run of consecutive cells (their CVs, HH CVs
// and synapses are contiguous in memory) and advances them through all K
// steps of the epoch with their state and constants held in LDS.
//
// Wavefronts take one of two roles for the whole epoch.  Solver wavefronts
// own a share of the cells' CVs: currents and assembly, the cable solve,
// the HH gates and spike detection.  Synapse wavefronts own a share of the
// cells' synapses: decay and plasticity, the protein trigger sum and p,
// the delivery of the next step's events and, in the mixed form, the next
// step's per-CV conductance sums.  The two chains of a step only meet
// through the synaptic conductance (double-buffered: step n reads one half
// while the synapse wavefronts write step n+1 into the other) and the
// post-synaptic flag (also double-buffered), so a step needs one workgroup
// barrier.  A 64-lane workgroup plays both roles in turn.
//
// The host part packs cells into workgroups under an LDS budget and picks
// the workgroup size, cells per workgroup and the split of roles by timing
// trial epochs (autotuning), then captures a graph of several epochs (fused
// step kernel, spike exchange) that the advance loop replays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/plasticarbor.h"
#include "device_common.hpp"
#include "sim.hpp"

namespace pa {

// Most rows per lane of the lanes' solve of unbranched cells (mixed form):
// a solver share of up to 64 CHAIN_ROWS CVs.
constexpr uint32_t CHAIN_ROWS = 4;

// LDS layout of a workgroup owning nv CVs, ns synapses, nh HH CVs, nc cells
// and ng branch segments for an epoch of at most K steps; gates,
// conductance, calcium and decay factors take tsize bytes (4 selects the
// mixed form).  The same arithmetic sizes the launch on the host and places
// the arrays on the device.
struct FusedLayout {
    // doubles
    uint32_t V, D, B, E, Ax, D0, Cdt, Gpe, DecCv, H, Z, Erev, P, Vold, Cu, Cb, HHp;
    // mixed form: per-CV conductance sums (two halves)
    uint32_t Gs, GsE;
    // particle diffusion: per CV both species, the volume, both species'
    // factors and a right-hand side; per synapse the change of |h - h0|;
    // per cell the soma threshold and synthesis amount
    uint32_t Sps, Prp, Dvol, SpsU, SpsF, SpsDp, PrpU, PrpF, PrpDp, Bx, Dlt, DThr, DPv;
    // T
    uint32_t G, C, Dec, M, HH, N;
    // 32-bit
    uint32_t Par, HHk, CvSyn, CvCl, Cb0, Cs0, Cg0, Ch0, Det, HHcv, EvN, EvOff, Scan;
    // events of the epoch, each slot's records sorted into delivery order
    uint32_t EvBuf, ev_cap;
    // incoming connections whose source spiked recently enough to matter
    // (offsets into the workgroup's connection range)
    uint32_t Act, act_cap;
    // 16-bit, 8-bit
    uint32_t SynCv, SegA, SegB, SegCell, KidOff, Kids, Kind, Post, SegLvl;
    uint32_t total;
    // lean: mixed-form workgroup of unbranched cells solved by the lanes
    // with the rows assembled in registers (no D, B); chain: the same with
    // more CVs than registers hold, a lane's chunk kept in D, B and E (each
    // 256 doubles beyond the CVs, room for every solver wavefront's
    // rounded-up share); carried: mixed form
    // with carried per-CV sums, so the synapse wavefronts alone read the
    // synapse conductances (one buffer), and the reversal potentials and
    // per-CV synapse ranges stay in global memory
    bool lean, chain, carried;
    __host__ __device__ FusedLayout(uint32_t nv, uint32_t ns, uint32_t nh, uint32_t nc, uint32_t K,
                                    uint32_t tsize, uint32_t ng, bool carried_sums, bool dif, uint32_t nq) {
        lean = tsize == 4 && ng == nc && nv <= 64 * CHAIN_ROWS;
        chain = tsize == 4 && ng == nc && !lean;
        carried = tsize == 4 && carried_sums;
        const uint32_t nvd = lean ? 0 : (chain ? nv + 256 : nv), nse = carried ? 0 : ns;
        uint32_t o = 0;
        auto take = [&](uint32_t bytes, uint32_t align) {
            o = (o + align - 1) / align * align;
            const uint32_t r = o;
            o += bytes;
            return r;
        };
        V = take(8 * nv, 16); D = take(8 * nvd, 8); B = take(8 * nvd, 8); E = take(8 * (chain ? nvd : 0), 8);
        Ax = take(8 * nv, 8);
        D0 = take(8 * nv, 8); Cdt = take(8 * nv, 8); Gpe = take(8 * nv, 8);
        DecCv = take(8 * (tsize == 4 ? nv : 0), 8);
        H = take(8 * ns, 8); Z = take(8 * ns, 8); Erev = take(8 * nse, 8);
        P = take(8 * nc, 8); Vold = take(8 * nc, 8);
        Cu = take(8 * ng, 8); Cb = take(8 * ng, 8); HHp = take(8 * 7 * nh, 8);
        const uint32_t nm = tsize == 4 ? nv : 0;
        Gs = take(16 * nm, 8); GsE = take(16 * nm, 8);
        const uint32_t nvf = dif ? nv : 0, nsf = dif ? ns : 0, ncf = dif ? nc : 0;
        Sps = take(8 * nvf, 8); Prp = take(8 * nvf, 8); Dvol = take(8 * nvf, 8);
        SpsU = take(8 * nvf, 8); SpsF = take(8 * nvf, 8); SpsDp = take(8 * nvf, 8);
        PrpU = take(8 * nvf, 8); PrpF = take(8 * nvf, 8); PrpDp = take(8 * nvf, 8);
        Bx = take(8 * nvf, 8); Dlt = take(8 * nsf, 8); DThr = take(8 * ncf, 8); DPv = take(8 * ncf, 8);
        G = take((carried ? 1 : 2) * tsize * ns, 8); C = take(tsize * ns, 8); Dec = take(tsize * ns, 8);
        M = take(tsize * nh, 8); HH = take(tsize * nh, 8); N = take(tsize * nh, 8);
        Par = take(4 * nv, 4); HHk = take(4 * nv, 4); CvSyn = take(carried ? 0 : 4 * (nv + 1), 4);
        CvCl = take(4 * (nv + 1), 4); Cb0 = take(4 * (nc + 1), 4); Cs0 = take(4 * (nc + 1), 4);
        Cg0 = take(4 * (nc + 1), 4); Ch0 = take(4 * (nc + 1), 4);
        Det = take(4 * nc, 4); HHcv = take(4 * nh, 4); EvN = take(4 * nc * K, 4);
        EvOff = take(4 * nc * K, 4); Scan = take(32, 4);
        act_cap = nq < 2048u ? nq : 2048u;
        Act = take(4 * act_cap, 4);
        ev_cap = 2 * nc * K + 32;
        EvBuf = take(32 * ev_cap, 16);
        SynCv = take(2 * ((tsize == 4 || dif) ? ns : 0), 2);
        SegA = take(2 * ng, 2); SegB = take(2 * ng, 2); SegCell = take(2 * ng, 2);
        KidOff = take(2 * (ng + 1), 2); Kids = take(2 * ng, 2);
        Kind = take(ns, 1); Post = take(2 * nc, 1); SegLvl = take(ng, 1);
        total = (o + 15) / 16 * 16;
    }
};


__device__ __forceinline__ uint32_t wave_max(uint32_t x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, off, 64));
    return x;
}

// Number of cells c < nc with off[c] < t (off increasing), over the lanes of
// one wavefront.
__device__ __forceinline__ uint32_t count_below(const uint32_t *off, uint32_t nc, uint32_t t, uint32_t lane) {
    uint32_t cnt = 0;
    for (uint32_t b = 0; b < nc; b += 64) {
        const uint32_t c = b + lane;
        cnt += (uint32_t)__popcll(__ballot(c < nc && off[c] < t));
    }
    return cnt;
}

// Cells [lo, hi) of part `part` of `parts` when the cells are split by the
// running count off[] (CVs or synapses) of total `tot`: a cell belongs to the
// part its first element falls in; the last part takes the rest.
__device__ __forceinline__ void split_cells(const uint32_t *off, uint32_t nc, uint32_t tot, uint32_t part,
                                            uint32_t parts, uint32_t lane, uint32_t &lo, uint32_t &hi) {
    lo = part == 0 ? 0u : count_below(off, nc, (uint32_t)((uint64_t)tot * part / parts), lane);
    hi = part + 1 == parts ? nc : count_below(off, nc, (uint32_t)((uint64_t)tot * (part + 1) / parts), lane);
}

// Value of x on lane l - 1 (wave_shr) or l + 1 (wave_shl) by a data-parallel
// lane shift of the whole wavefront; a lane without a source keeps its own.
template <int CTRL>
__device__ __forceinline__ double wave_shift1(double x) {
    const uint64_t u = __double_as_longlong(x);
    const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
    const int l2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
    const int h2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)h2 << 32) | (uint32_t)l2));
}
constexpr int DPP_WAVE_SHL1 = 0x130, DPP_WAVE_SHR1 = 0x138;

// Scales a row (lower coupling ra, diagonal rd, upper coupling rc,
// right-hand side rr) to unit diagonal.
__device__ __forceinline__ void pcr_unit(double rd, double &ra, double &rc, double &rr) {
    const double inv = qdiv<false>(1.0, rd);
    ra = ra * inv;
    rc = rc * inv;
    rr = rr * inv;
}

// One round of cyclic reduction across the lanes of a wavefront on rows of
// unit diagonal, lane l holding row l (lower coupling ra, upper coupling rc,
// right-hand side rr) of a tridiagonal system of n rows: the row subtracts
// ra times row l - sft and rc times row l + sft, read from their lanes, and
// is scaled back to unit diagonal.  A zero coupling marks the end of a
// cell, so rows never combine across cells.  The first round (sft = 1)
// reads its neighbours by lane shifts, the others by lane permutes.
__device__ __forceinline__ void pcr_round(uint32_t lane, uint32_t n, uint32_t sft, double &ra, double &rc,
                                          double &rr) {
    const bool act = lane < n;
    const bool hm = act && ra != 0.0 && lane >= sft;
    const bool hp = act && rc != 0.0 && lane + sft < n;
    double am, cm, rm, ap, cp, rp;
    if (sft == 1) {
        am = wave_shift1<DPP_WAVE_SHR1>(ra);
        cm = wave_shift1<DPP_WAVE_SHR1>(rc);
        rm = wave_shift1<DPP_WAVE_SHR1>(rr);
        ap = wave_shift1<DPP_WAVE_SHL1>(ra);
        cp = wave_shift1<DPP_WAVE_SHL1>(rc);
        rp = wave_shift1<DPP_WAVE_SHL1>(rr);
    } else {
        const int lm = (int)(hm ? lane - sft : lane), lp = (int)(hp ? lane + sft : lane);
        am = __shfl(ra, lm);
        cm = __shfl(rc, lm);
        rm = __shfl(rr, lm);
        ap = __shfl(ra, lp);
        cp = __shfl(rc, lp);
        rp = __shfl(rr, lp);
    }
    const double d1 = hm ? 1.0 - ra * cm : 1.0;
    const double r1 = hm ? rr - ra * rm : rr;
    const double dn = hp ? d1 - rc * ap : d1;
    const double rn = hp ? r1 - rc * rp : r1;
    const double an = hm ? -(ra * am) : 0.0;
    const double cn = hp ? -(rc * cp) : 0.0;
    ra = an;
    rc = cn;
    rr = rn;
    pcr_unit(dn, ra, rc, rr);
}

// Mixed-form parallel cyclic reduction of the tridiagonal systems of the
// unbranched cells whose CVs are [va, vb) (at most 64), CV va + l on lane
// l, in `levels` rounds; row(i, d, b) assembles CV i's diagonal and
// right-hand side.  Equal to the elimination up to rounding.  Writes V = x
// (after every row has read V).
template <class Row>
__device__ __forceinline__ bool pcr_cells(uint32_t va, uint32_t vb, uint32_t levels, uint32_t lane,
                                          const int32_t *par, const double *ax, Row &&row, double *V) {
    const uint32_t n = vb - va;
    const bool act = lane < n;
    const uint32_t i = act ? va + lane : va;
    const bool up = act && lane + 1 < n && par[i + 1] == (int32_t)i;
    double ra = act && par[i] >= 0 ? -ax[i] : 0.0;
    double rc = up ? -ax[i + 1] : 0.0;
    double rd = 1.0, rr = 0.0;
    if (act) row(i, rd, rr);
    pcr_unit(rd, ra, rc, rr);
    for (uint32_t k = 0, sft = 1; k < levels; ++k, sft <<= 1) pcr_round(lane, n, sft, ra, rc, rr);
    if (!act) return true;
    const double v = rr;
    V[i] = v;
    return isfinite(v);
}

// Mixed-form solve of the unbranched cells whose CVs are [va, vb) (at most
// 64 M) on one wavefront by the partition method: the range is cut into
// consecutive chunks of m = ceil(n / 64) rows, chunk l on lane l.  A lane
// first eliminates its chunk's lower couplings (each row then couples to
// the previous chunk's last CV instead of its predecessor), then its upper
// couplings (each row other than the last is expressed through the
// previous chunk's last CV and its own last CV).  The chunks' last CVs
// then obey a tridiagonal system with one row per lane (a row also takes
// in the next chunk's first row), solved by `levels` rounds of cyclic
// reduction across the lanes; the remaining CVs follow independently.
// Cell boundaries are zero couplings, so cells may share a chunk.  Equal to
// the elimination up to rounding.  Rows are assembled by row() as in
// pcr_cells.  Writes V = x (after every row has read V).
template <uint32_t M, class Row>
__device__ __forceinline__ bool part_cells(uint32_t va, uint32_t vb, uint32_t levels, uint32_t lane,
                                           const int32_t *par, const double *ax, Row &&row, double *V) {
    const uint32_t n = vb - va;
    const uint32_t m = (n + 63) >> 6;
    const uint32_t nact = (n + m - 1) / m;
    const uint32_t s = va + lane * m;
    const uint32_t cnt = lane < nact ? min(m, vb - s) : 0u;
    // row j of the chunk: A x_prev + (1 / Iv) x_j + Cc x_{j+1} = R
    double A[M], R[M], Iv[M], Cc[M];
    double ae = 0.0, re = 0.0, ce = 0.0, de = 1.0;  // the chunk's last row
#pragma unroll
    for (uint32_t j = 0; j < M; ++j) {
        if (j < cnt) {
            const uint32_t i = s + j;
            const double a = par[i] >= 0 ? -ax[i] : 0.0;
            const double c = i + 1 < vb && par[i + 1] == (int32_t)i ? -ax[i + 1] : 0.0;
            double aj = a, dj, rj;
            row(i, dj, rj);
            if (j > 0) {
                const double f = a * Iv[j - 1];
                aj = -f * A[j - 1];
                dj = dj - f * Cc[j - 1];
                rj = rj - f * R[j - 1];
            }
            A[j] = aj;
            R[j] = rj;
            Cc[j] = c;
            Iv[j] = qdiv<false>(1.0, dj);
            ae = aj;
            re = rj;
            ce = c;
            de = dj;
        }
    }
    // x_j = R - A x_prev - Cc x_last for the rows before the last; (rn, an,
    // cn) ends as the chunk's first row in that form (x_last itself when the
    // chunk has one row)
    double rn = 0.0, an = 0.0, cn = -1.0;
#pragma unroll
    for (int j = (int)M - 2; j >= 0; --j) {
        if ((uint32_t)j + 1 < cnt) {
            rn = (R[j] - Cc[j] * rn) * Iv[j];
            an = (A[j] - Cc[j] * an) * Iv[j];
            cn = -(Cc[j] * cn) * Iv[j];
            R[j] = rn;
            A[j] = an;
            Cc[j] = cn;
        }
    }
    // the last row with the next chunk's first row substituted
    const double rn1 = __shfl_down(rn, 1), an1 = __shfl_down(an, 1), cn1 = __shfl_down(cn, 1);
    const bool act = cnt > 0;
    double ra = act ? ae : 0.0;
    double rc = act ? -(ce * cn1) : 0.0;
    double rd = act ? de - ce * an1 : 1.0;
    double rr = act ? re - ce * rn1 : 0.0;
    pcr_unit(rd, ra, rc, rr);
    for (uint32_t k = 0, sft = 1; k < levels; ++k, sft <<= 1) pcr_round(lane, nact, sft, ra, rc, rr);
    const double xe = rr;
    const double xp0 = __shfl_up(xe, 1);
    const double xp = lane > 0 ? xp0 : 0.0;
    bool ok = !act || isfinite(xe);
#pragma unroll
    for (uint32_t j = 0; j < M; ++j) {
        if (j + 1 < cnt) {
            const double v = R[j] - A[j] * xp - Cc[j] * xe;
            V[s + j] = v;
            ok = ok && isfinite(v);
        } else if (j + 1 == cnt) {
            V[s + j] = xe;
        }
    }
    return ok;
}

// The partition method of part_cells for shares of unbranched cells too long
// for a lane's chunk to stay in registers: the same chunks and the same
// arithmetic in the same order (so the same values as part_cells would give
// for that chunking), with a chunk's rows kept in LDS scratch XA, XR, XI
// (row j of lane l at j * 64 + l, so every access of a wavefront is
// contiguous; each array holds 64 ceil(n / 64) doubles).  The rows are
// assembled first (independent of one another, so their loads overlap),
// then each pass over a chunk works through blocks of four rows whose
// operands are loaded before the block's dependent arithmetic.  XR, XI
// hold the assembled right-hand sides and diagonals, then the eliminated
// rows; XA the couplings to the previous chunk's last CV.  Writes V = x
// (after every row has read V).
template <class Row>
__device__ __forceinline__ bool part_chain(uint32_t va, uint32_t vb, uint32_t levels, uint32_t lane,
                                           const int32_t *par, const double *ax, Row &&row, double *V, double *XA,
                                           double *XR, double *XI) {
    const uint32_t n = vb - va;
    const uint32_t m = (n + 63) >> 6;
    const uint32_t nact = (n + m - 1) / m;
    const uint32_t s = va + lane * m;
    const uint32_t cnt = lane < nact ? min(m, vb - s) : 0u;
    // coupling of row i to its predecessor, and of row i to row i + 1
    auto lower = [&](uint32_t i) { return par[i] >= 0 ? -ax[i] : 0.0; };
    auto upper = [&](uint32_t i) { return i + 1 < vb && par[i + 1] == (int32_t)i ? -ax[i + 1] : 0.0; };
#pragma unroll 4
    for (uint32_t j = 0; j < cnt; ++j) {
        double dj, rj;
        row(s + j, dj, rj);
        XI[j * 64 + lane] = dj;
        XR[j * 64 + lane] = rj;
    }
    // lower couplings: row j becomes A x_prev + d x_j + C x_{j+1} = R with
    // 1 / d kept in XI
    double ap = 0.0, rp = 0.0, cp = 0.0, ivp = 0.0;
    double ae = 0.0, re = 0.0, ce = 0.0, de = 1.0;
    for (uint32_t j0 = 0; j0 < cnt; j0 += 4) {
        double a4[4], c4[4], d4[4], r4[4];
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            if (j0 + q < cnt) {
                const uint32_t i = s + j0 + q;
                a4[q] = lower(i);
                c4[q] = upper(i);
                d4[q] = XI[(j0 + q) * 64 + lane];
                r4[q] = XR[(j0 + q) * 64 + lane];
            }
        }
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            if (j0 + q < cnt) {
                const uint32_t j = j0 + q;
                double aj = a4[q], dj = d4[q], rj = r4[q];
                if (j > 0) {
                    const double f = a4[q] * ivp;
                    aj = -f * ap;
                    dj = dj - f * cp;
                    rj = rj - f * rp;
                }
                ivp = qdiv<false>(1.0, dj);
                XA[j * 64 + lane] = aj;
                XR[j * 64 + lane] = rj;
                XI[j * 64 + lane] = ivp;
                ap = aj;
                rp = rj;
                cp = c4[q];
                ae = aj;
                re = rj;
                ce = c4[q];
                de = dj;
            }
        }
    }
    // upper couplings, last row first: each row other than the chunk's
    // last becomes x_j = R - A x_prev - C x_last (C kept in XI)
    double rn = 0.0, an = 0.0, cn = -1.0;
    for (int j0 = (int)cnt - 2; j0 >= 0; j0 -= 4) {
        double c4[4], i4[4], r4[4], a4[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = j0 - q;
            if (j >= 0) {
                c4[q] = upper(s + (uint32_t)j);
                i4[q] = XI[j * 64 + lane];
                r4[q] = XR[j * 64 + lane];
                a4[q] = XA[j * 64 + lane];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = j0 - q;
            if (j >= 0) {
                rn = (r4[q] - c4[q] * rn) * i4[q];
                an = (a4[q] - c4[q] * an) * i4[q];
                cn = -(c4[q] * cn) * i4[q];
                XR[j * 64 + lane] = rn;
                XA[j * 64 + lane] = an;
                XI[j * 64 + lane] = cn;
            }
        }
    }
    const double rn1 = __shfl_down(rn, 1), an1 = __shfl_down(an, 1), cn1 = __shfl_down(cn, 1);
    const bool act = cnt > 0;
    double ra = act ? ae : 0.0;
    double rc = act ? -(ce * cn1) : 0.0;
    double rd = act ? de - ce * an1 : 1.0;
    double rr = act ? re - ce * rn1 : 0.0;
    pcr_unit(rd, ra, rc, rr);
    for (uint32_t k = 0, sft = 1; k < levels; ++k, sft <<= 1) pcr_round(lane, nact, sft, ra, rc, rr);
    const double xe = rr;
    const double xp0 = __shfl_up(xe, 1);
    const double xp = lane > 0 ? xp0 : 0.0;
    bool ok = !act || isfinite(xe);
#pragma unroll 4
    for (uint32_t j = 0; j < cnt; ++j) {
        if (j + 1 < cnt) {
            const double v = XR[j * 64 + lane] - XA[j * 64 + lane] * xp - XI[j * 64 + lane] * xe;
            V[s + j] = v;
            ok = ok && isfinite(v);
        } else {
            V[s + j] = xe;
        }
    }
    return ok;
}

// Barrier across all workgroups of a cooperative launch (all resident).
// Workgroup b counts itself into group counter b mod G (G = 32 counters on
// separate cache lines, so about nblocks/G workgroups contend for each);
// the workgroup that completes its group counts the group into a top
// counter, and the one that completes the top counter publishes the
// barrier's number in a release word, which the first wavefront of every
// workgroup polls (k-th barrier of the present plan: group counter at k
// times the group's size, top counter at k G; each workgroup keeps k in
// blk_done).  Everything other workgroups read after the barrier (event
// rings and counts) is written and read with device-coherent accesses, so
// no cache write-back or invalidation is needed; the count is ordered after
// this workgroup's writes by waiting for them to complete.  A wait that
// lasts about a second, or a barrier failure raised elsewhere, makes the
// workgroup give up (returns false) instead of hanging.
constexpr uint32_t BAR_GROUPS = 32, BAR_STRIDE = 32;  // counters 128 bytes apart
constexpr uint32_t BAR_TOP = BAR_GROUPS * BAR_STRIDE, BAR_RELEASE = BAR_TOP + BAR_STRIDE;

__device__ bool grid_sync(const DevNet &d, uint32_t nblocks, uint32_t *ok_word) {
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t lane = threadIdx.x;
        const uint32_t G = min(BAR_GROUPS, nblocks);
        // barriers this workgroup has passed with the present plan, this one
        // included
        const uint64_t k = ld_coh(d.blk_done + blockIdx.x) + 1;
        wave_sync();
        if (lane == 0) {
            st_coh(d.blk_done + blockIdx.x, k);
            const uint32_t g = blockIdx.x % G;
            const uint32_t size = nblocks / G + (g < nblocks % G ? 1u : 0u);
            const uint32_t before = __hip_atomic_fetch_add(d.bar_grp + g * BAR_STRIDE, 1u, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
            if ((uint64_t)before + 1 == k * size) {
                const uint32_t tb = __hip_atomic_fetch_add(d.bar_grp + BAR_TOP, 1u, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                if ((uint64_t)tb + 1 == k * G) st_coh(d.bar_grp + BAR_RELEASE, (uint32_t)k);
            }
        }
        uint32_t ok = 1, spins = 0;
        while ((uint64_t)ld_coh(d.bar_grp + BAR_RELEASE) < k) {
            // back off so that spinning wavefronts leave the issue slots of
            // their compute unit to workgroups still in the epoch
            if (spins < 256) __builtin_amdgcn_s_sleep(1);
            else if (spins < 1024) __builtin_amdgcn_s_sleep(4);
            else __builtin_amdgcn_s_sleep(16);
            if ((++spins & 255u) == 0 && (ld_coh(&d.ctr->flags) & FLAG_BARRIER)) {
                ok = 0;
                break;
            }
            if (spins == (1u << 21)) {
                if (lane == 0) raise_flag(d, FLAG_BARRIER, blockIdx.x);
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        if (lane == 0) *ok_word = ok;
    }
    __syncthreads();
    return *ok_word != 0;
}

// Steps of the cells blk[b] .. blk[b+1]-1 of workgroup b: one epoch of
// nsteps (<= K) steps, or, resident, nsteps steps in epochs of K (the last
// one shorter) with a grid barrier between epochs.  Mutable state of those
// cells (V, gates, g, c, h, z, p, post flag), their constants and the
// epoch's events live in LDS, so a step touches global memory only for
// spikes, clamps and rare noise keys.
#define PA_EPOCH_BOUNDS(BS_) __launch_bounds__(BS_)
// The incoming connections in [qa, qb) whose source's last spike is recent
// enough to bring events from step n0 on (its step at least n0 minus the
// connection's lag) are appended to act (offsets from qa) through the
// counter cnt; beyond cap only counted.  Each lane loads the operands of
// four connections before it tests any of them.
template <bool COH, uint32_t BS>
__device__ __forceinline__ void screen_conns(const DevNet &d, uint64_t qa, uint64_t qb, uint64_t n0, uint32_t tid,
                                             uint32_t *act, uint32_t cap, uint32_t *cnt) {
    for (uint64_t q0 = qa + tid; q0 < qb; q0 += 4 * BS) {
        uint32_t src[4], lag[4], last[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint64_t q = q0 + (uint64_t)j * BS;
            src[j] = q < qb ? d.in_src[q] : 0u;
            lag[j] = q < qb ? d.in_lag[q] : 0u;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) last[j] = (q0 + (uint64_t)j * BS < qb) ? ld_ring<COH>(d.spk_last + src[j]) : 0u;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (last[j] == 0 || (int64_t)last[j] - 1 < (int64_t)n0 - (int64_t)lag[j]) continue;
            const uint32_t pos = atomicAdd(cnt, 1u);
            if (pos < cap) act[pos] = (uint32_t)(q0 + (uint64_t)j * BS - qa);
        }
    }
}

template <class T, uint32_t BS>
__global__ PA_EPOCH_BOUNDS(BS) void k_epoch(DevNet d, const uint32_t *__restrict__ blk, uint32_t nsteps,
                                              uint32_t resident, uint32_t solver_waves) {
    extern __shared__ double lds[];
    uint8_t *L = (uint8_t *)lds;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    constexpr uint32_t NW = BS / 64;
    constexpr bool EXACT = sizeof(T) == 8;
    const uint32_t c0 = blk[blockIdx.x], c1 = blk[blockIdx.x + 1];
    const uint32_t ncb = c1 - c0;
    const uint32_t v0 = d.cv_off[c0], nv = d.cv_off[c1] - v0;
    const uint32_t s0 = d.syn_off[c0], ns = d.syn_off[c1] - s0;
    const uint32_t k0 = d.hh_off[c0], nhh = d.hh_off[c1] - k0;
    const uint32_t g0 = d.seg_off[c0], ng = d.seg_off[c1] - g0;
    const uint32_t K = d.K;
    // roles: wavefronts 0 .. SW-1 solve, SW .. NW-1 update synapses
    const uint32_t SW = NW == 1 ? 1u : min(max(solver_waves, 1u), NW - 1);
    const bool solver = wave < SW;
    const bool synw = NW == 1 || wave >= SW;
    // mixed form with one decay factor per CV: the per-CV conductance sums
    // are carried from step to step (decayed, plus each event's increment)
    // instead of being summed again
    const bool carry_sums = !EXACT && d.cv_dec_uniform != 0;
    const bool dif = d.dif != 0;
    const uint32_t nq = (uint32_t)(d.in_off[c1] - d.in_off[c0]);
    const FusedLayout lay(nv, ns, nhh, ncb, K, sizeof(T), ng, carry_sums, dif, nq);
    // offset of conductance half h (one buffer when the sums are carried)
    auto gofs = [&](uint32_t h) { return lay.carried ? 0u : h * ns; };
    double *sV = (double *)(L + lay.V), *sD = (double *)(L + lay.D), *sB = (double *)(L + lay.B);
    double *sE = (double *)(L + lay.E);
    double *sAx = (double *)(L + lay.Ax), *sD0 = (double *)(L + lay.D0), *sCdt = (double *)(L + lay.Cdt);
    double *sGpe = (double *)(L + lay.Gpe), *sH = (double *)(L + lay.H), *sZ = (double *)(L + lay.Z);
    double *sErev = (double *)(L + lay.Erev);
    double *sP = (double *)(L + lay.P), *sVold = (double *)(L + lay.Vold);
    double *sGs = (double *)(L + lay.Gs), *sGsE = (double *)(L + lay.GsE);
    double *sDecCv = (double *)(L + lay.DecCv);
    uint16_t *sSynCv = (uint16_t *)(L + lay.SynCv);
    T *sG = (T *)(L + lay.G), *sC = (T *)(L + lay.C), *sDec = (T *)(L + lay.Dec);
    T *sM = (T *)(L + lay.M), *sHH = (T *)(L + lay.HH), *sN = (T *)(L + lay.N);
    int32_t *sPar = (int32_t *)(L + lay.Par), *sHHk = (int32_t *)(L + lay.HHk);
    uint32_t *sCvSyn = (uint32_t *)(L + lay.CvSyn), *sCvCl = (uint32_t *)(L + lay.CvCl);
    uint32_t *sCb0 = (uint32_t *)(L + lay.Cb0), *sCs0 = (uint32_t *)(L + lay.Cs0);
    uint32_t *sCg0 = (uint32_t *)(L + lay.Cg0), *sCh0 = (uint32_t *)(L + lay.Ch0);
    uint32_t *sDet = (uint32_t *)(L + lay.Det), *sHHcv = (uint32_t *)(L + lay.HHcv);
    uint32_t *sEvN = (uint32_t *)(L + lay.EvN), *sEvOff = (uint32_t *)(L + lay.EvOff);
    uint32_t *sScan = (uint32_t *)(L + lay.Scan);
    uint32_t *sAct = (uint32_t *)(L + lay.Act);
    uint8_t *sKind = L + lay.Kind, *sPost = L + lay.Post, *sSegLvl = L + lay.SegLvl;
    double *sCu = (double *)(L + lay.Cu), *sCb = (double *)(L + lay.Cb), *sHHp = (double *)(L + lay.HHp);
    uint16_t *sSegA = (uint16_t *)(L + lay.SegA), *sSegB = (uint16_t *)(L + lay.SegB);
    uint16_t *sSegCell = (uint16_t *)(L + lay.SegCell), *sKidOff = (uint16_t *)(L + lay.KidOff);
    uint16_t *sKids = (uint16_t *)(L + lay.Kids);
    Event *sEv = (Event *)(L + lay.EvBuf);
    double *sSps = (double *)(L + lay.Sps), *sPrp = (double *)(L + lay.Prp), *sDvol = (double *)(L + lay.Dvol);
    double *sSpsU = (double *)(L + lay.SpsU), *sSpsF = (double *)(L + lay.SpsF), *sSpsDp = (double *)(L + lay.SpsDp);
    double *sPrpU = (double *)(L + lay.PrpU), *sPrpF = (double *)(L + lay.PrpF), *sPrpDp = (double *)(L + lay.PrpDp);
    double *sBx = (double *)(L + lay.Bx), *sDlt = (double *)(L + lay.Dlt);
    double *sDThr = (double *)(L + lay.DThr), *sDPv = (double *)(L + lay.DPv);
    // blocks whose cells are all unbranched (one segment per cell)
    const bool chains = (ng == ncb);
    const SynConst<T> sc{sErev, sDec, sKind, s0};
    const GateView<T> gv{sM, sHH, sN, k0};
    // first step of the launch; the resident form runs nsteps steps in
    // epochs of K, the single-epoch form one epoch of nsteps
    const uint64_t nbase = d.ctr->step;
    const bool multi = resident != 0;
    uint64_t n0 = nbase;
    // the epoch's events are in LDS, or, when they do not fit, in the
    // workgroup's queue in global memory
    Event *gEv = d.q_ev + d.q_off[c0];
    const uint64_t groom = d.q_off[c1] - d.q_off[c0];

    // ---- stage in: state, constants, this epoch's events
    for (uint32_t i = tid; i < nv; i += BS) {
        const uint32_t g = v0 + i;
        sV[i] = d.V[g];
        sAx[i] = d.axial[g];
        sD0[i] = d.d0[g];
        sCdt[i] = d.cdt[g];
        sGpe[i] = d.gpas_e[g];
        const int32_t p = d.parent[g];
        sPar[i] = p < 0 ? -1 : p - (int32_t)v0;
        sHHk[i] = d.hh_of[g];
        if (!lay.carried) sCvSyn[i] = d.cv_syn_off[g];
        sCvCl[i] = d.cv_cl_off[g];
        if constexpr (!EXACT) sDecCv[i] = d.cv_dec[g];
        if (lay.carried) {
            sGs[i] = d.gsum[g];
            sGsE[i] = d.gesum[g];
        }
        if (dif) {
            sSps[i] = d.sps[g];
            sPrp[i] = d.prp[g];
            sDvol[i] = d.dvol[g];
            sSpsU[i] = d.sps_u[g];
            sSpsF[i] = d.sps_f[g];
            sSpsDp[i] = d.sps_dp[g];
            sPrpU[i] = d.prp_u[g];
            sPrpF[i] = d.prp_f[g];
            sPrpDp[i] = d.prp_dp[g];
        }
        if (i == nv - 1) {
            if (!lay.carried) sCvSyn[nv] = d.cv_syn_off[g + 1];
            sCvCl[nv] = d.cv_cl_off[g + 1];
        }
    }
    for (uint32_t s = tid; s < ns; s += BS) {
        const uint32_t q = s0 + s;
        sG[s] = ((const T *)d.g)[q];
        sC[s] = ((const T *)d.c)[q];
        sH[s] = d.h[q];
        sZ[s] = d.z[q];
        if (!lay.carried) sErev[s] = d.syn_erev[q];
        if constexpr (EXACT) sDec[s] = (T)d.syn_decay[q];
        else sDec[s] = d.syn_decay_f[q];
        sKind[s] = d.syn_kind[q];
        if (!EXACT || dif) sSynCv[s] = (uint16_t)(d.syn_cv[q] - v0);
    }
    for (uint32_t k = tid; k < nhh; k += BS) {
        sM[k] = ((const T *)d.gm)[k0 + k];
        sHH[k] = ((const T *)d.gh)[k0 + k];
        sN[k] = ((const T *)d.gn)[k0 + k];
        sHHcv[k] = d.hh_cv[k0 + k] - v0;
        for (int j = 0; j < 6; ++j) sHHp[7 * k + j] = d.hh_par[6 * (size_t)(k0 + k) + j];
        sHHp[7 * k + 6] = d.hh_scale[k0 + k];
    }
    for (uint32_t c = tid; c <= ncb; c += BS) {
        sCb0[c] = d.cv_off[c0 + c] - v0;
        sCs0[c] = d.syn_off[c0 + c] - s0;
        sCg0[c] = d.seg_off[c0 + c] - g0;
        sCh0[c] = d.hh_off[c0 + c] - k0;
        if (c < ncb) {
            sP[c] = d.p[c0 + c];
            sPost[c] = d.post[c0 + c];
            sDet[c] = d.det_cv[c0 + c] - v0;
            if (dif) {
                sDThr[c] = d.dif_thr[c0 + c];
                sDPv[c] = d.dif_pv[c0 + c];
            }
        }
    }
    for (uint32_t g = tid; g < ng; g += BS) {
        sSegA[g] = (uint16_t)(d.seg_a[g0 + g] - v0);
        sSegB[g] = (uint16_t)(d.seg_b[g0 + g] - v0);
        sSegLvl[g] = d.seg_lvl[g0 + g];
        const uint32_t k0g = d.kid_off[g0];
        sKidOff[g] = (uint16_t)(d.kid_off[g0 + g] - k0g);
        if (g == ng - 1) sKidOff[ng] = (uint16_t)(d.kid_off[g0 + ng] - k0g);
        for (uint32_t q = d.kid_off[g0 + g]; q < d.kid_off[g0 + g + 1]; ++q) sKids[q - k0g] = (uint16_t)(d.kids[q] - g0);
    }
    for (uint32_t c = tid; c < ncb; c += BS)
        for (uint32_t g = d.seg_off[c0 + c]; g < d.seg_off[c0 + c + 1]; ++g) sSegCell[g - g0] = (uint16_t)c;
    __syncthreads();
    // the cells of this wavefront: a solver wavefront's share split by CV
    // count, a synapse wavefront's share split by synapse count
    uint32_t wc0 = 0, wc1 = 0, uc0 = 0, uc1 = 0;
    if (solver) split_cells(sCb0, ncb, nv, wave, SW, lane, wc0, wc1);
    if (synw) {
        const uint32_t nu = NW == 1 ? 1u : NW - SW, u = NW == 1 ? 0u : wave - SW;
        split_cells(sCs0, ncb, ns, u, nu, lane, uc0, uc1);
    }
    const uint32_t wva = sCb0[wc0], wvb = sCb0[wc1], wga = sCg0[wc0], wgb = sCg0[wc1];
    const uint32_t wha = sCh0[wc0], whb = sCh0[wc1];
    const uint32_t uva = sCb0[uc0], uvb = sCb0[uc1];
    // branch levels of the solver share, and cyclic-reduction steps for its
    // longest cell
    uint32_t wlev = 0, wlen = 1;
    for (uint32_t g = wga + lane; g < wgb; g += 64) wlev = max(wlev, (uint32_t)sSegLvl[g] + 1u);
    for (uint32_t c = wc0 + lane; c < wc1; c += 64) wlen = max(wlen, sCb0[c + 1] - sCb0[c]);
    wlev = wave_max(wlev);
    wlen = wave_max(wlen);
    // lanes' solve of unbranched cells (mixed form): rows per lane, and
    // reduction rounds for the most chunk ends one cell holds
    const uint32_t wrows = max(1u, (wvb - wva + 63) >> 6);
    const uint32_t wends = (wlen + wrows - 1) / wrows;
    uint32_t wpcr = 0;
    while ((1u << wpcr) < wends) ++wpcr;
    unsigned long long delivered = 0;

    // events of step index st (relative to n0) of the synapse share's cells
    // into conductance half gh (and, when carried, sum half `half`), in
    // delivery order
    auto deliver = [&](uint32_t st, T *gh, uint32_t half) {
        const SynView<T> sv{gh, sC, sH, sZ, s0};
        const bool inlds = sScan[3] == 0;
        for (uint32_t c = uc0 + lane; c < uc1; c += 64) {
            const uint32_t cnt = sEvN[c * K + st];
            if (!cnt) continue;
            const Event *ev = (inlds ? sEv : gEv) + sEvOff[c * K + st];
            for (uint32_t i = 0; i < cnt; ++i) {
                const Event e = ev[i];
                const uint32_t sy = e.syn;
                const T dg = apply_event<T>(d, sy, e.port, e.w, sv, sc);
                if (lay.carried && dg != T(0)) {
                    // the reversal potential: in the record's time field
                    // for an event staged in LDS, else from global memory
                    const double E = inlds ? e.t : d.syn_erev[sy];
                    const uint32_t cv = sSynCv[sy - s0];
                    sGs[half * nv + cv] += (double)dg;
                    sGsE[half * nv + cv] += (double)dg * E;
                }
            }
            delivered += cnt;
        }
    };
    // mixed form, sums not carried: summed conductance and conductance x
    // reversal potential of every CV of the synapse share, from conductance
    // half gh
    auto cv_sums = [&](const T *gh, uint32_t half) {
        for (uint32_t i = uva + lane; i < uvb; i += 64) {
            double gs = 0.0, ge = 0.0;
            for (uint32_t q = sCvSyn[i] - s0; q < sCvSyn[i + 1] - s0; ++q) {
                const double g = (double)gh[q];
                gs += g;
                ge += g * sErev[q];
            }
            sGs[half * nv + i] = gs;
            sGsE[half * nv + i] = ge;
        }
    };

    const uint32_t n_total = nsteps;
    for (uint32_t done = 0; done < n_total;) {
    n0 = nbase + done;
    const uint32_t nst = multi ? min(K, n_total - done) : nsteps;
    // ---- the epoch's events of the workgroup's cells: a counting pass over
    // their incoming connections, trains and Poisson sources (count per
    // (cell, step) slot), a prefix sum over the slots, a scatter pass into
    // LDS (or, if they do not fit, the workgroup's queue in global memory),
    // then each slot sorted into delivery order (one lane per slot); the
    // delivery statistics are counted there
    const uint32_t nslot = ncb * nst;
    for (uint32_t x = tid; x < nslot; x += BS) {
        const uint32_t c = x / nst, st = x - c * nst;
        sEvN[c * K + st] = 0;
    }
    __syncthreads();
    const uint64_t qa = d.in_off[c0], qb = d.in_off[c1];
    const uint32_t ta = d.tr_cell_off[c0], tb = d.tr_cell_off[c1];
    const uint32_t pa = d.po_cell_off[c0], pb = d.po_cell_off[c1];
    // screening: the incoming connections whose source spiked recently
    // enough to matter, listed once (their loads issued four at a time), so
    // that the counting and scatter passes visit only those
    if (tid == 0) sScan[4] = 0;
    __syncthreads();
    if (multi) screen_conns<true, BS>(d, qa, qb, n0, tid, sAct, lay.act_cap, sScan + 4);
    else screen_conns<false, BS>(d, qa, qb, n0, tid, sAct, lay.act_cap, sScan + 4);
    __syncthreads();
    const uint32_t nact = sScan[4];
    const bool act_ok = nact <= lay.act_cap;
    // visits fn(q) for every incoming connection that can bring an event
    auto each_conn = [&](auto &&fn) {
        if (act_ok)
            for (uint32_t i = tid; i < nact; i += BS) fn(qa + sAct[i]);
        else
            for (uint64_t q = qa + tid; q < qb; q += BS) fn(q);
    };
    {
        auto count = [&](uint32_t st, const Event &e) { atomicAdd(&sEvN[(d.syn_cell[e.syn] - c0) * K + st], 1u); };
        if (multi) each_conn([&](uint64_t q) { conn_events<true>(d, q, n0, nst, count); });
        else each_conn([&](uint64_t q) { conn_events<false>(d, q, n0, nst, count); });
        for (uint32_t x = ta + tid; x < tb; x += BS) train_events(d, d.tr_by_cell[x], n0, nst, false, count);
        for (uint32_t x = pa + tid; x < pb; x += BS) poisson_events(d, d.po_by_cell[x], n0, nst, false, count);
    }
    __syncthreads();
    if (wave == 0) {
        uint32_t base = 0;
        for (uint32_t x0 = 0; x0 < nslot; x0 += 64) {
            const uint32_t x = x0 + lane;
            const uint32_t c = x / nst, st = x - c * nst;
            const uint32_t v = x < nslot ? sEvN[c * K + st] : 0u;
            const uint32_t inc = wave_incl_scan(v, lane);
            if (x < nslot) sEvOff[c * K + st] = base + inc - v;
            base += (uint32_t)__shfl((int)inc, 63, 64);
        }
        if (lane == 0) {
            sScan[1] = base;
            sScan[3] = base > lay.ev_cap ? 1u : 0u;
            if (base > lay.ev_cap && base > groom) raise_flag(d, FLAG_QUEUE, c0);
        }
    }
    __syncthreads();
    const bool evlds = sScan[3] == 0;
    const uint64_t room = evlds ? lay.ev_cap : groom;
    Event *evb = evlds ? sEv : gEv;
    {
        auto place = [&](uint32_t st, const Event &e) {
            const uint32_t pos = atomicAdd(&sEvOff[(d.syn_cell[e.syn] - c0) * K + st], 1u);
            if (pos < room) evb[pos] = e;
        };
        if (multi) each_conn([&](uint64_t q) { conn_events<true>(d, q, n0, nst, place); });
        else each_conn([&](uint64_t q) { conn_events<false>(d, q, n0, nst, place); });
        for (uint32_t x = ta + tid; x < tb; x += BS) train_events(d, d.tr_by_cell[x], n0, nst, true, place);
        for (uint32_t x = pa + tid; x < pb; x += BS) poisson_events(d, d.po_by_cell[x], n0, nst, true, place);
    }
    __syncthreads();
    for (uint32_t x = tid; x < nslot; x += BS) {
        const uint32_t c = x / nst, st = x - c * nst;
        const uint32_t cnt = sEvN[c * K + st];
        const uint32_t off = sEvOff[c * K + st] - cnt;
        const uint32_t m = off >= room ? 0u : (uint32_t)min<uint64_t>(cnt, room - off);
        sEvN[c * K + st] = m;
        sEvOff[c * K + st] = off;
        if (!m) continue;
        Event *ev = evb + off;
        sort_slot(ev, m);
        for (uint32_t i = 0; i < m; ++i) {
            const Event e = ev[i];
            atomicAdd(&d.ev_cnt[2 * e.syn + e.port - 1], 1ull);
            atomicAdd(&d.ev_sum[2 * e.syn + e.port - 1], (unsigned long long)(n0 + st));
            // once sorted, a record's time field in LDS carries the
            // target's reversal potential for the carried sums
            if (lay.carried && evlds) ev[i].t = d.syn_erev[e.syn];
        }
    }
    __syncthreads();

    // the first step's events, and its conductance sums (carried sums
    // enter the epoch already decayed to this step)
    {
        const uint32_t h0 = (uint32_t)(n0 - nbase) & 1u;
        if (synw) {
            deliver(0, sG + gofs(h0), h0);
            if (!EXACT && !lay.carried) {
                wave_sync();
                cv_sums(sG + gofs(h0), h0);
            }
        }
    }
    __syncthreads();

    // one step of each role (n = n0 + st); the roles run in separate loops
    // so that each loop keeps only its own role's values live
    auto solver_step = [&](uint32_t st) {
        const uint64_t n = n0 + st;
        const double tn = (double)n * d.dt;
        const uint32_t cur = (uint32_t)(n - nbase) & 1u, nxt = cur ^ 1u;
        T *gc = sG + gofs(cur);
        uint8_t *postn = sPost + nxt * ncb;
        // currents at V^n and the diagonal and right-hand side of CV i
        const SynView<T> svc{gc, sC, sH, sZ, s0};
        auto row = [&](uint32_t i, double &Di, double &Bi) {
            const double v = sV[i];
            double I, G;
            const int32_t hk = sHHk[i];
            const double *P = hk >= 0 ? sHHp + 7 * (hk - (int32_t)k0) : nullptr;
            if constexpr (EXACT)
                cv_current<T>(d, hk, P, hk >= 0 ? P[6] : 0.0, v, tn, gv, svc, sc, sCvSyn[i], sCvSyn[i + 1],
                              sCvCl[i], sCvCl[i + 1], I, G);
            else
                cv_current_sums<T>(d, hk, P, hk >= 0 ? P[6] : 0.0, v, tn, gv, sGs[cur * nv + i],
                                   sGsE[cur * nv + i], sCvCl[i], sCvCl[i + 1], I, G);
            Di = sD0[i] + G;
            Bi = ((sCdt[i] * v + sGpe[i]) - I) + G * v;
        };
        for (uint32_t c = wc0 + lane; c < wc1; c += 64) sVold[c] = sV[sDet[c]];
        if (!lay.lean && !lay.chain) {
            for (uint32_t i = wva + lane; i < wvb; i += 64) row(i, sD[i], sB[i]);
        }
        wave_sync();
        // the cable solve of the share's cells
        if (wva == wvb) {
            // no cells of this share
        } else if (lay.lean) {
            // unbranched cells, mixed form: the lanes assemble the rows and
            // solve by cyclic reduction or the partition method
            const bool ok = wvb - wva <= 64 ? pcr_cells(wva, wvb, wpcr, lane, sPar, sAx, row, sV)
                                            : part_cells<CHAIN_ROWS>(wva, wvb, wpcr, lane, sPar, sAx, row, sV);
            if (!ok) raise_flag(d, FLAG_NONFINITE, c0 + wc0);
        } else if (lay.chain) {
            // the same, a chunk's rows in LDS (this wavefront's scratch
            // starts 64 doubles per solver wavefront beyond its share)
            const uint32_t xb = wva + 64 * wave;
            const bool ok = wvb - wva <= 64 ? pcr_cells(wva, wvb, wpcr, lane, sPar, sAx, row, sV)
                                            : part_chain(wva, wvb, wpcr, lane, sPar, sAx, row, sV, sE + xb,
                                                         sB + xb, sD + xb);
            if (!ok) raise_flag(d, FLAG_NONFINITE, c0 + wc0);
        } else {
            // Hines elimination level-scheduled over branch segments,
            // deepest level first; a branch point takes its children's
            // contributions in descending child order, as in the
            // sequential elimination
            for (int lv = (int)wlev - 1; lv >= 0; --lv) {
                for (uint32_t g = wga + lane; g < wgb; g += 64) {
                    if (sSegLvl[g] != (uint32_t)lv) continue;
                    const uint32_t a = sSegA[g], b = sSegB[g];
                    double dc = sD[b], bc = sB[b];
                    for (uint32_t q = sKidOff[g]; q < sKidOff[g + 1]; ++q) {
                        const uint32_t kd = sKids[q];
                        dc -= sCu[kd];
                        bc -= sCb[kd];
                    }
                    seg_backward<EXACT>(sD, sB, sAx, a, b, dc, bc);
                    if (sPar[a] >= 0) {
                        const double u = -sAx[a];
                        const double f = qdiv<EXACT>(u, dc);
                        sCu[g] = f * u;
                        sCb[g] = f * bc;
                    }
                }
                wave_sync();
            }
            for (uint32_t lv = 0; lv < wlev; ++lv) {
                for (uint32_t g = wga + lane; g < wgb; g += 64) {
                    if (sSegLvl[g] != lv) continue;
                    const uint32_t a = sSegA[g], b = sSegB[g];
                    const int32_t p = sPar[a];
                    sV[a] = (p < 0) ? qdiv<EXACT>(sB[a], sD[a]) : qdiv<EXACT>(sB[a] - (-sAx[a]) * sV[p], sD[a]);
                    if (!seg_forward<EXACT>(sD, sB, sV, sAx, a, b)) raise_flag(d, FLAG_NONFINITE, c0 + sSegCell[g]);
                }
                wave_sync();
            }
        }
        wave_sync();
        // HH gates at V^{n+1}, one lane per gate (the three gates of a
        // CV are independent), and threshold detection
        for (uint32_t t = lane; t < 3 * (whb - wha); t += 64) {
            const uint32_t k = wha + t / 3, j = t % 3;
            T *x = j == 0 ? sM + k : (j == 1 ? sHH + k : sN + k);
            *x = gate_next<T>(*x, (T)sV[sHHcv[k]], (T)d.dt, (int)j);
        }
        for (uint32_t c = wc0 + lane; c < wc1; c += 64) {
            const double v0 = sVold[c], v1 = sV[sDet[c]];
            const bool fired = crossed(d, v0, v1);
            if (fired) record_spike(d, c0 + c, n, spike_time(d, n, v0, v1));
            postn[c] = fired ? 1 : 0;
        }
        };
    auto synapse_step = [&](uint32_t st) {
        const uint64_t n = n0 + st;
        const uint32_t cur = (uint32_t)(n - nbase) & 1u, nxt = cur ^ 1u;
        T *gc = sG + gofs(cur), *gn = sG + gofs(nxt);
        uint8_t *postc = sPost + cur * ncb;
        // synapse updates of step n (from step-start values) with the
        // cell's protein trigger sum: lane l sums the cell's synapses
        // l, l+64, ..., then a fixed lane-shift tree; then p of the cell
        const SynView<T> svc{gc, sC, sH, sZ, s0};
        for (uint32_t c = uc0; c < uc1; ++c) {
            const uint32_t a = sCs0[c], e = sCs0[c + 1];
            const double p = sP[c];
            const bool post = postc[c] != 0;
            double S = 0.0;
            // two synapses per lane and pass, their arithmetic interleaved
            for (uint32_t s = a + lane; s < e; s += 128) {
                const bool two = s + 64 < e;
                const uint32_t s2 = two ? s + 64 : s;
                const SynIn<T> x1{gc[s], sDec[s], sC[s], sH[s], sZ[s]};
                const SynIn<T> x2{gc[s2], sDec[s2], sC[s2], sH[s2], sZ[s2]};
                const uint8_t kd1 = sKind[s], kd2 = sKind[s2];
                const bool k1 = kd1 == 1, k2 = kd2 == 1;
                // with diffusion, z takes the protein of the synapse's CV
                const double p1 = dif ? sPrp[sSynCv[s]] : p, p2 = dif ? sPrp[sSynCv[s2]] : p;
                // 256-lane workgroups draw both synapses' noise in one call,
                // the ids that key it requested before the update so that its
                // arithmetic covers the loads' latency; the smaller
                // workgroups keep a call per synapse, which measured faster
                // on networks whose synapses rarely draw noise
                constexpr bool pairs = sizeof(T) == 4 && BS == 256;
                bool dr1 = false, dr2 = false;
                uint32_t id1 = 0, id2 = 0;
                if constexpr (pairs) {
                    dr1 = k1 && syn_draws<T>(d.stc, post, x1.c);
                    dr2 = two && k2 && syn_draws<T>(d.stc, post, x2.c);
                    if (dr1 || dr2) {
                        id1 = d.syn_sid[s0 + s];
                        id2 = d.syn_sid[s0 + s2];
                    }
                }
                SynOut<T> o1, o2;
                syn_compute2<T>(d, p1, p2, post, x1, x2, o1, o2);
                if constexpr (pairs) {
                    if (dr1 || dr2) {
                        const NoisePair r = noise_increment2_f32(d.seed, id1, id2, n, d.stc.sigma_pl, o1.th, o2.th,
                                                                 d.dt / d.stc.tau_h);
                        if (dr1) o1.h += r.a;
                        if (dr2) o2.h += r.b;
                    }
                } else {
                    if (k1) syn_noise<T>(d, s0 + s, n, o1);
                    if (two && k2) syn_noise<T>(d, s0 + s2, n, o2);
                }
                if (kd1 == 2) stdp_compute<T>(d, post, x1, o1);
                if (kd2 == 2) stdp_compute<T>(d, post, x2, o2);
                if (dif) {
                    sDlt[s] = k1 ? fabs(o1.h - d.stc.h0) - o1.absdh : 0.0;
                    if (two) sDlt[s2] = k2 ? fabs(o2.h - d.stc.h0) - o2.absdh : 0.0;
                }
                S += syn_store<T>(svc, s, kd1 != 0, o1, gn);
                if (two) S += syn_store<T>(svc, s2, kd2 != 0, o2, gn);
            }
            if (!dif) {
                S = wave_sum(S);
                if (lane == 0) sP[c] = prp_next(d, p, S);
            }
        }
        if (dif) {
            // both diffusing species of the share's cells, one lane per
            // cell: the trigger from the step-start SPS at the soma, the
            // release per CV (its plastic synapses in (CV, id) order), the
            // SPS sweep, then the protein's decay, synthesis and sweep
            wave_sync();
            for (uint32_t c = uc0 + lane; c < uc1; c += 64) {
                const uint32_t b0 = sCb0[c], b1 = sCb0[c + 1], soma = sDet[c];
                const double trig = (sSps[soma] - sDThr[c] > 0.0) ? 1.0 : 0.0;
                for (uint32_t i = b0; i < b1; ++i) sBx[i] = 0.0;
                for (uint32_t q = sCs0[c]; q < sCs0[c + 1]; ++q)
                    if (sKind[q] == 1) sBx[sSynCv[q]] += sDlt[q];
                for (uint32_t i = b0; i < b1; ++i) sBx[i] = sDvol[i] * sSps[i] + sBx[i];
                species_sweep(sBx, sSps, sPar, sSpsF, sSpsU, sSpsDp, b0, b1);
                const double ap = d.dt / d.stc.tau_p;
                for (uint32_t i = b0; i < b1; ++i) {
                    const double x = sPrp[i];
                    sBx[i] = sDvol[i] * (x + ap * (-x));
                }
                sBx[soma] += ap * sDPv[c] * trig;
                species_sweep(sBx, sPrp, sPar, sPrpF, sPrpU, sPrpDp, b0, b1);
            }
        }
        // carried sums decay to the next step also after an epoch's last
        // step (the next epoch, or launch, starts from them)
        if (lay.carried) {
            for (uint32_t i = uva + lane; i < uvb; i += 64) {
                sGs[nxt * nv + i] = sGs[cur * nv + i] * sDecCv[i];
                sGsE[nxt * nv + i] = sGsE[cur * nv + i] * sDecCv[i];
            }
        }
        if (st + 1 < nst) {
            wave_sync();
            deliver(st + 1, gn, nxt);
            if (!EXACT && !lay.carried) {
                wave_sync();
                cv_sums(gn, nxt);
            }
        }
    };
    // halves of the double buffers alternate over the steps of the launch
    if (NW == 1) {
        for (uint32_t st = 0; st < nst; ++st) {
            solver_step(st);
            synapse_step(st);
            __syncthreads();
        }
    } else if (solver) {
        for (uint32_t st = 0; st < nst; ++st) {
            solver_step(st);
            __syncthreads();
        }
    } else {
        for (uint32_t st = 0; st < nst; ++st) {
            synapse_step(st);
            __syncthreads();
        }
    }
    done += nst;
    if (multi && done < n_total) {
        // the epoch's spikes are in their cells' rings; every workgroup
        // waits for all the others before the next epoch gathers from them
        const bool ok = grid_sync(d, gridDim.x, sScan + 2);
        if (!ok) break;
    }
    }
    // ---- stage out
    const uint32_t hfin = n_total & 1u;
    const T *gfin = sG + gofs(hfin);
    const uint8_t *pfin = sPost + hfin * ncb;
    for (uint32_t i = tid; i < nv; i += BS) {
        d.V[v0 + i] = sV[i];
        if (lay.carried) {
            d.gsum[v0 + i] = sGs[hfin * nv + i];
            d.gesum[v0 + i] = sGsE[hfin * nv + i];
        }
        if (dif) {
            d.sps[v0 + i] = sSps[i];
            d.prp[v0 + i] = sPrp[i];
        }
    }
    for (uint32_t s = tid; s < ns; s += BS) {
        ((T *)d.g)[s0 + s] = gfin[s];
        ((T *)d.c)[s0 + s] = sC[s];
        d.h[s0 + s] = sH[s];
        d.z[s0 + s] = sZ[s];
    }
    for (uint32_t k = tid; k < nhh; k += BS) {
        ((T *)d.gm)[k0 + k] = sM[k];
        ((T *)d.gh)[k0 + k] = sHH[k];
        ((T *)d.gn)[k0 + k] = sN[k];
    }
    for (uint32_t c = tid; c < ncb; c += BS) {
        d.p[c0 + c] = sP[c];
        d.post[c0 + c] = pfin[c];
    }
    if (delivered) atomicAdd((unsigned long long *)&d.ctr->events, delivered);
    // close the launch: the resident form's first workgroup moves the epoch
    // counter past its steps (every workgroup read it at its start); in the
    // single-epoch form the last workgroup to finish does
    if (multi) {
        if (blockIdx.x == 0 && tid == 0) d.ctr->step = nbase + n_total;
    } else {
        __syncthreads();
        if (tid == 0) {
            __threadfence();
            const uint32_t prev = atomicAdd(&d.ctr->blocks_done, 1u);
            if (prev == gridDim.x - 1) {
                d.ctr->blocks_done = 0;
                d.ctr->step = nbase + n_total;
                __threadfence();
            }
        }
    }
}

// Carried per-CV sums from the conductances (mixed form), one lane per CV,
// in synapse order.
__global__ void k_carried_sums(DevNet d) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.n_cv) return;
    const float *g = (const float *)d.g;
    double gs = 0.0, ge = 0.0;
    for (uint32_t q = d.cv_syn_off[i]; q < d.cv_syn_off[i + 1]; ++q) {
        gs += (double)g[q];
        ge += (double)g[q] * d.syn_erev[q];
    }
    d.gsum[i] = gs;
    d.gesum[i] = ge;
}

int launch_carried_sums(const DevNet &d, void *stream) {
    if (!d.gsum || d.n_cv == 0) return 0;
    hipLaunchKernelGGL(k_carried_sums, dim3((d.n_cv + 255) / 256), dim3(256), 0, (hipStream_t)stream, d);
    return (int)hipGetLastError();
}

template <class T, uint32_t BS>
static int launch_fused_t(const DevNet &d, uint32_t nsteps, uint32_t resident, const uint32_t *blk, uint32_t n_blocks,
                          size_t lds_bytes, uint32_t solver_waves, hipStream_t s) {
    if (!resident) {
        hipLaunchKernelGGL((k_epoch<T, BS>), dim3(n_blocks), dim3(BS), lds_bytes, s, d, blk, nsteps, 0u, solver_waves);
        return (int)hipGetLastError();
    }
    // all workgroups must be resident for the grid barrier: a cooperative
    // launch guarantees it or fails
    DevNet dc = d;
    const uint32_t *b = blk;
    uint32_t a_ns = nsteps, a_res = 1u, a_sw = solver_waves;
    void *args[] = {&dc, &b, &a_ns, &a_res, &a_sw};
    return (int)hipLaunchCooperativeKernel((const void *)k_epoch<T, BS>, dim3(n_blocks), dim3(BS), args,
                                           (unsigned)lds_bytes, s);
}

int launch_epoch_fused(const DevNet &d, uint32_t nsteps, uint32_t resident, const uint32_t *blk, uint32_t n_blocks,
                       size_t lds_bytes, uint32_t block_threads, uint32_t solver_waves, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (block_threads) {
    case 64: return d.mixed ? launch_fused_t<float, 64>(d, nsteps, resident, blk, n_blocks, lds_bytes, solver_waves, s)
                            : launch_fused_t<double, 64>(d, nsteps, resident, blk, n_blocks, lds_bytes, solver_waves, s);
    case 128: return d.mixed ? launch_fused_t<float, 128>(d, nsteps, resident, blk, n_blocks, lds_bytes, solver_waves, s)
                             : launch_fused_t<double, 128>(d, nsteps, resident, blk, n_blocks, lds_bytes, solver_waves, s);
    case 256: return d.mixed ? launch_fused_t<float, 256>(d, nsteps, resident, blk, n_blocks, lds_bytes, solver_waves, s)
                             : launch_fused_t<double, 256>(d, nsteps, resident, blk, n_blocks, lds_bytes, solver_waves, s);
    default: return (int)hipErrorInvalidValue;
    }
}

template <class T, uint32_t BS>
static uint32_t capacity_t(size_t lds_bytes) {
    int dev = 0, coop = 0, cus = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_epoch<T, BS>, (int)BS, lds_bytes) != hipSuccess)
        return 0;
    return (uint32_t)(nb * cus);
}

uint32_t epoch_fused_capacity(bool mixed, uint32_t block_threads, size_t lds_bytes) {
    switch (block_threads) {
    case 64: return mixed ? capacity_t<float, 64>(lds_bytes) : capacity_t<double, 64>(lds_bytes);
    case 128: return mixed ? capacity_t<float, 128>(lds_bytes) : capacity_t<double, 128>(lds_bytes);
    case 256: return mixed ? capacity_t<float, 256>(lds_bytes) : capacity_t<double, 256>(lds_bytes);
    default: return 0;
    }
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
    uint32_t threads = 256;
    uint32_t solver_waves = 1;
    bool multi = false;         // whole epochs in one cooperative launch
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t graph_epochs = 0;
};

BatchedPlan *&pa_plan(pa_sim *s);

namespace {

constexpr size_t LDS_MAX = 160 * 1024;

struct Offsets {
    std::vector<uint32_t> cv, syn, hh, seg;
    std::vector<uint64_t> in;  // incoming connections per cell (offsets)
    uint32_t tsize, K;
    bool carried;  // mixed form with carried per-CV sums
    bool dif;      // particle diffusion
};

// Packs consecutive cells, at most cpb per workgroup, within an LDS budget
// that leaves room for at least two resident workgroups per CU (160 KB of
// LDS); the autotuned cells per workgroup then choose between more, smaller
// workgroups and fewer, larger ones.
bool pack(const Offsets &o, uint32_t cpb, uint32_t threads, std::vector<uint32_t> &blk, size_t &lds) {
    const size_t budget = threads == 64 ? 32 * 1024 : 80 * 1024;
    const uint32_t nc = (uint32_t)o.cv.size() - 1;
    auto bytes = [&](uint32_t a, uint32_t e) {
        return (size_t)FusedLayout(o.cv[e] - o.cv[a], o.syn[e] - o.syn[a], o.hh[e] - o.hh[a], e - a, o.K,
                                   o.tsize, o.seg[e] - o.seg[a], o.carried, o.dif,
                                   (uint32_t)(o.in[e] - o.in[a])).total;
    };
    blk.assign(1, 0);
    lds = 0;
    uint32_t c = 0;
    while (c < nc) {
        uint32_t e = c + 1;
        size_t b = bytes(c, e);
        if (b > LDS_MAX) return false;
        while (e < nc && e - c < cpb && e - c < 65535) {
            size_t b2 = bytes(c, e + 1);
            if (b2 > budget) break;
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
    int r = 0;
    if (e0) (void)hipEventRecord(e0, st);
    r |= launch_epoch_fused(d, nsteps, 0u, P.d_blk, (uint32_t)P.blk.size() - 1, P.lds, P.threads, P.solver_waves, st);
    if (e1) (void)hipEventRecord(e1, st);
    return r;
}

int enqueue_resident(const DevNet &d, const BatchedPlan &P, uint32_t nsteps, hipStream_t st, hipEvent_t e0,
                     hipEvent_t e1) {
    int r = 0;
    if (e0) (void)hipEventRecord(e0, st);
    r |= launch_epoch_fused(d, nsteps, 1u, P.d_blk, (uint32_t)P.blk.size() - 1, P.lds, P.threads, P.solver_waves,
                            st);
    if (e1) (void)hipEventRecord(e1, st);
    return r;
}

}  // namespace

pa_status batched_setup(pa_sim *s) {
    DevNet &d = pa_devnet(s);
    hipStream_t st = pa_stream(s);
    BatchedPlan *&plan = pa_plan(s);
    plan = new BatchedPlan();
    // host copies of the offsets for packing
    Offsets o;
    o.cv.resize(d.n_cells + 1);
    o.syn.resize(d.n_cells + 1);
    o.hh.resize(d.n_cells + 1);
    o.tsize = d.mixed ? 4 : 8;
    o.K = d.K;
    o.dif = d.dif != 0;
    o.carried = d.mixed && d.cv_dec_uniform;
    o.seg.resize(d.n_cells + 1);
    o.in.resize(d.n_cells + 1);
    if (hipMemcpy(o.in.data(), d.in_off, o.in.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(o.seg.data(), d.seg_off, o.seg.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(o.cv.data(), d.cv_off, o.cv.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(o.syn.data(), d.syn_off, o.syn.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(o.hh.data(), d.hh_off, o.hh.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return pa_fail(s, PA_EDEVICE, "offsets");
    // candidates: workgroup size, cells per workgroup, and how many of its
    // wavefronts solve (the others update synapses; a 64-lane workgroup does
    // both in turn); the caller may fix any of the three
    struct Cand { uint32_t threads, cpb, sw; };
    std::vector<Cand> cands;
    {
        const pa_config &cf = pa_cfg(s);
        std::vector<Cand> all;
        for (uint32_t c : {1u, 2u, 4u}) all.push_back({64u, c, 1u});
        for (uint32_t c : {1u, 2u, 4u, 8u}) all.push_back({128u, c, 1u});
        for (uint32_t c : {2u, 4u, 8u, 16u, 32u})
            for (uint32_t w : {1u, 2u, 3u}) all.push_back({256u, c, w});
        for (Cand cd : all) {
            if (cf.block_threads && cd.threads != cf.block_threads) continue;
            if (cf.solver_waves && cd.threads > 64 && cd.sw != cf.solver_waves) continue;
            if (cf.cells_per_block) {
                cd.cpb = cf.cells_per_block;
                bool dup = false;
                for (const Cand &e : cands) dup |= e.threads == cd.threads && e.sw == cd.sw;
                if (dup) continue;
            }
            cands.push_back(cd);
        }
        if (cands.empty()) return pa_fail(s, PA_EINVAL, "no workgroup shape matches the configuration");
    }
    // each shape is tried with a separate exchange kernel per epoch and, if
    // all its workgroups fit on the device at once, resident over several
    // epochs per launch
    const uint32_t xmode = pa_cfg(s).exchange;
    struct Trial { Cand c; bool multi; };
    std::vector<Trial> trials;
    std::vector<BatchedPlan> packed;
    for (const Cand &cd : cands) {
        BatchedPlan P;
        P.threads = cd.threads;
        P.solver_waves = cd.sw;
        if (!pack(o, cd.cpb, cd.threads, P.blk, P.lds)) continue;
        const bool fits = epoch_fused_capacity(d.mixed != 0, cd.threads, P.lds) >= P.blk.size() - 1;
        if (xmode != PA_EXCHANGE_RESIDENT) trials.push_back({cd, false});
        if (xmode != PA_EXCHANGE_KERNEL && fits) trials.push_back({cd, true});
    }
    if (trials.empty())
        return pa_fail(s, xmode == PA_EXCHANGE_RESIDENT ? PA_EINVAL : PA_EINVAL,
                       xmode == PA_EXCHANGE_RESIDENT ? "the workgroups do not fit on the device at once"
                                                     : "a cell does not fit the LDS of one workgroup");
    double best_ms = INFINITY;
    Trial best{{0, 0, 0}, false};
    const bool tune = trials.size() > 1;
    if (tune && pa_snapshot(s, 0) != PA_OK) return PA_EDEVICE;
    for (const Trial &tr : trials) {
        const Cand &cd = tr.c;
        BatchedPlan P;
        P.threads = cd.threads;
        P.solver_waves = cd.sw;
        P.multi = tr.multi;
        pack(o, cd.cpb, cd.threads, P.blk, P.lds);
        if (!tune) {
            best = tr;
            break;
        }
        if (upload_plan(s, P) != PA_OK) return PA_EDEVICE;
        // trial: 1 warm epoch in the trial's own form, then time 4 epochs
        // of K steps
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
            return pa_fail(s, PA_EDEVICE, "event");
        int r = 0;
        if (tr.multi) {
            // a cooperative launch the device refuses (too many workgroups to
            // be resident) only rules this trial out
            const bool refused = enqueue_resident(d, P, d.K, st, nullptr, nullptr) != 0;
            if (!refused) r |= (int)hipEventRecord(a, st);
            if (refused || enqueue_resident(d, P, 4 * d.K, st, nullptr, nullptr) != 0) {
                (void)hipGetLastError();
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
                if (hipStreamSynchronize(st) != hipSuccess || pa_snapshot(s, 1) != PA_OK)
                    return pa_fail(s, PA_EDEVICE, "autotune trial");
                continue;
            }
        } else {
            r |= enqueue_epoch(d, P, d.K, st, nullptr, nullptr);
            r |= (int)hipEventRecord(a, st);
            for (int e = 0; e < 4; ++e) r |= enqueue_epoch(d, P, d.K, st, nullptr, nullptr);
        }
        r |= (int)hipEventRecord(b, st);
        if (r || hipEventSynchronize(b) != hipSuccess) return pa_fail(s, PA_EDEVICE, "autotune trial");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (ms < best_ms) {
            best_ms = ms;
            best = tr;
        }
        if (pa_snapshot(s, 1) != PA_OK) return PA_EDEVICE;
    }
    if (!best.c.cpb) return pa_fail(s, PA_EINVAL, "a cell does not fit the LDS of one workgroup");
    plan->cells_per_block = best.c.cpb;
    plan->threads = best.c.threads;
    plan->solver_waves = best.c.sw;
    plan->multi = best.multi;
    pack(o, best.c.cpb, best.c.threads, plan->blk, plan->lds);
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

void batched_plan_shape(pa_sim *s, uint32_t &threads, uint32_t &solver_waves, uint32_t &exchange) {
    BatchedPlan *p = pa_plan(s);
    threads = p ? p->threads : 0;
    solver_waves = p ? (p->threads == 64 ? 1 : p->solver_waves) : 0;
    exchange = p ? (p->multi ? PA_EXCHANGE_RESIDENT : PA_EXCHANGE_KERNEL) : 0;
}

// Steps one resident launch may run (0 when the plan exchanges spikes
// between launches); bounded so that a launch stays well under a second.
uint32_t batched_resident_steps(pa_sim *s) {
    BatchedPlan *p = pa_plan(s);
    return p && p->multi ? 256u * pa_devnet(s).K : 0u;
}

pa_status run_resident_batched(pa_sim *s, uint32_t nsteps, hipEvent_t e0, hipEvent_t e1) {
    const BatchedPlan &P = *pa_plan(s);
    if (enqueue_resident(pa_devnet(s), P, nsteps, pa_stream(s), e0, e1))
        return pa_fail(s, PA_EDEVICE, "resident epoch launch");
    return PA_OK;
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
