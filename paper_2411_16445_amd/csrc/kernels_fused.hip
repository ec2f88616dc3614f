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
#include <cstdlib>
#include <vector>

#include "../../include/plasticarbor.h"
#include "device_common.hpp"
#include "sim.hpp"

namespace pa {

// LDS layout of a workgroup owning nv CVs, ns synapses, nh HH CVs and nc
// cells for an epoch of at most K steps; gates, conductance, calcium and
// decay factors take tsize bytes.  The same arithmetic sizes the launch on
// the host and places the arrays on the device.
struct FusedLayout {
    // doubles
    uint32_t V, D, B, Ax, D0, Cdt, Gpe, H, Z, Erev, Abs, P, Vold;
    // T
    uint32_t G, C, Dec, M, HH, N;
    // 32-bit
    uint32_t Par, HHk, CvSyn, CvCl, Cb0, Cs0, Det, HHcv, EvN, EvOff, Scan;
    // events of the epoch, each slot's records sorted into delivery order
    uint32_t EvBuf, ev_cap;
    // 16-bit, 8-bit
    uint32_t SynCell, Run, Kind, Post;
    // branch segments
    uint32_t Cu, Cb, SegA, SegB, SegCell, KidOff, Kids, SegLvl;
    // HH constants: 6 channel parameters and the area factor per HH CV
    uint32_t HHp;
    // cyclic-reduction work arrays (mixed form): lower, upper, and a second
    // copy of lower, diagonal, upper, right-hand side
    uint32_t Pa, Pc, Qa, Qd, Qc, Qr;
    uint32_t total;
    __host__ __device__ FusedLayout(uint32_t nv, uint32_t ns, uint32_t nh, uint32_t nc, uint32_t K,
                                    uint32_t tsize, uint32_t ng) {
        uint32_t o = 0;
        auto take = [&](uint32_t bytes, uint32_t align) {
            o = (o + align - 1) / align * align;
            const uint32_t r = o;
            o += bytes;
            return r;
        };
        V = take(8 * nv, 16); D = take(8 * nv, 8); B = take(8 * nv, 8); Ax = take(8 * nv, 8);
        D0 = take(8 * nv, 8); Cdt = take(8 * nv, 8); Gpe = take(8 * nv, 8);
        H = take(8 * ns, 8); Z = take(8 * ns, 8); Erev = take(8 * ns, 8); Abs = take(8 * ns, 8);
        P = take(8 * nc, 8); Vold = take(8 * nc, 8);
        G = take(tsize * ns, 8); C = take(tsize * ns, 8); Dec = take(tsize * ns, 8);
        M = take(tsize * nh, 8); HH = take(tsize * nh, 8); N = take(tsize * nh, 8);
        Par = take(4 * nv, 4); HHk = take(4 * nv, 4); CvSyn = take(4 * (nv + 1), 4);
        CvCl = take(4 * (nv + 1), 4); Cb0 = take(4 * (nc + 1), 4); Cs0 = take(4 * (nc + 1), 4);
        Det = take(4 * nc, 4); HHcv = take(4 * nh, 4); EvN = take(4 * nc * K, 4);
        EvOff = take(4 * nc * K, 4); Scan = take(4 * 257, 4);
        ev_cap = 2 * nc * K + 32;
        EvBuf = take(32 * ev_cap, 16);
        Cu = take(8 * ng, 8); Cb = take(8 * ng, 8); HHp = take(8 * 7 * nh, 8);
        const uint32_t np = tsize == 4 ? nv : 0;
        Pa = take(8 * np, 8); Pc = take(8 * np, 8); Qa = take(8 * np, 8); Qd = take(8 * np, 8);
        Qc = take(8 * np, 8); Qr = take(8 * np, 8);
        SynCell = take(2 * ns, 2); Run = take(2 * nv, 2);
        SegA = take(2 * ng, 2); SegB = take(2 * ng, 2); SegCell = take(2 * ng, 2);
        KidOff = take(2 * (ng + 1), 2); Kids = take(2 * ng, 2);
        Kind = take(ns, 1); Post = take(nc, 1); SegLvl = take(ng, 1);
        total = (o + 15) / 16 * 16;
    }
};

#ifdef PA_STAGE_TIMING
// Diagnostic build only: wall-clock ticks per stage summed over workgroups.
__device__ unsigned long long pa_stage_ticks[8];
#define STAGE_INIT() uint64_t st_prev_ = wall_clock64(); uint64_t st_acc_[8] = {0, 0, 0, 0, 0, 0, 0, 0}
#define STAGE_MARK(k_) do { if (tid == 0) { const uint64_t t_ = wall_clock64(); st_acc_[k_] += t_ - st_prev_; st_prev_ = t_; } } while (0)
#define STAGE_FLUSH() do { if (tid == 0) for (int k_ = 0; k_ < 8; ++k_) atomicAdd(&pa_stage_ticks[k_], (unsigned long long)st_acc_[k_]); } while (0)
#else
#define STAGE_INIT() do {} while (0)
#define STAGE_MARK(k_) do {} while (0)
#define STAGE_FLUSH() do {} while (0)
#endif

__device__ __forceinline__ double wave_sum_down(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_down(x, off, 64);
    return x;
}

// One epoch of nsteps (<= K) steps for the cells blk[b] .. blk[b+1]-1 of
// workgroup b.  Mutable state of those cells (V, gates, g, c, h, z, p, post
// flag), their constants and the epoch's event counts live in LDS, so a
// step touches global memory only for events, spikes and rare noise keys.
template <class T, uint32_t BS>
__global__ __launch_bounds__(BS) void k_epoch(DevNet d, const uint32_t *__restrict__ blk,
                                              const uint32_t *__restrict__ blk_lvl, uint32_t nsteps) {
    extern __shared__ double lds[];
    uint8_t *L = (uint8_t *)lds;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    constexpr uint32_t NW = BS / 64;
    const uint32_t c0 = blk[blockIdx.x], c1 = blk[blockIdx.x + 1];
    const uint32_t ncb = c1 - c0;
    const uint32_t v0 = d.cv_off[c0], nv = d.cv_off[c1] - v0;
    const uint32_t s0 = d.syn_off[c0], ns = d.syn_off[c1] - s0;
    const uint32_t k0 = d.hh_off[c0], nhh = d.hh_off[c1] - k0;
    const uint32_t g0 = d.seg_off[c0], ng = d.seg_off[c1] - g0;
    const uint32_t nlev = blk_lvl[blockIdx.x];
    const uint32_t K = d.K;
    constexpr bool EXACT = sizeof(T) == 8;
    const FusedLayout lay(nv, ns, nhh, ncb, K, sizeof(T), ng);
    double *sV = (double *)(L + lay.V), *sD = (double *)(L + lay.D), *sB = (double *)(L + lay.B);
    double *sAx = (double *)(L + lay.Ax), *sD0 = (double *)(L + lay.D0), *sCdt = (double *)(L + lay.Cdt);
    double *sGpe = (double *)(L + lay.Gpe), *sH = (double *)(L + lay.H), *sZ = (double *)(L + lay.Z);
    double *sErev = (double *)(L + lay.Erev), *sAbs = (double *)(L + lay.Abs);
    double *sP = (double *)(L + lay.P), *sVold = (double *)(L + lay.Vold);
    T *sG = (T *)(L + lay.G), *sC = (T *)(L + lay.C), *sDec = (T *)(L + lay.Dec);
    T *sM = (T *)(L + lay.M), *sHH = (T *)(L + lay.HH), *sN = (T *)(L + lay.N);
    int32_t *sPar = (int32_t *)(L + lay.Par), *sHHk = (int32_t *)(L + lay.HHk);
    uint32_t *sCvSyn = (uint32_t *)(L + lay.CvSyn), *sCvCl = (uint32_t *)(L + lay.CvCl);
    uint32_t *sCb0 = (uint32_t *)(L + lay.Cb0), *sCs0 = (uint32_t *)(L + lay.Cs0);
    uint32_t *sDet = (uint32_t *)(L + lay.Det), *sHHcv = (uint32_t *)(L + lay.HHcv);
    uint32_t *sEvN = (uint32_t *)(L + lay.EvN), *sEvOff = (uint32_t *)(L + lay.EvOff);
    uint32_t *sScan = (uint32_t *)(L + lay.Scan);
    uint16_t *sSynCell = (uint16_t *)(L + lay.SynCell), *sRun = (uint16_t *)(L + lay.Run);
    uint8_t *sKind = L + lay.Kind, *sPost = L + lay.Post, *sSegLvl = L + lay.SegLvl;
    double *sCu = (double *)(L + lay.Cu), *sCb = (double *)(L + lay.Cb), *sHHp = (double *)(L + lay.HHp);
    uint16_t *sSegA = (uint16_t *)(L + lay.SegA), *sSegB = (uint16_t *)(L + lay.SegB);
    uint16_t *sSegCell = (uint16_t *)(L + lay.SegCell), *sKidOff = (uint16_t *)(L + lay.KidOff);
    uint16_t *sKids = (uint16_t *)(L + lay.Kids);
    // blocks whose cells are all unbranched (one segment per cell)
    const bool chains = (ng == ncb);
    uint32_t pcr_steps = 0;
    if (!EXACT && chains) {
        uint32_t len = 1;
        for (uint32_t c = 0; c < ncb; ++c) len = max(len, d.cv_off[c0 + c + 1] - d.cv_off[c0 + c]);
        while ((1u << pcr_steps) < len) ++pcr_steps;
    }
    const SynView<T> sv{sG, sC, sH, sZ, s0};
    const SynConst<T> sc{sErev, sDec, sKind, s0};
    const GateView<T> gv{sM, sHH, sN, k0};
    const uint64_t n0 = d.ctr->step;
    STAGE_INIT();

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
        sRun[i] = d.run[g];
        sHHk[i] = d.hh_of[g];
        sCvSyn[i] = d.cv_syn_off[g];
        sCvCl[i] = d.cv_cl_off[g];
        if (i == nv - 1) {
            sCvSyn[nv] = d.cv_syn_off[g + 1];
            sCvCl[nv] = d.cv_cl_off[g + 1];
        }
    }
    for (uint32_t s = tid; s < ns; s += BS) {
        const uint32_t q = s0 + s;
        sG[s] = ((const T *)d.g)[q];
        sC[s] = ((const T *)d.c)[q];
        sH[s] = d.h[q];
        sZ[s] = d.z[q];
        sErev[s] = d.syn_erev[q];
        if constexpr (sizeof(T) == 8) sDec[s] = (T)d.syn_decay[q];
        else sDec[s] = d.syn_decay_f[q];
        sKind[s] = d.syn_kind[q];
        sSynCell[s] = (uint16_t)(d.syn_cell[q] - c0);
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
        if (c < ncb) {
            sP[c] = d.p[c0 + c];
            sPost[c] = d.post[c0 + c];
            sDet[c] = d.det_cv[c0 + c] - v0;
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
    // external arrivals of this epoch for the workgroup's cells enter the
    // rings (trains and Poisson sources grouped by target cell)
    {
        const uint64_t epoch_end = n0 + nsteps;
        const uint32_t t0 = d.tr_cell_off[c0], t1 = d.tr_cell_off[c1];
        for (uint32_t x = t0 + tid; x < t1; x += BS) inject_train(d, d.tr_by_cell[x], n0, epoch_end);
        const uint32_t p0 = d.po_cell_off[c0], p1 = d.po_cell_off[c1];
        for (uint32_t x = p0 + tid; x < p1; x += BS) inject_poisson(d, d.po_by_cell[x], n0, epoch_end);
    }
    if (tid == 0) sScan[0] = 0;
    __syncthreads();
    // events of the epoch: one lane per (cell, step) slot takes the slot's
    // count, claims room in the LDS event buffer, copies the records there
    // and sorts them into delivery order (a slot that does not fit is
    // sorted in place in the ring); the delivery statistics are counted
    // here, in parallel
    const uint32_t nslot = ncb * nsteps;
    Event *sEv = (Event *)(L + lay.EvBuf);
    for (uint32_t x = tid; x < nslot; x += BS) {
        const uint32_t c = x / nsteps, st = x - c * nsteps;
        const uint64_t ring = (uint64_t)(c0 + c) * d.R + (uint32_t)((n0 + st) % d.R);
        const uint32_t cnt = min(d.ev_n[ring], d.Q);
        sEvN[c * K + st] = cnt;
        if (!cnt) continue;
        d.ev_n[ring] = 0;
        Event *ev = d.ev + ring * d.Q;
        const uint32_t off = atomicAdd(&sScan[0], cnt);
        Event *dst;
        if (off + cnt <= lay.ev_cap) {
            dst = sEv + off;
            for (uint32_t i = 0; i < cnt; ++i) dst[i] = ev[i];
            sEvOff[c * K + st] = off;
        } else {
            dst = ev;
            sEvOff[c * K + st] = 0xffffffffu;
        }
        sort_slot(dst, cnt);
        for (uint32_t i = 0; i < cnt; ++i) {
            const uint32_t sy = dst[i].syn, po = dst[i].port;
            atomicAdd(&d.ev_cnt[2 * sy + po - 1], 1ull);
            atomicAdd(&d.ev_sum[2 * sy + po - 1], (unsigned long long)(n0 + st));
        }
    }
    unsigned long long delivered = 0;
    __syncthreads();
    STAGE_MARK(6);

    // protein trigger sum of step m (one wavefront per cell: strided lane
    // sums, then a fixed shuffle tree), protein synthesis, detection
    auto stage_e = [&](uint64_t m) {
        for (uint32_t c = wave; c < ncb; c += NW) {
            const uint32_t a = sCs0[c], e = sCs0[c + 1];
            double S = 0.0;
            for (uint32_t s = a + lane; s < e; s += 64) S += sAbs[s];
            S = wave_sum_down(S);
            if (lane == 0) {
                sP[c] = prp_next(d, sP[c], S);
                sPost[c] = detect(d, c0 + c, m, sVold[c], sV[sDet[c]]) ? 1 : 0;
            }
        }
    };

    for (uint32_t st = 0; st < nsteps; ++st) {
        const uint64_t n = n0 + st;
        const double tn = (double)n * d.dt;
        // A. events due at step n, already in delivery order; the protein
        //    update and detection of step n-1 (independent of them)
        for (uint32_t c = tid; c < ncb; c += BS) {
            const uint32_t cnt = sEvN[c * K + st];
            if (!cnt) continue;
            const uint32_t off = sEvOff[c * K + st];
            const Event *ev = off != 0xffffffffu ? sEv + off
                                                 : d.ev + ((uint64_t)(c0 + c) * d.R + (uint32_t)(n % d.R)) * d.Q;
            for (uint32_t i = 0; i < cnt; ++i) apply_event<T>(d, ev[i].syn, ev[i].port, ev[i].w, sv, sc);
            delivered += cnt;
        }
        if (st > 0) stage_e(n - 1);
        __syncthreads();
        STAGE_MARK(0);
        // B. currents at V^n and assembly of the cable system
        for (uint32_t i = tid; i < nv; i += BS) {
            const double v = sV[i];
            double I, G;
            const int32_t hk = sHHk[i];
            const double *P = hk >= 0 ? sHHp + 7 * (hk - (int32_t)k0) : nullptr;
            cv_current<T>(d, hk, P, hk >= 0 ? P[6] : 0.0, v, tn, gv, sv, sc, sCvSyn[i], sCvSyn[i + 1], sCvCl[i],
                          sCvCl[i + 1], I, G);
            sD[i] = sD0[i] + G;
            sB[i] = ((sCdt[i] * v + sGpe[i]) - I) + G * v;
        }
        __syncthreads();
        STAGE_MARK(1);
        // C. Hines elimination on wavefront 0, level-scheduled over branch
        //    segments: the segments of one level are eliminated in parallel
        //    lanes, deepest level first; a branch point takes its children's
        //    contributions in descending child order, as in the sequential
        //    elimination.  Meanwhile the other wavefronts update the synapses
        //    (decay, post-synaptic hook, plasticity from step-start values),
        //    which do not depend on the new voltage.
        if (wave == 0 && !EXACT && chains) {
            // mixed form, unbranched cells: parallel cyclic reduction of each
            // cell's tridiagonal system across the wavefront's lanes (FP64;
            // equal to the elimination up to rounding)
            double *pa = (double *)(L + lay.Pa), *pc = (double *)(L + lay.Pc);
            double *qa = (double *)(L + lay.Qa), *qd = (double *)(L + lay.Qd);
            double *qc = (double *)(L + lay.Qc), *qr = (double *)(L + lay.Qr);
            for (uint32_t c = lane; c < ncb; c += 64) sVold[c] = sV[sDet[c]];
            for (uint32_t i = lane; i < nv; i += 64) {
                pa[i] = sPar[i] >= 0 ? -sAx[i] : 0.0;
                pc[i] = (i + 1 < nv && sPar[i + 1] == (int32_t)i) ? -sAx[i + 1] : 0.0;
            }
            wave_sync();
            double *A = pa, *Dd = sD, *Cc = pc, *Rr = sB;
            double *A2 = qa, *D2 = qd, *C2 = qc, *R2 = qr;
            for (uint32_t k = 0, sft = 1; k < pcr_steps; ++k, sft <<= 1) {
                for (uint32_t i = lane; i < nv; i += 64) {
                    const double ai = A[i], ci = Cc[i];
                    double na = 0.0, nc2 = 0.0, nd = Dd[i], nr = Rr[i];
                    // neighbours at distance sft inside the same cell: a
                    // nonzero coupling marks a neighbour
                    if (ai != 0.0 && i >= sft) {
                        const uint32_t im = i - sft;
                        const double al = -qdiv<false>(ai, Dd[im]);
                        na = al * A[im];
                        nd += al * Cc[im];
                        nr += al * Rr[im];
                    }
                    if (ci != 0.0 && i + sft < nv) {
                        const uint32_t ip = i + sft;
                        const double ga = -qdiv<false>(ci, Dd[ip]);
                        nc2 = ga * Cc[ip];
                        nd += ga * A[ip];
                        nr += ga * Rr[ip];
                    }
                    A2[i] = na;
                    D2[i] = nd;
                    C2[i] = nc2;
                    R2[i] = nr;
                }
                wave_sync();
                double *t;
                t = A; A = A2; A2 = t;
                t = Dd; Dd = D2; D2 = t;
                t = Cc; Cc = C2; C2 = t;
                t = Rr; Rr = R2; R2 = t;
            }
            for (uint32_t i = lane; i < nv; i += 64) {
                const double v = qdiv<false>(Rr[i], Dd[i]);
                sV[i] = v;
                if (!isfinite(v)) raise_flag(d, FLAG_NONFINITE, c0);
            }
        } else if (wave == 0) {
            for (uint32_t c = lane; c < ncb; c += 64) sVold[c] = sV[sDet[c]];
            for (int lv = (int)nlev - 1; lv >= 0; --lv) {
                for (uint32_t g = lane; g < ng; g += 64) {
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
            for (uint32_t lv = 0; lv < nlev; ++lv) {
                for (uint32_t g = lane; g < ng; g += 64) {
                    if (sSegLvl[g] != lv) continue;
                    const uint32_t a = sSegA[g], b = sSegB[g];
                    const int32_t p = sPar[a];
                    sV[a] = (p < 0) ? qdiv<EXACT>(sB[a], sD[a]) : qdiv<EXACT>(sB[a] - (-sAx[a]) * sV[p], sD[a]);
                    if (!seg_forward<EXACT>(sD, sB, sV, sAx, a, b)) raise_flag(d, FLAG_NONFINITE, c0 + sSegCell[g]);
                }
                wave_sync();
            }
        }
        STAGE_MARK(7);
        {
            // synapses on wavefronts 1.. (all lanes when there is one wavefront)
            const uint32_t first = NW > 1 ? 64u : 0u;
            if (tid >= first) {
                for (uint32_t s = tid - first; s < ns; s += BS - first) {
                    const uint32_t cl = sSynCell[s];
                    sAbs[s] = syn_update<T>(d, s0 + s, n, sP[cl], sPost[cl] != 0, sv, sc);
                }
            }
        }
        __syncthreads();
        STAGE_MARK(2);
        // D. gates at V^{n+1}
        for (uint32_t k = tid; k < nhh; k += BS) gate_update<T>(d, k0 + k, sV[sHHcv[k]], gv);
        STAGE_MARK(3);
    }
    // E of the epoch's last step
    stage_e(n0 + nsteps - 1);
    __syncthreads();
    STAGE_MARK(4);
    // ---- stage out
    for (uint32_t i = tid; i < nv; i += BS) d.V[v0 + i] = sV[i];
    for (uint32_t s = tid; s < ns; s += BS) {
        ((T *)d.g)[s0 + s] = sG[s];
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
        d.post[c0 + c] = sPost[c];
    }
    if (delivered) atomicAdd((unsigned long long *)&d.ctr->events, delivered);
    __syncthreads();
    STAGE_MARK(5);
    STAGE_FLUSH();
}

int launch_epoch_fused(const DevNet &d, uint32_t nsteps, const uint32_t *blk, const uint32_t *blk_lvl,
                       uint32_t n_blocks, size_t lds_bytes, uint32_t block_threads, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (block_threads == 64) {
        if (d.mixed) hipLaunchKernelGGL((k_epoch<float, 64>), dim3(n_blocks), dim3(64), lds_bytes, s, d, blk, blk_lvl, nsteps);
        else hipLaunchKernelGGL((k_epoch<double, 64>), dim3(n_blocks), dim3(64), lds_bytes, s, d, blk, blk_lvl, nsteps);
    } else {
        if (d.mixed) hipLaunchKernelGGL((k_epoch<float, 256>), dim3(n_blocks), dim3(256), lds_bytes, s, d, blk, blk_lvl, nsteps);
        else hipLaunchKernelGGL((k_epoch<double, 256>), dim3(n_blocks), dim3(256), lds_bytes, s, d, blk, blk_lvl, nsteps);
    }
    return (int)hipGetLastError();
}

}  // namespace pa

#ifdef PA_STAGE_TIMING
extern "C" int pa_debug_stage_ticks(unsigned long long *out, int reset) {
    if (hipMemcpyFromSymbol(out, HIP_SYMBOL(pa::pa_stage_ticks), 8 * sizeof(unsigned long long)) != hipSuccess)
        return -1;
    if (reset) {
        unsigned long long z[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (hipMemcpyToSymbol(HIP_SYMBOL(pa::pa_stage_ticks), z, sizeof z) != hipSuccess) return -1;
    }
    return 0;
}
#endif

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
    std::vector<uint32_t> lvl;  // branch levels per block
    uint32_t *d_blk = nullptr, *d_lvl = nullptr;
    size_t lds = 0;
    uint32_t cells_per_block = 0;
    uint32_t threads = 256;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t graph_epochs = 0;
};

BatchedPlan *&pa_plan(pa_sim *s);

namespace {

constexpr size_t LDS_MAX = 160 * 1024;

struct Offsets {
    std::vector<uint32_t> cv, syn, hh, seg, nlev;  // nlev: branch levels per cell
    uint32_t tsize, K;
};

// Packs consecutive cells, at most cpb per workgroup, within an LDS budget
// that leaves room for several resident workgroups per CU.
bool pack(const Offsets &o, uint32_t cpb, uint32_t threads, std::vector<uint32_t> &blk, size_t &lds) {
    const size_t budget = threads == 64 ? 32 * 1024 : 64 * 1024;
    const uint32_t nc = (uint32_t)o.cv.size() - 1;
    auto bytes = [&](uint32_t a, uint32_t e) {
        return (size_t)FusedLayout(o.cv[e] - o.cv[a], o.syn[e] - o.syn[a], o.hh[e] - o.hh[a], e - a, o.K,
                                   o.tsize, o.seg[e] - o.seg[a]).total;
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

pa_status upload_plan(pa_sim *s, BatchedPlan &P, const Offsets &o) {
    P.lvl.assign(P.blk.size() - 1, 1);
    for (size_t b = 0; b + 1 < P.blk.size(); ++b)
        for (uint32_t c = P.blk[b]; c < P.blk[b + 1]; ++c) P.lvl[b] = std::max(P.lvl[b], o.nlev[c]);
    P.d_blk = (uint32_t *)pa_dev_alloc(s, P.blk.size() * 4);
    P.d_lvl = (uint32_t *)pa_dev_alloc(s, P.lvl.size() * 4);
    if (!P.d_blk || !P.d_lvl) return pa_fail(s, PA_ENOMEM, "block table");
    if (hipMemcpy(P.d_blk, P.blk.data(), P.blk.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P.d_lvl, P.lvl.data(), P.lvl.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return pa_fail(s, PA_EDEVICE, "block table upload");
    return PA_OK;
}

int enqueue_epoch(const DevNet &d, const BatchedPlan &P, uint32_t nsteps, hipStream_t st,
                  hipEvent_t e0, hipEvent_t e1) {
    int r = 0;
    if (e0) (void)hipEventRecord(e0, st);
    r |= launch_epoch_fused(d, nsteps, P.d_blk, P.d_lvl, (uint32_t)P.blk.size() - 1, P.lds, P.threads, st);
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
    Offsets o;
    o.cv.resize(d.n_cells + 1);
    o.syn.resize(d.n_cells + 1);
    o.hh.resize(d.n_cells + 1);
    o.tsize = d.mixed ? 4 : 8;
    o.K = d.K;
    o.seg.resize(d.n_cells + 1);
    o.nlev.assign(d.n_cells, 1);
    {
        std::vector<uint8_t> lvl(d.n_seg);
        if (hipMemcpy(o.seg.data(), d.seg_off, o.seg.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            (d.n_seg && hipMemcpy(lvl.data(), d.seg_lvl, d.n_seg, hipMemcpyDeviceToHost) != hipSuccess))
            return pa_fail(s, PA_EDEVICE, "segments");
        for (uint32_t c = 0; c < d.n_cells; ++c)
            for (uint32_t g = o.seg[c]; g < o.seg[c + 1]; ++g) o.nlev[c] = std::max<uint32_t>(o.nlev[c], lvl[g] + 1u);
    }
    if (hipMemcpy(o.cv.data(), d.cv_off, o.cv.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(o.syn.data(), d.syn_off, o.syn.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(o.hh.data(), d.hh_off, o.hh.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return pa_fail(s, PA_EDEVICE, "offsets");
    struct Cand { uint32_t threads, cpb; };
    std::vector<Cand> cands;
    const uint32_t fixed = pa_cfg(s).cells_per_block;
    if (fixed) cands.push_back({fixed >= 4 ? 256u : 64u, fixed});
    else {
        for (uint32_t c : {1u, 2u, 4u}) cands.push_back({64u, c});
        for (uint32_t c : {4u, 8u, 16u, 32u, 64u}) cands.push_back({256u, c});
    }
    double best_ms = INFINITY;
    Cand best{0, 0};
    const bool tune = cands.size() > 1;
    if (tune && pa_snapshot(s, 0) != PA_OK) return PA_EDEVICE;
    for (const Cand &cd : cands) {
        BatchedPlan P;
        P.threads = cd.threads;
        if (!pack(o, cd.cpb, cd.threads, P.blk, P.lds)) continue;
        if (!tune) {
            best = cd;
            break;
        }
        if (upload_plan(s, P, o) != PA_OK) return PA_EDEVICE;
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
        if (getenv("PA_AUTOTUNE_VERBOSE"))
            fprintf(stderr, "[autotune] threads %u cells/block %u blocks %zu lds %zu: %.3f ms / 4 epochs\n",
                    cd.threads, cd.cpb, P.blk.size() - 1, P.lds, ms);
        if (ms < best_ms) {
            best_ms = ms;
            best = cd;
        }
        if (pa_snapshot(s, 1) != PA_OK) return PA_EDEVICE;
    }
    if (!best.cpb) return pa_fail(s, PA_EINVAL, "a cell does not fit the LDS of one workgroup");
    plan->cells_per_block = best.cpb;
    plan->threads = best.threads;
    pack(o, best.cpb, best.threads, plan->blk, plan->lds);
    if (upload_plan(s, *plan, o) != PA_OK) return PA_EDEVICE;
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
