// Search by triplet for MI355X (gfx950): kernels and the C ABI of include/sbt.h.
//
// Plain form: one workgroup per event and one launch per stage.
// Batched form: a persistent work-stealing kernel (sbt_persistent.hip) that
// runs every stage of an event inside one workgroup and then takes the next
// event from a device counter, followed by a scan over events and the CSR
// write, replayed as one captured HIP graph.  Both forms share the device
// stages of sbt_device.h and give byte-identical outputs.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <mutex>
#include <vector>

#include "sbt.h"
#include "sbt_device.h"
#include "sbt_internal.h"
#include "sbt_kernels.h"

using namespace sbt;

// ============================================================== kernels

// plain form ----------------------------------------------------------------

// one workgroup of 512 lanes per event: on the mu=7.6 x 1,000, mu in
// U{1..25} x 2,000 and mu=30 x 400 batches 512 lanes beat 256 (1.30x, 1.34x,
// 1.49x) and 1,024 (except on the densest events)
constexpr int kPlainThreads = 512;
constexpr int kPlainCap = 672;
constexpr int kPlainOwnCap = 16384;
// dynamic LDS of the plain compaction kernel: its LDS form (previous-hit
// links and the key-ordered track list, 2 N + 2 (N / 3 + 1) bytes) fits
// events of up to about 24,000 hits; larger ones take the memory form
constexpr int kPlainCompactLds = 64 * 1024;

template <int B>
__global__ __launch_bounds__(B) void k_phi_sort(sbt_params P, HitsArgs H, Work W, int sortcap)
{
    __shared__ Shared<B> S;
    const int e = blockIdx.x;
    int hb, N;
    const int st = load_event<B>(P, H, e, S, &hb, &N);
    if (threadIdx.x == 0) ws_evinfo(W)[e].st = st;
    if (st != 0) return;
    stage_sort<B>(P, H, event_view(W, e, hb, N), S, sortcap);
}

// The paper's sort by phi, for comparison (Section 3, "Sort by phi": a
// parallel insertion sort computes the permutation): every hit counts the
// hits of its module with a smaller (phi16, id) key, which is its rank,
// O(n^2) per module.  Keys are in LDS when kLdsKeys, else in the workspace.
// Writes the same sorted hits as stage_sort.
template <int B, bool kLdsKeys>
__global__ __launch_bounds__(B) void k_phi_sort_rank(sbt_params P, HitsArgs H, Work W)
{
    __shared__ Shared<B> S;
    const int e = blockIdx.x;
    int hb, N;
    const int st = load_event<B>(P, H, e, S, &hb, &N);
    if (threadIdx.x == 0) ws_evinfo(W)[e].st = st;
    if (st != 0) return;
    const Ev v = event_view(W, e, hb, N);
    const HitSrc src = hit_src(H, hb);
    uint32_t *keys = kLdsKeys ? reinterpret_cast<uint32_t *>(g_lds) : v.keys();
    for (int i = threadIdx.x; i < N; i += B) {
        float x, y;
        src.xy(i, x, y);
        keys[i] = ((uint32_t)phi16(x, y) << 16) | (uint32_t)i;
    }
    __syncthreads();
    const int M = P.n_modules;
    for (int i = threadIdx.x; i < N; i += B) {
        const int m = module_of(S.mo, M, i);
        const int lo = S.mo[m], hi = S.mo[m + 1];
        const uint32_t key = keys[i];
        int rank = lo;
        for (int j = lo; j < hi; ++j) rank += keys[j] < key;
        Hit16 h;
        src.xyz(i, h.x, h.y, h.z);
        h.qid = (key >> 16) | (key << 16);
        at(v.hs(), rank) = h;
    }
}

template <int B, int CAP, bool kCand>
__global__ __launch_bounds__(B) void k_seed_follow(sbt_params P, HitsArgs H, Work W, int own_cap)
{
    __shared__ Shared<B> S;
    const int e = blockIdx.x;
    if (ws_evinfo(W)[e].st != 0) return;
    int hb, N;
    load_event<B>(P, H, e, S, &hb, &N);
    stage_track<B, CAP, kCand>(P, event_view(W, e, hb, N), S, own_cap, true);
    if (threadIdx.x == 0) ws_evinfo(W)[e].nfin = S.cnt[3];
}

// The paper's separate candidate pass (ablation): the pendulum start of every
// hit, written before the seeding kernel runs.
template <int B>
__global__ __launch_bounds__(B) void k_fill_candidates(sbt_params P, HitsArgs H, Work W)
{
    __shared__ Shared<B> S;
    const int e = blockIdx.x;
    if (ws_evinfo(W)[e].st != 0) return;
    int hb, N;
    load_event<B>(P, H, e, S, &hb, &N);
    stage_fill_candidates<B>(P, event_view(W, e, hb, N), S);
}

template <int B>
__global__ __launch_bounds__(B) void k_weak_filter(sbt_params P, HitsArgs H, Work W)
{
    const int e = blockIdx.x;
    if (ws_evinfo(W)[e].st != 0) return;
    const int hb = H.eo[e];
    const Ev v = event_view(W, e, hb, H.eo[e + 1] - hb);
    stage_filter<B>(P, v, ws_evinfo(W)[e].nfin, v.own());
}

template <int B>
__global__ __launch_bounds__(B) void k_compact(HitsArgs H, Work W, int lds_bytes)
{
    __shared__ int scan[2 * (B / 64)];
    const int e = blockIdx.x;
    if (ws_evinfo(W)[e].st != 0) {
        if (threadIdx.x == 0) { ws_evinfo(W)[e].nt = 0; ws_evinfo(W)[e].nh = 0; }
        return;
    }
    const int hb = H.eo[e];
    stage_compact<B>(event_view(W, e, hb, H.eo[e + 1] - hb), scan, lds_bytes);
}

// batched form ----------------------------------------------------------------

// Resets the work counter and orders the events by size, largest first, so
// the persistent workgroups start the longest events early (the order of
// processing never changes an event's result).  Counting sort on N / 64.
constexpr int kOrderThreads = 256;    // small, so it fits beside another stream's persistent workgroups
constexpr int kOrderClasses = 1024;
constexpr int kOrderBatch = 4;        // events whose offsets a lane loads together
__global__ __launch_bounds__(kOrderThreads) void k_prepare(HitsArgs H, Work W)
{
    __shared__ int hist[kOrderClasses + 1];
    __shared__ int fill[kOrderClasses];
    __shared__ int sw[2 * (kOrderThreads / 64)];
    if (threadIdx.x == 0) {
        *ws_counterp(W) = 0u;
        *ws_defer_countp(W) = 0u;
    }
    for (int i = threadIdx.x; i <= kOrderClasses; i += kOrderThreads) hist[i] = 0;
    for (int i = threadIdx.x; i < kOrderClasses; i += kOrderThreads) fill[i] = 0;
    __syncthreads();
    const int E = H.n_events;
    // bucket of event e (largest first), -1 past the end; a lane loads the
    // offsets of kOrderBatch events before using them
    auto bucket = [&](int e) -> int {
        if (e >= E) return -1;
        const int n = H.eo[e + 1] - H.eo[e];
        int cls = n < 0 ? 0 : (n >> 6);
        cls = cls > kOrderClasses - 1 ? kOrderClasses - 1 : cls;
        return kOrderClasses - 1 - cls;
    };
    // the buckets of a lane's first kOrderBatch events stay in registers for
    // the second pass (all of them when E <= kOrderBatch * kOrderThreads)
    int kf[kOrderBatch];
    for (int e0 = threadIdx.x; e0 < E; e0 += kOrderBatch * kOrderThreads) {
        int k[kOrderBatch];
#pragma unroll
        for (int j = 0; j < kOrderBatch; ++j) k[j] = bucket(e0 + j * kOrderThreads);
        if (e0 == (int)threadIdx.x) {
#pragma unroll
            for (int j = 0; j < kOrderBatch; ++j) kf[j] = k[j];
        }
#pragma unroll
        for (int j = 0; j < kOrderBatch; ++j)
            if (k[j] >= 0) atomicAdd(&hist[k[j]], 1);
    }
    __syncthreads();
    block_scan_inplace<kOrderThreads>(hist, kOrderClasses + 1, sw);
    __syncthreads();
    for (int e0 = threadIdx.x; e0 < E; e0 += kOrderBatch * kOrderThreads) {
        int k[kOrderBatch];
#pragma unroll
        for (int j = 0; j < kOrderBatch; ++j) k[j] = e0 == (int)threadIdx.x ? kf[j] : bucket(e0 + j * kOrderThreads);
#pragma unroll
        for (int j = 0; j < kOrderBatch; ++j)
            if (k[j] >= 0) ws_orderp(W)[hist[k[j]] + atomicAdd(&fill[k[j]], 1)] = e0 + j * kOrderThreads;
    }
}

// Between the passes of a two-pass launch: the events the first pass set
// aside (in the order it met them, largest first) move to the end of the event
// order, and the work counter starts at them, so that the second pass runs
// exactly those.
constexpr int kDeferThreads = 256;
__global__ __launch_bounds__(kDeferThreads) void k_defer(HitsArgs H, Work W)
{
    const int E = H.n_events;
    const int D = (int)*ws_defer_countp(W);
    for (int i = threadIdx.x; i < D; i += kDeferThreads) ws_orderp(W)[E - D + i] = ws_deferp(W)[i];
    if (threadIdx.x == 0) *ws_counterp(W) = (unsigned int)(E - D);
}

// shared tail -----------------------------------------------------------------

// exclusive scan over events of the per-event track and hit counts
constexpr int kScanThreads = 256;     // small, so it fits beside another stream's persistent workgroups
constexpr int kScanBatch = 8;         // events whose counts a lane loads together
__global__ __launch_bounds__(kScanThreads) void k_scan(HitsArgs H, Work W, OutArgs O)
{
    const int E = H.n_events;
    __shared__ int sw[2 * (kScanThreads / 64)];
    const int chunk = (E + kScanThreads - 1) / kScanThreads;
    const int beg = threadIdx.x * chunk;
    const int end = min(beg + chunk, E);
    EvInfo *ev = ws_evinfo(W);
    // a lane's counts (nt, nh: one 8-byte load per event), kScanBatch of
    // them in flight at once
    auto counts = [&](int i) -> int2 {
        return i < end ? *reinterpret_cast<const int2 *>(&ev[i].nt) : make_int2(0, 0);
    };
    // the counts of a lane's first kScanBatch events stay in registers for
    // the second pass (all of them when E <= kScanBatch * kScanThreads)
    int2 cf[kScanBatch];
    int st = 0, sh = 0;
    for (int i0 = beg; i0 < end; i0 += kScanBatch) {
        int2 c[kScanBatch];
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) c[k] = counts(i0 + k);
        if (i0 == beg) {
#pragma unroll
            for (int k = 0; k < kScanBatch; ++k) cf[k] = c[k];
        }
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
            st += c[k].x;
            sh += c[k].y;
        }
    }
    int tt, th;
    int ot = block_excl_scan<kScanThreads>(st, sw, 0, &tt);
    int oh = block_excl_scan<kScanThreads>(sh, sw, 1, &th);
    for (int i0 = beg; i0 < end; i0 += kScanBatch) {
        int2 c[kScanBatch];
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) c[k] = i0 == beg ? cf[k] : counts(i0 + k);
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
            if (i0 + k < end) {
                O.eto[i0 + k] = ot;
                ev[i0 + k].out_t = ot;
                ev[i0 + k].out_h = oh;
                ot += c[k].x;
                oh += c[k].y;
            }
        }
    }
    if (threadIdx.x == 0) {
        O.eto[E] = tt;
        if (O.tho && tt <= H.n_hits / 3) O.tho[tt] = th;
    }
}

constexpr int kWriteThreads = 256;
__global__ __launch_bounds__(kWriteThreads) void k_write(HitsArgs H, Work W, OutArgs O)
{
    for (int e = blockIdx.x; e < H.n_events; e += gridDim.x) {
        if (O.status && threadIdx.x == 0) O.status[e] = ws_evinfo(W)[e].st;
        const int nt = ws_evinfo(W)[e].nt, nh = ws_evinfo(W)[e].nh;
        if (nt == 0) continue;
        const int hb = H.eo[e];
        const int t0 = ws_evinfo(W)[e].out_t, p0 = ws_evinfo(W)[e].out_h;
        // four elements per lane and pass, their loads in flight together
        for (int i0 = threadIdx.x; i0 < nt; i0 += 4 * kWriteThreads) {
            int v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (i0 + k * kWriteThreads < nt) v[k] = ws_toff(W)[hb + i0 + k * kWriteThreads];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (i0 + k * kWriteThreads < nt) O.tho[t0 + i0 + k * kWriteThreads] = p0 + v[k];
        }
        for (int j0 = threadIdx.x; j0 < nh; j0 += 4 * kWriteThreads) {
            int v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (j0 + k * kWriteThreads < nh) v[k] = ws_sthits(W)[hb + j0 + k * kWriteThreads];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (j0 + k * kWriteThreads < nh) O.th[p0 + j0 + k * kWriteThreads] = v[k];
        }
    }
}

// Each event's tracks as a CSR of their own (offsets from zero), for callers
// that hand out one event at a time.  Reads only the workspace, so the
// outputs may live in host memory the device can write.
__global__ __launch_bounds__(kWriteThreads) void k_write_events(HitsArgs H, Work W, EventOut O)
{
    for (int e = blockIdx.x; e < H.n_events; e += gridDim.x) {
        const EvInfo I = ws_evinfo(W)[e];
        if (threadIdx.x == 0) {
            O.status[e] = I.st;
            O.hoff[e] = I.out_h;
        }
        const int hb = H.eo[e];
        int32_t *tho = O.tho + I.out_t + e;
        for (int i = threadIdx.x; i <= I.nt; i += kWriteThreads) tho[i] = i < I.nt ? ws_toff(W)[hb + i] : I.nh;
        // four hit ids per lane and pass, their loads in flight together
        for (int j0 = threadIdx.x; j0 < I.nh; j0 += 4 * kWriteThreads) {
            int v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (j0 + k * kWriteThreads < I.nh) v[k] = ws_sthits(W)[hb + j0 + k * kWriteThreads];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (j0 + k * kWriteThreads < I.nh) O.th[I.out_h + j0 + k * kWriteThreads] = v[k];
        }
    }
}

// Consolidation: one workgroup per event, one lane per track.  The lane
// copies the coordinates of its track's hits in track order, then fits
// x(z) and y(z) by unweighted least squares: means, sums centred on the
// means, residuals, each accumulated over the hits in track order (binary32,
// no contraction, correctly rounded division).  A track of up to
// kConsRegHits hits is loaded into registers at once (every load in flight
// together); a longer one is read again from the inputs for each pass.
constexpr int kConsThreads = 256;
constexpr int kConsRegHits = 32;

__device__ __forceinline__ void write_state(float *__restrict__ state, int t, float xm, float ym, float zm, float tx,
                                            float ty, float c2, int n)
{
    float *st = state + 6 * (size_t)t;
    st[0] = xm;
    st[1] = ym;
    st[2] = zm;
    st[3] = tx;
    st[4] = ty;
    st[5] = c2 / (float)(2 * n - 4);
}

__global__ __launch_bounds__(kConsThreads) void k_consolidate(HitsArgs H, const int32_t *__restrict__ eto,
                                                              const int32_t *__restrict__ tho,
                                                              const int32_t *__restrict__ th,
                                                              float *__restrict__ px, float *__restrict__ py,
                                                              float *__restrict__ pz, float *__restrict__ state)
{
    const float *__restrict__ X = H.x;
    const float *__restrict__ Y = H.y;
    const float *__restrict__ Z = H.z;
    for (int e = blockIdx.x; e < H.n_events; e += gridDim.x) {
        const int hb = H.eo[e];
        const int t1 = eto[e + 1];
        for (int t = eto[e] + (int)threadIdx.x; t < t1; t += kConsThreads) {
            const int lo = tho[t], hi = tho[t + 1];
            const int n = hi - lo;
            const float fn = (float)n;
            if (n <= kConsRegHits) {
                int id[kConsRegHits];
                float xs[kConsRegHits], ys[kConsRegHits], zs[kConsRegHits];
#pragma unroll
                for (int j = 0; j < kConsRegHits; ++j)
                    if (j < n) id[j] = hb + th[lo + j];
#pragma unroll
                for (int j = 0; j < kConsRegHits; ++j)
                    if (j < n) {
                        xs[j] = X[id[j]];
                        ys[j] = Y[id[j]];
                        zs[j] = Z[id[j]];
                    }
                float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
                for (int j = 0; j < kConsRegHits; ++j)
                    if (j < n) {
                        px[lo + j] = xs[j];
                        py[lo + j] = ys[j];
                        pz[lo + j] = zs[j];
                        sx = sx + xs[j];
                        sy = sy + ys[j];
                        sz = sz + zs[j];
                    }
                const float xm = sx / fn, ym = sy / fn, zm = sz / fn;
                float szz = 0.0f, sxz = 0.0f, syz = 0.0f;
#pragma unroll
                for (int j = 0; j < kConsRegHits; ++j)
                    if (j < n) {
                        const float dz = zs[j] - zm;
                        szz = szz + dz * dz;
                        sxz = sxz + dz * (xs[j] - xm);
                        syz = syz + dz * (ys[j] - ym);
                    }
                const float tx = sxz / szz, ty = syz / szz;
                float c2 = 0.0f;
#pragma unroll
                for (int j = 0; j < kConsRegHits; ++j)
                    if (j < n) {
                        const float dz = zs[j] - zm;
                        const float rx = xs[j] - (xm + tx * dz);
                        const float ry = ys[j] - (ym + ty * dz);
                        c2 = c2 + ((rx * rx) + (ry * ry));
                    }
                write_state(state, t, xm, ym, zm, tx, ty, c2, n);
                continue;
            }
            float sx = 0.0f, sy = 0.0f, sz = 0.0f;
            for (int k = lo; k < hi; ++k) {
                const int i = hb + th[k];
                const float x = X[i], y = Y[i], z = Z[i];
                px[k] = x;
                py[k] = y;
                pz[k] = z;
                sx = sx + x;
                sy = sy + y;
                sz = sz + z;
            }
            const float xm = sx / fn, ym = sy / fn, zm = sz / fn;
            float szz = 0.0f, sxz = 0.0f, syz = 0.0f;
            for (int k = lo; k < hi; ++k) {
                const int i = hb + th[k];
                const float dz = Z[i] - zm;
                szz = szz + dz * dz;
                sxz = sxz + dz * (X[i] - xm);
                syz = syz + dz * (Y[i] - ym);
            }
            const float tx = sxz / szz, ty = syz / szz;
            float c2 = 0.0f;
            for (int k = lo; k < hi; ++k) {
                const int i = hb + th[k];
                const float dz = Z[i] - zm;
                const float rx = X[i] - (xm + tx * dz);
                const float ry = Y[i] - (ym + ty * dz);
                c2 = c2 + ((rx * rx) + (ry * ry));
            }
            write_state(state, t, xm, ym, zm, tx, ty, c2, n);
        }
    }
}

// debug: copy the sorted phi16 and ids
__global__ void k_copy_sorted(int H, Work W, uint16_t *phi, uint16_t *ids)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < H; i += gridDim.x * blockDim.x) {
        const uint32_t qid = ws_hs(W)[i].qid;
        phi[i] = (uint16_t)(qid & 0xFFFFu);
        ids[i] = (uint16_t)(qid >> 16);
    }
}

// ============================================================== host side

namespace {

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// Lays out the workspace; with base == nullptr only the size is computed.
size_t carve(int32_t E, int32_t H, char *base, Work *W)
{
    const uint32_t h = (uint32_t)(((size_t)(H > 0 ? H : 1) + 255) / 256 * 256);
    const uint32_t e = (uint32_t)(E > 0 ? E : 1);
    if (W) {
        W->base = base;
        W->H = h;
        W->E = e;
    }
    return (size_t)ws_bytes(h, e);
}

bool is_pow_tpe(int v) { return v == 64 || v == 128 || v == 256 || v == 512 || v == 1024; }

// dynamic LDS a workgroup may ask for (gfx950: 160 KiB per compute unit)
constexpr size_t kMaxDynLds = 160 * 1024 - 1024;

int check_hits(const sbt_hits *h)
{
    if (!h) return SBT_ERR_INVALID_ARG;
    if (h->n_events < 0 || h->n_hits < 0) return SBT_ERR_INVALID_ARG;
    if (h->n_events > 0 && (!h->event_offsets || !h->module_offsets)) return SBT_ERR_INVALID_ARG;
    if (h->n_hits > 0 && (!h->x || !h->y || !h->z)) return SBT_ERR_INVALID_ARG;
    return SBT_OK;
}

int check_tracks(const sbt_tracks *t)
{
    if (!t || !t->event_track_offsets || !t->track_hit_offsets || !t->track_hits) return SBT_ERR_INVALID_ARG;
    return SBT_OK;
}

HitsArgs hits_args(const sbt_hits *h)
{
    HitsArgs a;
    a.n_events = h->n_events;
    a.n_hits = h->n_hits;
    a.eo = h->event_offsets;
    a.mo = h->module_offsets;
    a.x = h->x;
    a.y = h->y;
    a.z = h->z;
    a.h16 = nullptr;
    return a;
}

int check_hits_f16(const sbt_hits_f16 *h)
{
    if (!h) return SBT_ERR_INVALID_ARG;
    if (h->n_events < 0 || h->n_hits < 0) return SBT_ERR_INVALID_ARG;
    if (h->n_events > 0 && (!h->event_offsets || !h->module_offsets)) return SBT_ERR_INVALID_ARG;
    if (h->n_hits > 0 && (!h->xyzw || ((uintptr_t)h->xyzw & 7))) return SBT_ERR_INVALID_ARG;
    return SBT_OK;
}

HitsArgs hits_args_f16(const sbt_hits_f16 *h)
{
    HitsArgs a;
    a.n_events = h->n_events;
    a.n_hits = h->n_hits;
    a.eo = h->event_offsets;
    a.mo = h->module_offsets;
    a.x = a.y = a.z = nullptr;
    a.h16 = reinterpret_cast<const uint2 *>(h->xyzw);
    return a;
}

OutArgs out_args(const sbt_tracks *t)
{
    OutArgs o;
    o.eto = t->event_track_offsets;
    o.tho = t->track_hit_offsets;
    o.th = t->track_hits;
    o.status = t->event_status;
    return o;
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        if ((expr) != hipSuccess) return SBT_ERR_HIP;   \
    } while (0)

int launch_plain_front(const sbt_params &P, const HitsArgs &H, const Work &W, hipStream_t s,
                       bool fill_candidates = false)
{
    const dim3 g(H.n_events), b(kPlainThreads);
    const uint32_t lds = lds_bytes(kPlainCap, kPlainOwnCap);
    hipLaunchKernelGGL(k_phi_sort<kPlainThreads>, g, b, lds, s, P, H, W, lds_sortcap(kPlainCap, kPlainOwnCap));
    if (fill_candidates) {
        hipLaunchKernelGGL(k_fill_candidates<kPlainThreads>, g, b, 0, s, P, H, W);
        hipLaunchKernelGGL((k_seed_follow<kPlainThreads, kPlainCap, true>), g, b, lds, s, P, H, W, kPlainOwnCap);
    } else {
        hipLaunchKernelGGL((k_seed_follow<kPlainThreads, kPlainCap, false>), g, b, lds, s, P, H, W, kPlainOwnCap);
    }
    hipLaunchKernelGGL(k_weak_filter<kPlainThreads>, g, b, 0, s, P, H, W);
    hipLaunchKernelGGL(k_compact<kPlainThreads>, g, b, kPlainCompactLds, s, H, W, kPlainCompactLds);
    return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
}

int launch_tail(const HitsArgs &H, const Work &W, const OutArgs &O, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, H, W, O);
    const int grid = std::min(H.n_events, 8192);
    if (grid > 0) hipLaunchKernelGGL(k_write, dim3(grid), dim3(kWriteThreads), 0, s, H, W, O);
    return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
}

// the compiled slot capacity a requested one runs with: the largest not above it
int effective_cap(int requested)
{
    int c = 0;
    for (int i = 0; i < kNumCaps; ++i)
        if (kCaps[i] <= requested) c = kCaps[i];
    return c;
}

// events a workgroup runs side by side (0 reads as 1)
int events_per_block(const sbt_tuning &T) { return T.events_per_block > 1 ? T.events_per_block : 1; }

// lanes of a persistent workgroup
int block_lanes(const sbt_tuning &T) { return T.threads_per_event * events_per_block(T); }

// dynamic LDS of a persistent workgroup: 64-lane events carry their Shared
// block in it, one region per event; wider ones keep it in static LDS
uint32_t tuning_lds(const sbt_tuning &T)
{
    const int cap = effective_cap(T.lds_window_hits);
    if (T.threads_per_event == 64) return (uint32_t)events_per_block(T) * event_region_bytes<64>(cap, T.lds_owner_hits);
    return lds_bytes(cap, T.lds_owner_hits);
}

const void *persistent_kernel(int tpe, int cap)
{
    switch (tpe) {
    case 64: return persistent_kernel_64(cap);
    case 128: return persistent_kernel_128(cap);
    case 256: return persistent_kernel_256(cap);
    case 512: return persistent_kernel_512(cap);
    case 1024: return persistent_kernel_1024(cap);
    default: return nullptr;
    }
}

// The persistent kernel a tuning runs: three or more 512-lane workgroups per
// CU with 448-hit slots take the instance held to six waves per SIMD (with
// the default register budget only two fit a CU).
const void *persistent_fn(const sbt_tuning &T)
{
    const int cap = effective_cap(T.lds_window_hits);
    if (T.threads_per_event == 512 && T.blocks_per_cu >= 3)
        if (const void *fn = persistent_kernel_512_dense(cap)) return fn;
    return persistent_kernel(T.threads_per_event, cap);
}

int device_cus(int *cus)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev));
    return SBT_OK;
}

// Allows dynamic LDS above 64 KiB for a persistent kernel.
int allow_lds(const void *fn, size_t bytes)
{
    if (bytes <= 64 * 1024) return SBT_OK;
    HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return SBT_OK;
}

// resident workgroups per CU of the persistent kernel under a tuning
int persistent_occupancy(const sbt_tuning &T, int *occ)
{
    const void *fn = persistent_fn(T);
    if (!fn) return SBT_ERR_INVALID_ARG;
    const size_t lds = tuning_lds(T);
    if (int rc = allow_lds(fn, lds)) return rc;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, fn, block_lanes(T), lds));
    return SBT_OK;
}

int persistent_grid(const sbt_tuning &T, int n_events, int *grid)
{
    int cus = 0, occ = 0;
    int rc = device_cus(&cus);
    if (rc) return rc;
    if ((rc = persistent_occupancy(T, &occ))) return rc;
    int bpc = std::max(1, std::min(T.blocks_per_cu, std::max(occ, 1)));
    const int epb = events_per_block(T);
    *grid = std::max(1, std::min(cus * bpc, (std::max(n_events, 1) + epb - 1) / epb));
    return SBT_OK;
}

// The configuration of the second pass of a two-pass tuning: the events set
// aside, with slots of deferred_window_hits, on 512 lanes x 2 per CU (1,024
// lanes x 1 above 768-hit slots, which two workgroups per CU cannot hold).
sbt_tuning deferred_tuning(const sbt_tuning &T)
{
    sbt_tuning t = T;
    const bool wide = effective_cap(T.deferred_window_hits) > 768;
    t.threads_per_event = wide ? 1024 : 512;
    t.blocks_per_cu = wide ? 1 : 2;
    t.lds_window_hits = T.deferred_window_hits;
    t.events_per_block = 1;
    t.deferred_window_hits = 0;
    return t;
}

// launch of one persistent pass (defer: set aside the events that do not fit
// the LDS form; only the six-waves instance has that mode)
int launch_pass(const sbt_params &P, const sbt_tuning &T, const HitsArgs &H, const Work &W, hipStream_t s,
                int defer)
{
    int grid = 0;
    int rc = persistent_grid(T, H.n_events, &grid);
    if (rc) return rc;
    const int cap = effective_cap(T.lds_window_hits);
    const uint32_t lds = tuning_lds(T);
    int own_cap = T.lds_owner_hits;
    int sortcap = lds_sortcap(cap, T.lds_owner_hits);
    sbt_params Pc = P;
    HitsArgs Hc = H;
    Work Wc = W;
    // the six-waves instance takes one argument more (defer); the others read
    // the first five
    void *args[] = {&Pc, &Hc, &Wc, &own_cap, &sortcap, &defer};
    HIP_TRY(hipLaunchKernel(persistent_fn(T), dim3(grid), dim3(block_lanes(T)), args, lds, s));
    return SBT_OK;
}

// k_prepare and the persistent kernel: per-event track lists in the workspace.
// A two-pass tuning (deferred_window_hits > 0) runs the six-waves instance
// first, setting aside the events its slots cannot hold, then those events
// on larger slots.
int launch_persistent(const sbt_params &P, const sbt_tuning &T, const HitsArgs &H, const Work &W, hipStream_t s)
{
    hipLaunchKernelGGL(k_prepare, dim3(1), dim3(kOrderThreads), 0, s, H, W);
    if (T.deferred_window_hits <= 0) return launch_pass(P, T, H, W, s, 0);
    if (int rc = launch_pass(P, T, H, W, s, 1)) return rc;
    hipLaunchKernelGGL(k_defer, dim3(1), dim3(kDeferThreads), 0, s, H, W);
    return launch_pass(P, deferred_tuning(T), H, W, s, 0);
}

int launch_batched(const sbt_params &P, const sbt_tuning &T, const HitsArgs &H, const Work &W,
                   const OutArgs &O, hipStream_t s, hipEvent_t *marks)
{
    if (marks) HIP_TRY(hipEventRecord(marks[0], s));
    if (int rc = launch_persistent(P, T, H, W, s)) return rc;
    if (marks) HIP_TRY(hipEventRecord(marks[1], s));
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, H, W, O);
    if (marks) HIP_TRY(hipEventRecord(marks[2], s));
    const int wg = std::min(H.n_events, 8192);
    if (wg > 0) hipLaunchKernelGGL(k_write, dim3(wg), dim3(kWriteThreads), 0, s, H, W, O);
    if (marks) HIP_TRY(hipEventRecord(marks[3], s));
    return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
}

// write an empty result (no events) without launching kernels that need any
__global__ void k_empty(OutArgs O)
{
    if (threadIdx.x == 0) {
        O.eto[0] = 0;
        O.tho[0] = 0;
    }
}

}  // namespace

// ============================================================== C ABI

extern "C" {

const char *sbt_error_string(int code)
{
    switch (code) {
    case SBT_OK: return "ok";
    case SBT_ERR_INVALID_ARG: return "invalid argument";
    case SBT_ERR_EVENT_TOO_LARGE: return "event has more than 65535 hits";
    case SBT_ERR_HIP: return "HIP runtime error";
    case SBT_ERR_WORKSPACE: return "workspace or context too small";
    case SBT_ERR_NOMEM: return "allocation failed";
    case SBT_ERR_NOT_READY: return "not ready";
    default: return "unknown error";
    }
}

int sbt_params_validate(const sbt_params *p)
{
    if (!p) return SBT_ERR_INVALID_ARG;
    if (p->n_modules < 3 || p->n_modules > SBT_MAX_MODULES) return SBT_ERR_INVALID_ARG;
    if (p->max_doublet_candidates < 1) return SBT_ERR_INVALID_ARG;
    if (p->phi_window_seeding < 0 || p->phi_window_seeding > 32767) return SBT_ERR_INVALID_ARG;
    if (p->phi_window_forwarding < 0 || p->phi_window_forwarding > 32767) return SBT_ERR_INVALID_ARG;
    if (p->max_consecutive_misses < 0) return SBT_ERR_INVALID_ARG;
    if (p->reverse != 0 && p->reverse != 1) return SBT_ERR_INVALID_ARG;
    if (p->max_event_hits < 0) return SBT_ERR_INVALID_ARG;
    // nominal z strictly monotone in the module index
    bool inc = true, dec = true;
    for (int k = 1; k < p->n_modules; ++k) {
        if (!(p->module_z[k] > p->module_z[k - 1])) inc = false;
        if (!(p->module_z[k] < p->module_z[k - 1])) dec = false;
    }
    if (!inc && !dec) return SBT_ERR_INVALID_ARG;
    return SBT_OK;
}

int sbt_validate_offsets_host(int32_t M, int32_t E, int32_t H, const int32_t *eo, const int32_t *mo)
{
    if (M < 3 || M > SBT_MAX_MODULES || E < 0 || H < 0) return SBT_ERR_INVALID_ARG;
    if (E > 0 && (!eo || !mo)) return SBT_ERR_INVALID_ARG;
    if (E == 0) return SBT_OK;
    if (eo[0] != 0 || eo[E] != H) return SBT_ERR_INVALID_ARG;
    int too_large = 0;
    for (int32_t e = 0; e < E; ++e) {
        if (eo[e + 1] < eo[e]) return SBT_ERR_INVALID_ARG;
        if (eo[e + 1] - eo[e] > SBT_MAX_EVENT_HITS) too_large = 1;
        const int64_t b = (int64_t)e * M;
        if (mo[b] != eo[e] || mo[b + M] != eo[e + 1]) return SBT_ERR_INVALID_ARG;
        for (int k = 0; k < M; ++k)
            if (mo[b + k + 1] < mo[b + k]) return SBT_ERR_INVALID_ARG;
    }
    return too_large ? SBT_ERR_EVENT_TOO_LARGE : SBT_OK;
}

int sbt_workspace_size(int32_t n_events, int32_t n_hits, size_t *bytes)
{
    if (!bytes || n_events < 0 || n_hits < 0) return SBT_ERR_INVALID_ARG;
    *bytes = carve(n_events, n_hits, nullptr, nullptr);
    return SBT_OK;
}

int sbt_reconstruct(const sbt_params *params, const sbt_hits *hits, sbt_tracks *tracks, void *workspace,
                    size_t workspace_bytes, void *stream)
{
    int rc = sbt_params_validate(params);
    if (rc) return rc;
    if ((rc = check_hits(hits)) || (rc = check_tracks(tracks))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const HitsArgs H = hits_args(hits);
    const OutArgs O = out_args(tracks);
    if (H.n_events == 0) {
        hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s, O);
        return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
    }
    if (!workspace || ((uintptr_t)workspace & 255)) return SBT_ERR_INVALID_ARG;
    if (workspace_bytes < carve(H.n_events, H.n_hits, nullptr, nullptr)) return SBT_ERR_WORKSPACE;
    Work W;
    carve(H.n_events, H.n_hits, (char *)workspace, &W);
    if ((rc = launch_plain_front(*params, H, W, s))) return rc;
    return launch_tail(H, W, O, s);
}

int sbt_debug_reconstruct_fill_candidates(const sbt_params *params, const sbt_hits *hits, sbt_tracks *tracks,
                                          void *workspace, size_t workspace_bytes, void *stream)
{
    int rc = sbt_params_validate(params);
    if (rc) return rc;
    if ((rc = check_hits(hits)) || (rc = check_tracks(tracks))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const HitsArgs H = hits_args(hits);
    const OutArgs O = out_args(tracks);
    if (H.n_events == 0) {
        hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s, O);
        return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
    }
    if (!workspace || ((uintptr_t)workspace & 255)) return SBT_ERR_INVALID_ARG;
    if (workspace_bytes < carve(H.n_events, H.n_hits, nullptr, nullptr)) return SBT_ERR_WORKSPACE;
    Work W;
    carve(H.n_events, H.n_hits, (char *)workspace, &W);
    if ((rc = launch_plain_front(*params, H, W, s, true))) return rc;
    return launch_tail(H, W, O, s);
}

int sbt_debug_phi_sort(const sbt_params *params, const sbt_hits *hits, uint16_t *phi_sorted, uint16_t *ids_sorted,
                       void *workspace, size_t workspace_bytes, void *stream)
{
    int rc = sbt_params_validate(params);
    if (rc) return rc;
    if ((rc = check_hits(hits))) return rc;
    if (!phi_sorted || !ids_sorted) return SBT_ERR_INVALID_ARG;
    if (hits->n_events == 0 || hits->n_hits == 0) return SBT_OK;
    if (!workspace || ((uintptr_t)workspace & 255)) return SBT_ERR_INVALID_ARG;
    if (workspace_bytes < carve(hits->n_events, hits->n_hits, nullptr, nullptr)) return SBT_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Work W;
    carve(hits->n_events, hits->n_hits, (char *)workspace, &W);
    const HitsArgs H = hits_args(hits);
    hipLaunchKernelGGL(k_phi_sort<kPlainThreads>, dim3(H.n_events), dim3(kPlainThreads),
                       lds_bytes(kPlainCap, kPlainOwnCap), s, *params, H, W, lds_sortcap(kPlainCap, kPlainOwnCap));
    hipLaunchKernelGGL(k_copy_sorted, dim3(std::min((H.n_hits + 255) / 256, 4096)), dim3(256), 0, s, H.n_hits, W,
                       phi_sorted, ids_sorted);
    return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
}

int sbt_debug_phi_sort_rank(const sbt_params *params, const sbt_hits *hits, uint16_t *phi_sorted,
                            uint16_t *ids_sorted, void *workspace, size_t workspace_bytes, void *stream)
{
    int rc = sbt_params_validate(params);
    if (rc) return rc;
    if ((rc = check_hits(hits))) return rc;
    if (!phi_sorted || !ids_sorted) return SBT_ERR_INVALID_ARG;
    if (hits->n_events == 0 || hits->n_hits == 0) return SBT_OK;
    if (!workspace || ((uintptr_t)workspace & 255)) return SBT_ERR_INVALID_ARG;
    if (workspace_bytes < carve(hits->n_events, hits->n_hits, nullptr, nullptr)) return SBT_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Work W;
    carve(hits->n_events, hits->n_hits, (char *)workspace, &W);
    const HitsArgs H = hits_args(hits);
    // keys in LDS when the largest event's fit beside the static shared data
    int max_n = 0;
    {
        std::vector<int32_t> eo((size_t)H.n_events + 1);
        HIP_TRY(hipMemcpyAsync(eo.data(), H.eo, 4 * eo.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int32_t e = 0; e < H.n_events; ++e) max_n = std::max(max_n, eo[(size_t)e + 1] - eo[(size_t)e]);
    }
    const size_t lds = 4 * (size_t)max_n;
    if (lds <= 64 * 1024) {
        hipLaunchKernelGGL((k_phi_sort_rank<kPlainThreads, true>), dim3(H.n_events), dim3(kPlainThreads), lds, s,
                           *params, H, W);
    } else {
        hipLaunchKernelGGL((k_phi_sort_rank<kPlainThreads, false>), dim3(H.n_events), dim3(kPlainThreads), 0, s,
                           *params, H, W);
    }
    hipLaunchKernelGGL(k_copy_sorted, dim3(std::min((H.n_hits + 255) / 256, 4096)), dim3(256), 0, s, H.n_hits, W,
                       phi_sorted, ids_sorted);
    return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
}

int sbt_gec_threshold(int32_t n_events, const int32_t *event_offsets, double fraction, int32_t *max_hits)
{
    if (n_events < 0 || !max_hits || !(fraction >= 0.0 && fraction <= 1.0)) return SBT_ERR_INVALID_ARG;
    if (n_events > 0 && !event_offsets) return SBT_ERR_INVALID_ARG;
    const int64_t k = (int64_t)std::floor(fraction * (double)n_events);
    std::vector<int32_t> sizes((size_t)n_events);
    for (int32_t e = 0; e < n_events; ++e) {
        sizes[(size_t)e] = event_offsets[e + 1] - event_offsets[e];
        if (sizes[(size_t)e] < 0) return SBT_ERR_INVALID_ARG;
    }
    if (k >= n_events) {
        *max_hits = 1;
        return SBT_OK;
    }
    // the (k+1)-th largest size: at most k sizes exceed it, k+1 exceed anything smaller
    std::nth_element(sizes.begin(), sizes.begin() + k, sizes.end(), std::greater<int32_t>());
    *max_hits = std::max(1, sizes[(size_t)k]);
    return SBT_OK;
}

int sbt_consolidate(const sbt_hits *hits, const sbt_tracks *tracks, sbt_track_states *out, void *stream)
{
    int rc;
    if ((rc = check_hits(hits)) || (rc = check_tracks(tracks))) return rc;
    if (!out || !out->hit_x || !out->hit_y || !out->hit_z || !out->state) return SBT_ERR_INVALID_ARG;
    if (hits->n_events == 0) return SBT_OK;
    const HitsArgs H = hits_args(hits);
    hipLaunchKernelGGL(k_consolidate, dim3(std::min(H.n_events, 8192)), dim3(kConsThreads), 0, (hipStream_t)stream,
                       H, tracks->event_track_offsets, tracks->track_hit_offsets, tracks->track_hits, out->hit_x,
                       out->hit_y, out->hit_z, out->state);
    return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
}

}  // extern "C"

// ============================================================== context

struct GraphEntry {
    std::vector<uintptr_t> key;
    hipGraphExec_t exec;
    uint64_t last_use;
};

struct sbt_context {
    sbt_params params;
    sbt_tuning tuning;
    int32_t max_events;
    int32_t max_hits;
    void *workspace;
    size_t workspace_bytes;
    Work W;
    std::vector<GraphEntry> graphs;
    uint64_t clock;
    int profiling;
    hipEvent_t marks[4];
    int have_marks;
    int per_launch;   // created without a tuning: chosen per call from the batch's size
    int cus;          // compute units of the device the context was created on
    int64_t captures, replays, evictions, direct;   // graph cache counters
};

namespace {

constexpr size_t kMaxGraphs = 8;

void drop_graphs(sbt_context *c)
{
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
    c->graphs.clear();
}

int valid_tuning(const sbt_tuning &t)
{
    if (!is_pow_tpe(t.threads_per_event)) return SBT_ERR_INVALID_ARG;
    if (t.blocks_per_cu < 1 || t.blocks_per_cu > 16) return SBT_ERR_INVALID_ARG;
    if (t.lds_window_hits < 0 || t.lds_window_hits > 2048) return SBT_ERR_INVALID_ARG;
    if (t.lds_owner_hits < 0 || t.lds_owner_hits > 65536) return SBT_ERR_INVALID_ARG;
    if (t.events_per_block < 0 || t.events_per_block > kMaxEventsPerBlock) return SBT_ERR_INVALID_ARG;
    if (events_per_block(t) > 1 && t.threads_per_event != 64) return SBT_ERR_INVALID_ARG;
    if (tuning_lds(t) > kMaxDynLds) return SBT_ERR_INVALID_ARG;
    if (t.deferred_window_hits < 0 || t.deferred_window_hits > 2048) return SBT_ERR_INVALID_ARG;
    if (t.deferred_window_hits > 0) {
        // a first pass on the six-waves instance, a second on larger slots
        if (t.threads_per_event != 512 || t.blocks_per_cu < 3 || !persistent_kernel_512_dense(effective_cap(t.lds_window_hits)))
            return SBT_ERR_INVALID_ARG;
        if (effective_cap(t.deferred_window_hits) <= effective_cap(t.lds_window_hits)) return SBT_ERR_INVALID_ARG;
        if (tuning_lds(deferred_tuning(t)) > kMaxDynLds) return SBT_ERR_INVALID_ARG;
    }
    return SBT_OK;
}

sbt_tuning default_tuning()
{
    sbt_tuning t;
    t.threads_per_event = 512;
    t.blocks_per_cu = 2;
    t.lds_window_hits = 672;
    t.lds_owner_hits = 16384;
    t.events_per_block = 1;
    t.deferred_window_hits = 0;
    return t;
}

// Launch configuration for a batch of E events and H hits on a device of
// `cus` compute units.  A batch of at most one event per compute unit, or at
// most two large ones (4,000 hits or more on average), runs 1,024 lanes per
// event, one workgroup per CU with 1,536-hit slots: each event then finishes
// sooner, and there are too few events to fill the device twice.  Larger
// batches run 512 lanes, two workgroups per CU; batches of large events take
// 768-hit slots (the largest that still fit two workgroups' LDS on a CU), so
// that their busiest modules stay in LDS rather than in memory.  Batches of
// six or more mid-size events per CU are throughput-bound rather than bound
// by their largest event, and run 512 lanes, three workgroups per CU, with
// 448-hit slots (the instance held to six waves per SIMD): 1.05x the
// throughput of two per CU on 1,536 mu = 7.6 events, 1.16-1.19x on 2,000 to
// 8,000 (1,280: 0.98x); the
// few events with a larger module run from memory, which a long batch hides
// but a batch of 1,000 does not (0.62 ms against 0.45).  Long batches of
// large events (fifteen or more per CU) run the same way in two passes: the
// events whose busiest module exceeds 448 hits (38 % of mu in U{1..25}) are
// set aside and then run with 768-hit slots, two per CU (mu in U{1..25} x
// 10,000: 5.59 ms against 6.03; x 4,000: 2.33 against 2.42; x 2,500: 1.58
// against 1.54, so not below fifteen per CU).  Batches
// of very large events (9,000 hits or more on average) have modules beyond
// the 768-hit slots, and run 1,024 lanes per event with 1,536-hit slots
// whatever their number (mu = 30 x 2,000: 3.72 ms against 4.48 ms).
// Batches of small events (2,500 hits or fewer on average), whose modules
// fit 256-hit slots, run 256 lanes, five workgroups per CU, when there are
// more than two per CU (1,024 events of about 860 hits: 0.20 ms against
// 0.34 ms with 512 lanes x 2 per CU; 2,048: 0.36 against 0.63), and 512
// lanes, two per CU, with 448-hit slots when there are fewer (128 to 512
// such events: 0.17-0.21 ms, about 10 % below 1,024 lanes per event).
sbt_tuning size_tuning(int E, int H, int cus)
{
    sbt_tuning t = default_tuning();
    const bool small = (long long)H <= 2500LL * E;
    const bool large = (long long)H >= 4000LL * E;
    const bool huge = (long long)H >= 9000LL * E;
    if (small) {
        if (E > 2 * cus) {
            t.threads_per_event = 256;
            t.blocks_per_cu = 5;
            t.lds_window_hits = 256;
        } else {
            t.lds_window_hits = 448;
        }
    } else if (E <= cus || (E <= 2 * cus && large) || huge) {
        t.threads_per_event = 1024;
        t.blocks_per_cu = 1;
        t.lds_window_hits = 1536;
    } else if (large && E >= 15 * cus) {
        t.blocks_per_cu = 3;
        t.lds_window_hits = 448;
        t.deferred_window_hits = 768;
    } else if (large) {
        t.lds_window_hits = 768;
    } else if (E >= 6 * cus) {
        t.blocks_per_cu = 3;
        t.lds_window_hits = 448;
    }
    return t;
}

}  // namespace

extern "C" {

int sbt_context_create(const sbt_params *params, const sbt_tuning *tuning, int32_t max_events, int32_t max_hits,
                       sbt_context **out)
{
    int rc = sbt_params_validate(params);
    if (rc) return rc;
    if (!out || max_events < 0 || max_hits < 0) return SBT_ERR_INVALID_ARG;
    sbt_tuning t = tuning ? *tuning : default_tuning();
    if ((rc = valid_tuning(t))) return rc;
    sbt_context *c = new (std::nothrow) sbt_context();
    if (!c) return SBT_ERR_NOMEM;
    c->params = *params;
    c->tuning = t;
    c->max_events = max_events;
    c->max_hits = max_hits;
    c->workspace_bytes = carve(max_events, max_hits, nullptr, nullptr);
    c->clock = 0;
    c->captures = c->replays = c->evictions = c->direct = 0;
    c->profiling = 0;
    c->have_marks = 0;
    c->per_launch = tuning == nullptr;
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            delete c;
            return SBT_ERR_HIP;
        }
    }
    if (hipMalloc(&c->workspace, c->workspace_bytes) != hipSuccess) {
        delete c;
        return SBT_ERR_NOMEM;
    }
    carve(max_events, max_hits, (char *)c->workspace, &c->W);
    for (int i = 0; i < 4; ++i) {
        if (hipEventCreate(&c->marks[i]) != hipSuccess) {
            for (int j = 0; j < i; ++j) (void)hipEventDestroy(c->marks[j]);
            (void)hipFree(c->workspace);
            delete c;
            return SBT_ERR_HIP;
        }
    }
    *out = c;
    return SBT_OK;
}

void sbt_context_destroy(sbt_context *c)
{
    if (!c) return;
    (void)hipDeviceSynchronize();
    drop_graphs(c);
    for (int i = 0; i < 4; ++i) (void)hipEventDestroy(c->marks[i]);
    (void)hipFree(c->workspace);
    delete c;
}

int sbt_context_set_tuning(sbt_context *c, const sbt_tuning *t)
{
    if (!c || !t) return SBT_ERR_INVALID_ARG;
    int rc = valid_tuning(*t);
    if (rc) return rc;
    if (c->per_launch || memcmp(&c->tuning, t, sizeof *t) != 0) {
        c->tuning = *t;
        c->per_launch = 0;
        drop_graphs(c);
    }
    return SBT_OK;
}

int sbt_context_get_tuning(const sbt_context *c, sbt_tuning *out)
{
    if (!c || !out) return SBT_ERR_INVALID_ARG;
    *out = c->per_launch ? size_tuning(c->max_events, c->max_hits, c->cus) : c->tuning;
    return SBT_OK;
}

int sbt_context_set_profiling(sbt_context *c, int32_t on)
{
    if (!c) return SBT_ERR_INVALID_ARG;
    c->profiling = on ? 1 : 0;
    return SBT_OK;
}

int sbt_context_graph_stats(const sbt_context *c, sbt_graph_stats *out)
{
    if (!c || !out) return SBT_ERR_INVALID_ARG;
    out->cached = (int32_t)c->graphs.size();
    out->capacity = (int32_t)kMaxGraphs;
    out->captures = c->captures;
    out->replays = c->replays;
    out->evictions = c->evictions;
    out->direct = c->direct;
    return SBT_OK;
}

int sbt_context_stage_ms(sbt_context *c, float *ms, int32_t n)
{
    if (!c || !ms || n < 1) return SBT_ERR_INVALID_ARG;
    if (!c->have_marks) return SBT_ERR_NOT_READY;
    HIP_TRY(hipEventSynchronize(c->marks[3]));
    for (int i = 0; i < n && i < 3; ++i) HIP_TRY(hipEventElapsedTime(&ms[i], c->marks[i], c->marks[i + 1]));
    return SBT_OK;
}

}  // extern "C"

namespace {

int batched(sbt_context *c, const HitsArgs &H, sbt_tracks *tracks, void *stream)
{
    int rc;
    if ((rc = check_tracks(tracks))) return rc;
    if (H.n_events > c->max_events || H.n_hits > c->max_hits) return SBT_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const OutArgs O = out_args(tracks);
    if (H.n_events == 0) {
        hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s, O);
        return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
    }
    const sbt_tuning T = c->per_launch ? size_tuning(H.n_events, H.n_hits, c->cus) : c->tuning;
    if (c->profiling || s == nullptr) {
        rc = launch_batched(c->params, T, H, c->W, O, s, c->profiling ? c->marks : nullptr);
        if (rc == SBT_OK && c->profiling) c->have_marks = 1;
        if (rc == SBT_OK) ++c->direct;
        return rc;
    }
    std::vector<uintptr_t> key = {
        (uintptr_t)H.n_events, (uintptr_t)H.n_hits, (uintptr_t)H.eo, (uintptr_t)H.mo, (uintptr_t)H.x,
        (uintptr_t)H.y, (uintptr_t)H.z, (uintptr_t)H.h16, (uintptr_t)O.eto, (uintptr_t)O.tho, (uintptr_t)O.th,
        (uintptr_t)O.status};
    ++c->clock;
    for (auto &g : c->graphs) {
        if (g.key == key) {
            g.last_use = c->clock;
            HIP_TRY(hipGraphLaunch(g.exec, s));
            ++c->replays;
            return SBT_OK;
        }
    }
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rc = launch_batched(c->params, T, H, c->W, O, s, nullptr);
    hipError_t ec = hipStreamEndCapture(s, &graph);
    if (rc != SBT_OK || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc ? rc : SBT_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ec != hipSuccess) return SBT_ERR_HIP;
    if (c->graphs.size() >= kMaxGraphs) {
        auto victim = std::min_element(c->graphs.begin(), c->graphs.end(),
                                       [](const GraphEntry &a, const GraphEntry &b) { return a.last_use < b.last_use; });
        (void)hipGraphExecDestroy(victim->exec);
        c->graphs.erase(victim);
        ++c->evictions;
    }
    c->graphs.push_back(GraphEntry{key, exec, c->clock});
    ++c->captures;
    HIP_TRY(hipGraphLaunch(exec, s));
    return SBT_OK;
}

}  // namespace

extern "C" {

int sbt_reconstruct_batched(sbt_context *c, const sbt_hits *hits, sbt_tracks *tracks, void *stream)
{
    if (!c) return SBT_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_hits(hits))) return rc;
    return batched(c, hits_args(hits), tracks, stream);
}

// ---------------------------------------------------------------- no allocation
// The batched sequence with its workspace in a static device array, for
// callers that cannot allocate.  Every GPU the library runs on holds its own
// copy of the array until the process ends.  In host code `scratch` names a
// host-side stand-in, not the device array: its device address is taken once
// per device with hipGetSymbolAddress and only that address is passed on.
// The kernels initialise everything they read (k_prepare resets the work
// counter; every event clears its flags, claims and links before use), so
// nothing is cleared on the host.
}  // extern "C"

static __device__ __align__(256) char scratch[SBT_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices];
int g_scratch_cus[kMaxDevices];

// The device address of the current device's scratch array and its compute
// unit count, looked up on the first call on that device.
int scratch_for_device(char **ptr, int *cus)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return SBT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255)) return SBT_ERR_HIP;
        int n = 0;
        HIP_TRY(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
        g_scratch_cus[dev] = n;
        g_scratch_ptr[dev] = (char *)p;
    }
    *ptr = g_scratch_ptr[dev];
    *cus = g_scratch_cus[dev];
    return SBT_OK;
}

}  // namespace

extern "C" {

int sbt_reconstruct_batched_static(const sbt_params *params, const sbt_hits *hits, sbt_tracks *tracks, void *stream)
{
    int rc = sbt_params_validate(params);
    if (rc) return rc;
    if ((rc = check_hits(hits)) || (rc = check_tracks(tracks))) return rc;
    if (carve(hits->n_events, hits->n_hits, nullptr, nullptr) > (size_t)SBT_STATIC_SCRATCH_BYTES)
        return SBT_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const HitsArgs H = hits_args(hits);
    const OutArgs O = out_args(tracks);
    if (H.n_events == 0) {
        hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, s, O);
        return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
    }
    char *base = nullptr;
    int cus = 0;
    if ((rc = scratch_for_device(&base, &cus))) return rc;
    Work W;
    carve(H.n_events, H.n_hits, base, &W);
    return launch_batched(*params, size_tuning(H.n_events, H.n_hits, cus), H, W, O, s, nullptr);
}

int sbt_reconstruct_batched_f16(sbt_context *c, const sbt_hits_f16 *hits, sbt_tracks *tracks, void *stream)
{
    if (!c) return SBT_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_hits_f16(hits))) return rc;
    return batched(c, hits_args_f16(hits), tracks, stream);
}

int sbt_autotune(sbt_context *c, const sbt_hits *sample, sbt_tracks *tracks, void *stream, int32_t reps,
                 sbt_tuning *best, float *best_ms)
{
    if (!c || reps < 1) return SBT_ERR_INVALID_ARG;
    int rc;
    if ((rc = check_hits(sample)) || (rc = check_tracks(tracks))) return rc;
    if (sample->n_events > c->max_events || sample->n_hits > c->max_hits) return SBT_ERR_WORKSPACE;
    if (sample->n_events == 0) return SBT_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    const HitsArgs H = hits_args(sample);
    const OutArgs O = out_args(tracks);
    hipEvent_t t0, t1;
    HIP_TRY(hipEventCreate(&t0));
    if (hipEventCreate(&t1) != hipSuccess) {
        (void)hipEventDestroy(t0);
        return SBT_ERR_HIP;
    }
    // candidates: lanes per event x LDS slot capacity (x events per
    // workgroup for 64-lane events), each at the largest number of resident
    // workgroups per CU and one less
    struct Cand {
        int tpe, cap, epb, deferred;
    };
    std::vector<Cand> cands;
    for (int tpe : {128, 256, 512, 1024})
        for (int cap : {256, 448, 672, 768, 1024, 1536}) cands.push_back({tpe, cap, 1, 0});
    for (int epb : {2, 4, 8})
        for (int cap : {256, 448}) cands.push_back({64, cap, epb, 0});
    cands.push_back({512, 448, 1, 768});   // two passes: three per CU, then the events set aside
    sbt_tuning win = c->tuning;
    float win_ms = -1.0f;
    rc = SBT_OK;
    for (const Cand &cd : cands) {
        sbt_tuning t = c->tuning;
        t.threads_per_event = cd.tpe;
        t.lds_window_hits = cd.cap;
        t.lds_owner_hits = cd.tpe == 64 ? 4096 : 16384;
        t.events_per_block = cd.epb;
        t.deferred_window_hits = cd.deferred;
        // occupancy of the instance the most workgroups per CU would run
        // (the six-waves one where it exists)
        t.blocks_per_cu = 16;
        if (valid_tuning(t) != SBT_OK) continue;
        int occ = 0;
        if ((rc = persistent_occupancy(t, &occ))) break;
        if (occ < 1) continue;
        for (int bpc = occ; bpc >= 1 && bpc >= occ - 1; --bpc) {
            t.blocks_per_cu = bpc;
            if (valid_tuning(t) != SBT_OK) continue;   // a two-pass tuning needs three per CU
            if ((rc = launch_batched(c->params, t, H, c->W, O, s, nullptr))) break;   // warm-up
            if (hipEventRecord(t0, s) != hipSuccess) { rc = SBT_ERR_HIP; break; }
            for (int r = 0; r < reps && rc == SBT_OK; ++r) rc = launch_batched(c->params, t, H, c->W, O, s, nullptr);
            if (rc) break;
            float ms = 0.0f;
            if (hipEventRecord(t1, s) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
                hipEventElapsedTime(&ms, t0, t1) != hipSuccess) {
                rc = SBT_ERR_HIP;
                break;
            }
            ms /= (float)reps;
            if (win_ms < 0.0f || ms < win_ms) {
                win_ms = ms;
                win = t;
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (rc) return rc;
    sbt_context_set_tuning(c, &win);
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return SBT_OK;
}

}  // extern "C"

// ============================================================== internal API

namespace sbt {

size_t workspace_bytes(int32_t E, int32_t H) { return carve(E, H, nullptr, nullptr); }

int launch_batched_raw(const sbt_params &params, const sbt_tuning &tuning, const sbt_hits &hits,
                       const sbt_tracks &tracks, void *workspace, hipStream_t stream)
{
    const HitsArgs H = hits_args(&hits);
    const OutArgs O = out_args(&tracks);
    if (H.n_events == 0) {
        hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, stream, O);
        return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
    }
    Work W;
    carve(H.n_events, H.n_hits, (char *)workspace, &W);
    return launch_batched(params, tuning, H, W, O, stream, nullptr);
}

namespace {

int batched_events(const sbt_params &params, const sbt_tuning &tuning, const HitsArgs &H, const EventOut &out,
                   void *workspace, hipStream_t stream)
{
    if (H.n_events == 0) return SBT_ERR_INVALID_ARG;
    Work W;
    carve(H.n_events, H.n_hits, (char *)workspace, &W);
    if (int rc = launch_persistent(params, tuning, H, W, stream)) return rc;
    OutArgs O;
    O.eto = out.eto;
    O.tho = nullptr;
    O.th = nullptr;
    O.status = nullptr;
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, stream, H, W, O);
    hipLaunchKernelGGL(k_write_events, dim3(std::min(H.n_events, 8192)), dim3(kWriteThreads), 0, stream, H, W,
                       out);
    return hipGetLastError() == hipSuccess ? SBT_OK : SBT_ERR_HIP;
}

}  // namespace

int launch_batched_events(const sbt_params &params, const sbt_tuning &tuning, const sbt_hits &hits,
                          const EventOut &out, void *workspace, hipStream_t stream)
{
    return batched_events(params, tuning, hits_args(&hits), out, workspace, stream);
}

int launch_batched_events_f16(const sbt_params &params, const sbt_tuning &tuning, const sbt_hits_f16 &hits,
                              const EventOut &out, void *workspace, hipStream_t stream)
{
    return batched_events(params, tuning, hits_args_f16(&hits), out, workspace, stream);
}

sbt_tuning default_tuning_config() { return default_tuning(); }
sbt_tuning batch_tuning(int32_t E, int32_t H, int cus) { return size_tuning(E, H, cus); }
int tuning_valid(const sbt_tuning &t) { return valid_tuning(t); }

}  // namespace sbt
