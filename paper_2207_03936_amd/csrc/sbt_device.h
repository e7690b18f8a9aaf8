// Device-side stages of Search by triplet for gfx950 (wave64).
//
// One event is processed by one workgroup of B lanes.  Every stage is a pure
// function of the event state at the stage start (the paper's barrier between
// seeding and following, Section 3) and every choice is a minimum over unique
// keys, so the parallel evaluation order never changes the result.
//
// Per-event state lives in the workspace, in regions indexed by the event's
// absolute hit offset hb (capacity N = hits of the event):
//   sorted hits   sx, sy, sz, sq (phi16), sid (event-local id)   by sorted position
//   owner         u16 per hit id: 0xFFFF (free) or the key of the track owning it
//   claim         u64 per hit id: minimum claim key of the current stage
//   prev          u16 per hit id: previous hit of the owning track
//   rec           32-byte forming-track records (one per seed; <= N)
// Hit ids, keys and record indices are 16-bit (events hold <= 65,535 hits).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sbt.h"

namespace sbt {

constexpr uint16_t kNone = 0xFFFFu;
constexpr unsigned long long kNoClaim = ~0ull;

// forming-track record
struct Rec {
    float xb, yb, zb;   // last hit
    float tx, ty;       // slope of the last two hits
    uint16_t key;       // id of the seed's middle hit (unique per event)
    uint16_t h0, h1, h2;
    uint16_t last;      // id of the last hit
    uint8_t len;        // hits
    uint8_t last_t;     // traversal index of the last hit
};
static_assert(sizeof(Rec) == 32, "record layout");

// record flags
constexpr uint8_t kFlagSeedClaim = 1;  // claimed its three seed hits this stage
constexpr uint8_t kFlagCandidate = 2;  // tracklet candidate
constexpr uint8_t kFlagAccepted = 4;

struct Work {
    uint16_t *q;        // phi16 by id (sort scratch)
    uint16_t *bucket;   // sort bucket scratch
    float *sx, *sy, *sz;
    uint16_t *sq, *sid;
    uint16_t *owner;
    unsigned long long *claim;
    uint16_t *prev;
    Rec *rec;
    uint16_t *rbest;
    float *rbsc;
    float *rchi2;
    uint8_t *rflag;
    uint16_t *act0, *act1, *fin;
    uint16_t *key2rec;
    uint16_t *st_hits;  // per-event compacted hit ids
    int32_t *st_toff;   // per-event track hit offsets
    int32_t *ev_nt, *ev_nh, *ev_hb, *ev_st, *ev_nfin;
    unsigned int *counter;
};

struct HitsArgs {
    int32_t n_events;
    int32_t n_hits;
    const int32_t *eo;
    const int32_t *mo;
    const float *x, *y, *z;
};

struct OutArgs {
    int32_t *eto;
    int32_t *tho;
    int32_t *th;
    int32_t *status;
};

// ---------------------------------------------------------------- phi16
// Simplified atan2 on 16 bits (Section 3, "Sort by phi"): atan(r), r in
// [0,1], as r * P(r^2) with a degree-4 polynomial fitted in float64 and
// rounded to binary32 (max error 1.2e-5 rad), folded into the full circle and
// scaled by 32768/pi with round-to-nearest-even, so -pi and +pi meet at 0x8000.
__device__ __forceinline__ uint16_t phi16(float x, float y)
{
    const float c0 = 0x1.ffee7ap-1f;
    const float c1 = -0x1.523b6cp-2f;
    const float c2 = 0x1.70f766p-3f;
    const float c3 = -0x1.5ccd12p-4f;
    const float c4 = 0x1.55871cp-6f;
    const float half_pi = 0x1.921fb6p+0f;
    const float pi = 0x1.921fb6p+1f;
    const float scale = 0x1.45f306p+13f;   // 32768 / pi
    float a = x < 0.0f ? -x : x;
    float b = y < 0.0f ? -y : y;
    if (a == 0.0f && b == 0.0f) return 0;
    float mn = a < b ? a : b;
    float mx = a < b ? b : a;
    float r = mn / mx;
    float s = r * r;
    float p = c4;
    p = p * s + c3;
    p = p * s + c2;
    p = p * s + c1;
    p = p * s + c0;
    float at = r * p;
    if (b > a) at = half_pi - at;
    if (x < 0.0f) at = pi - at;
    if (y < 0.0f) at = -at;
    int q = (int)__builtin_rintf(at * scale);
    return (uint16_t)(q & 0xFFFF);
}

// ---------------------------------------------------------------- small helpers
__device__ __forceinline__ int kmod(const sbt_params &P, int t)
{
    return P.reverse ? P.n_modules - 1 - t : t;
}

// largest k in [0, M) with mo[k] <= i (requires mo[0] <= i < mo[M])
__device__ __forceinline__ int module_of(const int *mo, int M, int i)
{
    int lo = 0, hi = M;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (mo[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int lower_bound16(const uint16_t *a, int n, uint16_t v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ unsigned long long claim_key(float score, uint16_t key)
{
    // scores are >= +0, so their binary32 bits order like their values
    return ((unsigned long long)__float_as_uint(score) << 32) | key;
}

// Append under a predicate with one LDS atomic per wave; every lane of the
// wave must call it.  Returns the slot, or -1 where pred is false.
__device__ __forceinline__ int wave_append(bool pred, int *counter)
{
    unsigned long long m = __ballot(pred);
    if (m == 0) return -1;
    int lane = __lane_id();
    int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    int rank = __popcll(m & ((1ull << lane) - 1ull));
    return pred ? base + rank : -1;
}

__device__ __forceinline__ int wave_inclusive_scan(int v)
{
    int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive scan over the workgroup; s_w holds B/64 + 1 ints
template <int B>
__device__ __forceinline__ int block_excl_scan(int v, int *s_w, int *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = wave_inclusive_scan(v);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < B / 64; ++i) {
            int t = s_w[i];
            s_w[i] = acc;
            acc += t;
        }
        s_w[B / 64] = acc;
    }
    __syncthreads();
    int r = s_w[w] + inc - v;
    *total = s_w[B / 64];
    __syncthreads();
    return r;
}

// in-place exclusive scan of a[0..n) in LDS
template <int B>
__device__ void block_scan_inplace(int *a, int n, int *s_w)
{
    const int chunk = (n + B - 1) / B;
    const int beg = threadIdx.x * chunk;
    const int end = beg + chunk < n ? beg + chunk : n;
    int sum = 0;
    for (int i = beg; i < end; ++i) sum += a[i];
    int total;
    int off = block_excl_scan<B>(sum, s_w, &total);
    for (int i = beg; i < end; ++i) {
        int v = a[i];
        a[i] = off;
        off += v;
    }
}

// sort bins: 4096 in total, a power of two per module
__host__ __device__ __forceinline__ int sort_shift(int M)
{
    int bits = 6;                       // M <= 64 -> at least 64 bins per module
    while (bits < 12 && (M << (bits + 1)) <= 4096) ++bits;
    return 16 - bits;
}
constexpr int kSortBins = 4096;

// LDS shared by the stages of one event
template <int B>
struct Shared {
    int mo[SBT_MAX_MODULES + 1];
    int cnt[4];          // records, list[0], list[1], final
    int status;
    int e;
    int scan[B / 64 + 1];
    int hist[kSortBins + 1];
    int fill[kSortBins];
};

// ---------------------------------------------------------------- validation
// Loads the event-local module offsets into LDS and checks the offsets.
template <int B>
__device__ int load_event(const sbt_params &P, const HitsArgs &H, int e, Shared<B> &S,
                          int *hb_out, int *n_out)
{
    const int M = P.n_modules;
    int lo = H.eo[e], hi = H.eo[e + 1];
    if (threadIdx.x == 0) S.status = 0;
    __syncthreads();
    unsigned st = 0;
    if (lo < 0 || hi > H.n_hits || hi < lo) st = SBT_EV_BAD_OFFSETS;
    else if (hi - lo > SBT_MAX_EVENT_HITS) st = SBT_EV_TOO_LARGE;
    if (st == 0) {
        const long long base = (long long)e * M;
        for (int k = threadIdx.x; k <= M; k += B) {
            int v = H.mo[base + k];
            S.mo[k] = v - lo;
            bool bad = (k == 0 && v != lo) || (k == M && v != hi) || v < lo || v > hi;
            if (k > 0 && H.mo[base + k - 1] > v) bad = true;
            if (bad) atomicOr(&S.status, (int)SBT_EV_BAD_OFFSETS);
        }
    } else if (threadIdx.x == 0) {
        S.status = (int)st;
    }
    __syncthreads();
    *hb_out = lo;
    *n_out = hi - lo;
    return S.status;
}

// ---------------------------------------------------------------- sort by phi
// Counting sort on (module, top bits of phi16), then each hit's rank inside
// its bin by counting the bin members with a smaller (phi16, id) key.
template <int B>
__device__ void stage_sort(const sbt_params &P, const HitsArgs &H, const Work &W, int hb, int N,
                           Shared<B> &S)
{
    const int M = P.n_modules;
    const int shift = sort_shift(M);
    const int bpm = 1 << (16 - shift);
    const int nb = M * bpm;
    for (int i = threadIdx.x; i <= nb; i += B) S.hist[i] = 0;
    for (int i = threadIdx.x; i < nb; i += B) S.fill[i] = 0;
    __syncthreads();
    const float *__restrict__ X = H.x + hb;
    const float *__restrict__ Y = H.y + hb;
    const float *__restrict__ Z = H.z + hb;
    uint16_t *__restrict__ q = W.q + hb;
    uint16_t *__restrict__ bucket = W.bucket + hb;
    for (int i = threadIdx.x; i < N; i += B) {
        uint16_t qi = phi16(X[i], Y[i]);
        q[i] = qi;
        int k = module_of(S.mo, M, i);
        atomicAdd(&S.hist[k * bpm + (qi >> shift)], 1);
    }
    __syncthreads();
    block_scan_inplace<B>(S.hist, nb + 1, S.scan);
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += B) {
        uint16_t qi = q[i];
        int bin = module_of(S.mo, M, i) * bpm + (qi >> shift);
        int slot = S.hist[bin] + atomicAdd(&S.fill[bin], 1);
        bucket[slot] = (uint16_t)i;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += B) {
        uint16_t qi = q[i];
        int bin = module_of(S.mo, M, i) * bpm + (qi >> shift);
        int lo = S.hist[bin], hi = S.hist[bin + 1];
        uint32_t key = ((uint32_t)qi << 16) | (uint32_t)i;
        int rank = lo;
        for (int s = lo; s < hi; ++s) {
            uint32_t j = bucket[s];
            uint32_t kj = ((uint32_t)q[j] << 16) | j;
            rank += kj < key;
        }
        W.sx[hb + rank] = X[i];
        W.sy[hb + rank] = Y[i];
        W.sz[hb + rank] = Z[i];
        W.sq[hb + rank] = qi;
        W.sid[hb + rank] = (uint16_t)i;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- seeding
// Seeding(t), t >= 2 (Section 3): modules A = kmod(t-2), Bm = kmod(t-1),
// C = kmod(t).  One lane per middle hit of Bm.
template <int B>
__device__ void stage_seeding(const sbt_params &P, const HitsArgs &H, const Work &W, int hb, int t,
                              Shared<B> &S, uint16_t *nxt, int *n_nxt)
{
    const int A = kmod(P, t - 2), Bm = kmod(P, t - 1), C = kmod(P, t);
    const int a0 = S.mo[A], na = S.mo[A + 1] - a0;
    const int b0 = S.mo[Bm], nbm = S.mo[Bm + 1] - b0;
    const int c0 = S.mo[C], nc = S.mo[C + 1] - c0;
    const float Zc = P.module_z[C];
    const float Ss = P.max_scatter_seeding;
    const int K = P.max_doublet_candidates;
    const uint16_t Ws = (uint16_t)P.phi_window_seeding;
    const uint16_t span = (uint16_t)(2 * P.phi_window_seeding);
    const uint16_t *__restrict__ owner = W.owner + hb;
    const float *sx = W.sx + hb, *sy = W.sy + hb, *sz = W.sz + hb;
    const uint16_t *sq = W.sq + hb, *sid = W.sid + hb;

    for (int base = 0; base < nbm; base += B) {
        const int p1 = base + (int)threadIdx.x;
        bool found = false;
        float bsc = 0.0f;
        uint16_t b0id = kNone, b2id = kNone, id1 = kNone;
        float x0b = 0, y0b = 0, z0b = 0, x2b = 0, y2b = 0, z2b = 0, x1 = 0, y1 = 0, z1 = 0;
        if (p1 < nbm && na > 0) {
            id1 = sid[b0 + p1];
            if (owner[id1] == kNone) {
                x1 = sx[b0 + p1]; y1 = sy[b0 + p1]; z1 = sz[b0 + p1];
                const uint16_t q1 = sq[b0 + p1];
                int s0 = lower_bound16(sq + a0, na, q1);
                if (s0 == na) s0 = 0;
                int got = 0;
                for (int v = 0; v < na && got < K; ++v) {
                    int off = (v & 1) ? -((v + 1) >> 1) : (v >> 1);
                    int pos = s0 + off;
                    if (pos < 0) pos += na;
                    else if (pos >= na) pos -= na;
                    const uint16_t id0 = sid[a0 + pos];
                    if (owner[id0] != kNone) continue;
                    ++got;
                    const float x0 = sx[a0 + pos], y0 = sy[a0 + pos], z0 = sz[a0 + pos];
                    const float d01 = z1 - z0;
                    const float tx = (x1 - x0) / d01;
                    const float ty = (y1 - y0) / d01;
                    const float dzc = Zc - z1;
                    const uint16_t qe = phi16(x1 + tx * dzc, y1 + ty * dzc);
                    if (nc == 0) continue;
                    const uint16_t lo = (uint16_t)(qe - Ws);
                    int st = lower_bound16(sq + c0, nc, lo);
                    if (st == nc) st = 0;
                    for (int j = 0; j < nc; ++j) {
                        int pc = st + j;
                        if (pc >= nc) pc -= nc;
                        const uint16_t qc = sq[c0 + pc];
                        if ((uint16_t)(qc - lo) > span) break;
                        const uint16_t id2 = sid[c0 + pc];
                        if (owner[id2] != kNone) continue;
                        const float x2 = sx[c0 + pc], y2 = sy[c0 + pc], z2 = sz[c0 + pc];
                        const float dz = z2 - z1;
                        const float dx = (x1 + tx * dz) - x2;
                        const float dy = (y1 + ty * dz) - y2;
                        const float sc = (dx * dx) + (dy * dy);
                        if (!(sc < Ss)) continue;
                        if (!found || sc < bsc || (sc == bsc && (id0 < b0id || (id0 == b0id && id2 < b2id)))) {
                            found = true;
                            bsc = sc;
                            b0id = id0; b2id = id2;
                            x0b = x0; y0b = y0; z0b = z0;
                            x2b = x2; y2b = y2; z2b = z2;
                        }
                    }
                }
            }
        }
        const int r = wave_append(found, &S.cnt[0]);
        const int l = wave_append(found, n_nxt);
        if (found) {
            Rec R;
            const float d12 = z2b - z1;
            R.xb = x2b; R.yb = y2b; R.zb = z2b;
            R.tx = (x2b - x1) / d12;
            R.ty = (y2b - y1) / d12;
            R.key = id1; R.h0 = b0id; R.h1 = id1; R.h2 = b2id; R.last = b2id;
            R.len = 3; R.last_t = (uint8_t)t;
            W.rec[hb + r] = R;
            // tracklet fit of the seed, hits in traversal order (Section 3,
            // "Tracklet filter"): chi2 = ((v.x)^2 + (v.y)^2) / (v.v) with
            // v = (z2-z1, z0-z2, z1-z0) orthogonal to (1,1,1) and to z
            const float v0 = z2b - z1, v1 = z0b - z2b, v2 = z1 - z0b;
            const float ssx = ((v0 * x0b) + (v1 * x1)) + (v2 * x2b);
            const float ssy = ((v0 * y0b) + (v1 * y1)) + (v2 * y2b);
            const float n2 = ((v0 * v0) + (v1 * v1)) + (v2 * v2);
            W.rchi2[hb + r] = ((ssx * ssx) + (ssy * ssy)) / n2;
            nxt[l] = (uint16_t)r;
        }
    }
}

// ---------------------------------------------------------------- following
// Search against the flags at stage start, then claim (Section 3, "track
// following"; conflicting claims resolved by minimum (scatter, key)).
template <int B>
__device__ void stage_follow_search(const sbt_params &P, const Work &W, int hb, int t, Shared<B> &S,
                                    const uint16_t *act, int n_act)
{
    const int C = kmod(P, t);
    const int c0 = S.mo[C], nc = S.mo[C + 1] - c0;
    const float Zc = P.module_z[C];
    const float Sf = P.max_scatter_forwarding;
    const uint16_t Wf = (uint16_t)P.phi_window_forwarding;
    const uint16_t span = (uint16_t)(2 * P.phi_window_forwarding);
    uint16_t *__restrict__ owner = W.owner + hb;
    unsigned long long *__restrict__ claim = W.claim + hb;
    const float *sx = W.sx + hb, *sy = W.sy + hb, *sz = W.sz + hb;
    const uint16_t *sq = W.sq + hb, *sid = W.sid + hb;
    for (int a = threadIdx.x; a < n_act; a += B) {
        const int r = act[a];
        const Rec R = W.rec[hb + r];
        uint16_t best = kNone;
        float bsc = 0.0f;
        uint8_t flag = 0;
        bool elig = (t - (int)R.last_t) <= P.max_consecutive_misses + 1;
        if (elig && R.len == 3)
            elig = owner[R.h0] == kNone && owner[R.h1] == kNone && owner[R.h2] == kNone;
        if (elig && nc > 0) {
            const float dzc = Zc - R.zb;
            const uint16_t qe = phi16(R.xb + R.tx * dzc, R.yb + R.ty * dzc);
            const uint16_t lo = (uint16_t)(qe - Wf);
            int st = lower_bound16(sq + c0, nc, lo);
            if (st == nc) st = 0;
            for (int j = 0; j < nc; ++j) {
                int pc = st + j;
                if (pc >= nc) pc -= nc;
                const uint16_t qc = sq[c0 + pc];
                if ((uint16_t)(qc - lo) > span) break;
                const uint16_t id = sid[c0 + pc];
                if (owner[id] != kNone) continue;
                const float dz = sz[c0 + pc] - R.zb;
                const float dx = (R.xb + R.tx * dz) - sx[c0 + pc];
                const float dy = (R.yb + R.ty * dz) - sy[c0 + pc];
                const float sc = (dx * dx) + (dy * dy);
                if (!(sc < Sf)) continue;
                if (best == kNone || sc < bsc || (sc == bsc && id < best)) {
                    best = id;
                    bsc = sc;
                }
            }
            if (best != kNone) {
                const unsigned long long kap = claim_key(bsc, R.key);
                atomicMin(&claim[best], kap);
                if (R.len == 3) {
                    atomicMin(&claim[R.h0], kap);
                    atomicMin(&claim[R.h1], kap);
                    atomicMin(&claim[R.h2], kap);
                    flag = kFlagSeedClaim;
                }
            }
        }
        W.rbest[hb + r] = best;
        W.rbsc[hb + r] = bsc;
        W.rflag[hb + r] = flag;
    }
}

// A track wins iff its key is the minimum on every hit it claimed; winners
// append their best hit and flag their claim set.
template <int B>
__device__ void stage_follow_resolve(const HitsArgs &H, const Work &W, int hb, int t,
                                     const uint16_t *act, int n_act)
{
    uint16_t *__restrict__ owner = W.owner + hb;
    const unsigned long long *__restrict__ claim = W.claim + hb;
    for (int a = threadIdx.x; a < n_act; a += B) {
        const int r = act[a];
        const uint16_t best = W.rbest[hb + r];
        if (best == kNone) continue;
        Rec R = W.rec[hb + r];
        const unsigned long long kap = claim_key(W.rbsc[hb + r], R.key);
        bool win = claim[best] == kap;
        if (R.len == 3) win = win && claim[R.h0] == kap && claim[R.h1] == kap && claim[R.h2] == kap;
        if (!win) continue;
        owner[best] = R.key;
        if (R.len == 3) {
            owner[R.h0] = R.key;
            owner[R.h1] = R.key;
            owner[R.h2] = R.key;
        }
        W.prev[hb + best] = R.last;
        const float xn = H.x[hb + best], yn = H.y[hb + best], zn = H.z[hb + best];
        const float dab = zn - R.zb;
        R.tx = (xn - R.xb) / dab;
        R.ty = (yn - R.yb) / dab;
        R.xb = xn; R.yb = yn; R.zb = zn;
        R.last = best;
        R.len = (uint8_t)(R.len + 1);
        R.last_t = (uint8_t)t;
        W.rec[hb + r] = R;
    }
}

// Clears this stage's claims and moves tracks that missed too many modules
// to the final list.
template <int B>
__device__ void stage_follow_cleanup(const sbt_params &P, const Work &W, int hb, int t, Shared<B> &S,
                                     const uint16_t *act, int n_act, uint16_t *nxt, int *n_nxt)
{
    unsigned long long *__restrict__ claim = W.claim + hb;
    for (int base = 0; base < n_act; base += B) {
        const int a = base + (int)threadIdx.x;
        bool done = false, keep = false;
        int r = 0;
        if (a < n_act) {
            r = act[a];
            const uint16_t best = W.rbest[hb + r];
            const Rec R = W.rec[hb + r];
            if (best != kNone) {
                claim[best] = kNoClaim;
                if (W.rflag[hb + r] & kFlagSeedClaim) {
                    claim[R.h0] = kNoClaim;
                    claim[R.h1] = kNoClaim;
                    claim[R.h2] = kNoClaim;
                }
            }
            done = (t - (int)R.last_t) >= P.max_consecutive_misses + 1;
            keep = !done;
        }
        const int f = wave_append(done, &S.cnt[3]);
        if (done) W.fin[hb + f] = (uint16_t)r;
        const int l = wave_append(keep, n_nxt);
        if (keep) nxt[l] = (uint16_t)r;
    }
}

// Seeding and following over all modules.  Leaves the final record list in
// W.fin and its length in S.cnt[3].
template <int B>
__device__ void stage_track(const sbt_params &P, const HitsArgs &H, const Work &W, int hb, int N,
                            Shared<B> &S)
{
    const int M = P.n_modules;
    for (int i = threadIdx.x; i < N; i += B) {
        W.owner[hb + i] = kNone;
        W.claim[hb + i] = kNoClaim;
        W.key2rec[hb + i] = kNone;
    }
    if (threadIdx.x == 0) {
        S.cnt[0] = 0; S.cnt[1] = 0; S.cnt[2] = 0; S.cnt[3] = 0;
    }
    __syncthreads();
    uint16_t *const l0 = W.act0 + hb;
    uint16_t *const l1 = W.act1 + hb;
    int par = 0;
    stage_seeding<B>(P, H, W, hb, 2, S, l0, &S.cnt[1]);
    __syncthreads();
    for (int t = 3; t < M; ++t) {
        const int n_act = S.cnt[1 + par];
        const uint16_t *act = par ? l1 : l0;
        uint16_t *nxt = par ? l0 : l1;
        if (threadIdx.x == 0) S.cnt[1 + (par ^ 1)] = 0;
        stage_follow_search<B>(P, W, hb, t, S, act, n_act);
        __syncthreads();
        stage_follow_resolve<B>(H, W, hb, t, act, n_act);
        __syncthreads();
        stage_follow_cleanup<B>(P, W, hb, t, S, act, n_act, nxt, &S.cnt[1 + (par ^ 1)]);
        stage_seeding<B>(P, H, W, hb, t, S, nxt, &S.cnt[1 + (par ^ 1)]);
        __syncthreads();
        par ^= 1;
    }
    const int n_act = S.cnt[1 + par];
    const int nf = S.cnt[3];
    const uint16_t *act = par ? l1 : l0;
    for (int a = threadIdx.x; a < n_act; a += B) W.fin[hb + nf + a] = act[a];
    __syncthreads();
    if (threadIdx.x == 0) S.cnt[3] = nf + n_act;
    __syncthreads();
}

// ---------------------------------------------------------------- tracklet filter
// Tracks of >= 4 hits are accepted; a three-hit track is a candidate when its
// fit chi2 is under the threshold and none of its hits is flagged; candidates
// sharing hits keep the one with the minimum (chi2, key).
template <int B>
__device__ void stage_filter(const sbt_params &P, const Work &W, int hb, int n_fin)
{
    const float X = P.max_tracklet_chi2;
    const uint16_t *__restrict__ owner = W.owner + hb;
    unsigned long long *__restrict__ claim = W.claim + hb;
    for (int a = threadIdx.x; a < n_fin; a += B) {
        const int r = W.fin[hb + a];
        const Rec R = W.rec[hb + r];
        uint8_t fl = 0;
        if (R.len >= 4) {
            fl = kFlagAccepted;
        } else {
            const float c2 = W.rchi2[hb + r];
            if (c2 < X && owner[R.h0] == kNone && owner[R.h1] == kNone && owner[R.h2] == kNone) {
                const unsigned long long kap = claim_key(c2, R.key);
                atomicMin(&claim[R.h0], kap);
                atomicMin(&claim[R.h1], kap);
                atomicMin(&claim[R.h2], kap);
                fl = kFlagCandidate;
            }
        }
        W.rflag[hb + r] = fl;
    }
    __syncthreads();
    for (int a = threadIdx.x; a < n_fin; a += B) {
        const int r = W.fin[hb + a];
        uint8_t fl = W.rflag[hb + r];
        const Rec R = W.rec[hb + r];
        if (fl == kFlagCandidate) {
            const unsigned long long kap = claim_key(W.rchi2[hb + r], R.key);
            fl = (claim[R.h0] == kap && claim[R.h1] == kap && claim[R.h2] == kap) ? kFlagAccepted : 0;
        }
        if (fl == kFlagAccepted) W.key2rec[hb + R.key] = (uint16_t)r;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- per-event compaction
// Accepted tracks in key order: per-event track offsets and hit ids into the
// staging arrays, counts into ev_nt / ev_nh.
template <int B>
__device__ void stage_compact(const Work &W, int e, int hb, int N, int *s_scan)
{
    int tcarry = 0, hcarry = 0;
    bool bad = false;
    for (int base = 0; base < N; base += B) {
        const int key = base + (int)threadIdx.x;
        const uint16_t r = key < N ? W.key2rec[hb + key] : kNone;
        Rec R;
        int packed = 0;
        if (r != kNone) {
            R = W.rec[hb + r];
            packed = (1 << 16) | R.len;
        }
        int total;
        const int ex = block_excl_scan<B>(packed, s_scan, &total);
        if (r != kNone) {
            const int ti = tcarry + (ex >> 16);
            const int hi = hcarry + (ex & 0xFFFF);
            // tracks are disjoint, so hi + len <= N; the checks below only
            // keep a broken invariant from turning into a stray access
            if (hi + R.len <= N) {
                W.st_toff[hb + ti] = hi;
                uint16_t *out = W.st_hits + hb + hi;
                uint16_t p = R.last;
                for (int j = R.len - 1; j >= 3; --j) {
                    if (p >= N) { bad = true; break; }
                    out[j] = p;
                    p = W.prev[hb + p];
                }
                out[2] = R.h2;
                out[1] = R.h1;
                out[0] = R.h0;
            } else {
                bad = true;
            }
        }
        tcarry += total >> 16;
        hcarry += total & 0xFFFF;
    }
    if (bad) W.ev_st[e] = (int)SBT_EV_INTERNAL;
    if (threadIdx.x == 0) {
        W.ev_nt[e] = hcarry <= N ? tcarry : 0;
        W.ev_nh[e] = hcarry <= N ? hcarry : 0;
    }
}

}  // namespace sbt
