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
//   owner         one bit per hit id: set once a track has taken the hit (the
//                 method only ever asks whether a hit is flagged; which track
//                 holds it is settled by the claim keys)
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
constexpr uint8_t kFlagCandidate = 2;  // tracklet candidate
constexpr uint8_t kFlagAccepted = 4;

struct Work {
    uint32_t *keys;     // sort keys (phi16 << 16 | id) of events too large for LDS
    float *sx, *sy, *sz;
    uint16_t *sq, *sid;
    uint32_t *owner;    // flag bitmaps; event e's starts at word (hb >> 5) + e
    unsigned long long *claim;
    uint16_t *prev;
    Rec *rec;
    uint32_t *rbest;    // best hit id | window position << 16, or ~0
    float *rbsc;
    float *rchi2;
    uint8_t *rflag;
    uint16_t *act0, *act1, *fin;
    uint16_t *freel;    // unflagged-position lists of modules too large for LDS
    uint16_t *freem;
    uint16_t *frank;
    uint16_t *key2rec;
    uint16_t *st_hits;  // per-event compacted hit ids
    int32_t *st_toff;   // per-event track hit offsets
    int32_t *ev_nt, *ev_nh, *ev_hb, *ev_st, *ev_nfin;
    int32_t *order;     // events, largest first (batched form)
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
// Workgroup barrier that orders LDS accesses only: stores to memory issued
// before it are not waited for.  Used where the next phase reads nothing the
// previous one wrote to memory.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A value every lane of the wave holds alike (read from LDS, for instance),
// moved to a scalar register.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

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

// hit flags: one bit per event-local hit id
__device__ __forceinline__ bool is_free(const uint32_t *own, unsigned id)
{
    return ((own[id >> 5] >> (id & 31u)) & 1u) == 0u;
}

__device__ __forceinline__ void set_flag(uint32_t *own, unsigned id)
{
    atomicOr(&own[id >> 5], 1u << (id & 31u));
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

// Claim key of a stage: (255 - stage) in bits 48..55, the score's binary32
// bits in 16..47 (scores are >= +0, so the bits order like the values) and
// the track key in 0..15.  Within a stage the order is (score, key); a claim
// left from an earlier stage is larger than any claim of a later one, so the
// claim words never need clearing between stages.
__device__ __forceinline__ unsigned long long claim_key(float score, uint16_t key, int stage)
{
    return ((unsigned long long)(255 - stage) << 48) | ((unsigned long long)__float_as_uint(score) << 16) | key;
}
constexpr int kFilterStage = 64;

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
    lds_barrier();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < B / 64; ++i) {
            int t = s_w[i];
            s_w[i] = acc;
            acc += t;
        }
        s_w[B / 64] = acc;
    }
    lds_barrier();
    int r = s_w[w] + inc - v;
    *total = s_w[B / 64];
    lds_barrier();
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

// sort bins: 1024 in total, a power of two per module
constexpr int kSortBins = 1024;
__host__ __device__ __forceinline__ int sort_shift(int M)
{
    int bits = 4;                       // M <= 64 -> at least 16 bins per module
    while (bits < 12 && (M << (bits + 1)) <= kSortBins) ++bits;
    return 16 - bits;
}

// Dynamic LDS of one event workgroup.  The sort scratch (histogram, fill
// counters and the 32-bit sort keys of events with at most sortcap hits)
// aliases the module ring, which is filled only after the sort.
//   ring  4 slots x cap hits: phi16, id, x, y, z (16 B per hit)
//   freel unflagged positions of the seeding stage's doublet module
//   frank rank of each doublet-module position among its unflagged positions
//   tab   coarse phi index of each slot
//   al0/al1, sbest, sbsc  active-track lists and per-stage search results of
//         the first cap active tracks (the rest live in memory)
//   own   hit-flag bitmap of the event when N <= own_cap
struct Lds {
    int cap, own_cap, sortcap;
    uint32_t *keys;
    uint16_t *rq, *rid;
    float *rx, *ry, *rz;
    uint16_t *freel;     // unflagged positions of the doublet module (cap entries)
    uint16_t *freem;     // unflagged positions of the middle module (cap entries)
    uint16_t *frank;     // unflagged positions before each doublet-module position
    uint16_t *tab;       // per slot: first position whose phi16 high byte is >= b, b = 0..256
    uint16_t *al0, *al1; // active track lists (first cap entries)
    uint32_t *sbest;     // per active slot: best hit id | window position << 16
    float *sbsc;         // per active slot: its scatter
    uint32_t *own;
    int *hist, *fill;
};

__host__ __device__ __forceinline__ size_t lds_align(size_t v) { return (v + 15) & ~size_t(15); }

constexpr int kTab = 257;

__host__ __device__ __forceinline__ size_t lds_ring_bytes(int cap)
{
    return lds_align((size_t)4 * cap * 16) + 5 * lds_align((size_t)cap * 2) + lds_align((size_t)4 * kTab * 2) +
           2 * lds_align((size_t)cap * 4);
}

__host__ __device__ __forceinline__ size_t lds_sort_head() { return lds_align((size_t)(2 * kSortBins + 1) * 4); }

__host__ __device__ __forceinline__ size_t lds_bytes(int cap, int own_cap)
{
    const size_t sort = lds_sort_head() + 4 * 1024;   // room for the keys of 1,024 hits at least
    const size_t track = lds_ring_bytes(cap) + lds_align((size_t)((own_cap + 31) / 32) * 4);
    return sort > track ? sort : track;
}

__device__ __forceinline__ Lds carve_lds(char *base, int cap, int own_cap)
{
    Lds L;
    L.cap = cap;
    L.own_cap = own_cap;
    L.sortcap = (int)((lds_bytes(cap, own_cap) - lds_sort_head()) / 4);
    L.keys = (uint32_t *)(base + lds_sort_head());
    const int c4 = 4 * cap;
    L.rx = (float *)base;
    L.ry = L.rx + c4;
    L.rz = L.ry + c4;
    L.rq = (uint16_t *)(L.rz + c4);
    L.rid = L.rq + c4;
    L.freel = (uint16_t *)(base + lds_align((size_t)4 * cap * 16));
    L.freem = (uint16_t *)(base + lds_align((size_t)4 * cap * 16) + lds_align((size_t)cap * 2));
    L.frank = (uint16_t *)(base + lds_align((size_t)4 * cap * 16) + 2 * lds_align((size_t)cap * 2));
    char *p = base + lds_align((size_t)4 * cap * 16) + 3 * lds_align((size_t)cap * 2);
    L.tab = (uint16_t *)p;
    p += lds_align((size_t)4 * kTab * 2);
    L.al0 = (uint16_t *)p;
    p += lds_align((size_t)cap * 2);
    L.al1 = (uint16_t *)p;
    p += lds_align((size_t)cap * 2);
    L.sbest = (uint32_t *)p;
    p += lds_align((size_t)cap * 4);
    L.sbsc = (float *)p;
    L.own = (uint32_t *)(base + lds_ring_bytes(cap));
    L.hist = (int *)base;
    L.fill = L.hist + kSortBins + 1;
    return L;
}

// static LDS shared by the stages of one event
template <int B>
struct Shared {
    int mo[SBT_MAX_MODULES + 1];
    int cnt[4];          // records, list[0], list[1], final
    int status;
    int e;
    int scan[B / 64 + 1];
    int slot_n[4];       // hits of the module held by each ring slot
    int maxmod;          // hits of the event's largest module
};

// ---------------------------------------------------------------- validation
// Loads the event-local module offsets into LDS and checks the offsets.
template <int B>
__device__ int load_event(const sbt_params &P, const HitsArgs &H, int e, Shared<B> &S,
                          int *hb_out, int *n_out)
{
    const int M = P.n_modules;
    int lo = H.eo[e], hi = H.eo[e + 1];
    if (threadIdx.x == 0) {
        S.status = 0;
        S.maxmod = 0;
    }
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
            if (k < M) atomicMax(&S.maxmod, H.mo[base + k + 1] - v);
        }
    } else if (threadIdx.x == 0) {
        S.status = (int)st;
    }
    __syncthreads();
    *hb_out = uni(lo);
    *n_out = uni(hi - lo);
    return uni(S.status);
}

// ---------------------------------------------------------------- sort by phi
// Counting sort on (module, top bits of phi16) into buckets of 32-bit keys
// phi16 << 16 | id, then each key's rank inside its bucket by counting the
// smaller keys of the bucket; ties in phi16 fall to the lower id because the
// id is the key's low half.
template <int B>
__device__ void stage_sort(const sbt_params &P, const HitsArgs &H, const Work &W, int hb, int N,
                           Shared<B> &S, const Lds &L)
{
    const int M = P.n_modules;
    const int shift = sort_shift(M);
    const int bpm = 1 << (16 - shift);
    const int nb = M * bpm;
    int *hist = L.hist, *fill = L.fill;
    uint32_t *keys = N <= L.sortcap ? L.keys : W.keys + hb;
    for (int i = threadIdx.x; i <= nb; i += B) hist[i] = 0;
    for (int i = threadIdx.x; i < nb; i += B) fill[i] = 0;
    __syncthreads();
    const float *__restrict__ X = H.x + hb;
    const float *__restrict__ Y = H.y + hb;
    const float *__restrict__ Z = H.z + hb;
    for (int i = threadIdx.x; i < N; i += B) {
        const uint16_t qi = phi16(X[i], Y[i]);
        atomicAdd(&hist[module_of(S.mo, M, i) * bpm + (qi >> shift)], 1);
    }
    __syncthreads();
    block_scan_inplace<B>(hist, nb + 1, S.scan);
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += B) {
        const uint16_t qi = phi16(X[i], Y[i]);
        const int bin = module_of(S.mo, M, i) * bpm + (qi >> shift);
        keys[hist[bin] + atomicAdd(&fill[bin], 1)] = ((uint32_t)qi << 16) | (uint32_t)i;
    }
    __syncthreads();
    for (int s = threadIdx.x; s < N; s += B) {
        const uint32_t key = keys[s];
        const int i = (int)(key & 0xFFFFu);
        const uint16_t qi = (uint16_t)(key >> 16);
        const int bin = module_of(S.mo, M, i) * bpm + (qi >> shift);
        const int lo = hist[bin], hi = hist[bin + 1];
        int rank = lo;
        for (int m = lo; m < hi; ++m) rank += keys[m] < key;
        W.sx[hb + rank] = X[i];
        W.sy[hb + rank] = Y[i];
        W.sz[hb + rank] = Z[i];
        W.sq[hb + rank] = qi;
        W.sid[hb + rank] = (uint16_t)i;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- module windows
// An event whose modules all fit the LDS slots (and whose hit flags fit the
// LDS bitmap) runs the LDS instantiation of the tracking stages: traversal
// index u lives in ring slot u & 3 and every window access is an LDS access.
// Any other event runs the memory instantiation, which reads the sorted
// arrays in memory directly.  Both compute the same thing.
struct Win {
    const uint16_t *q, *id;
    const float *x, *y, *z;
    const uint16_t *tab;   // coarse index (LDS instantiation)
    int n;
};

// first position of the window whose phi16 is >= v
template <bool kLds>
__device__ __forceinline__ int win_lower_bound(const Win &w, uint16_t v)
{
    if (kLds) {
        int p = w.tab[v >> 8];
        const int end = w.tab[(v >> 8) + 1];
        while (p < end && w.q[p] < v) ++p;
        return p;
    }
    return lower_bound16(w.q, w.n, v);
}

template <int B, bool kLds>
__device__ __forceinline__ Win window(const sbt_params &P, const Lds &L, const Shared<B> &S, const Work &W, int hb,
                                      int u)
{
    Win w;
    if (kLds) {
        const int s = u & 3;
        const int o = s * L.cap;
        w.n = uni(S.slot_n[s]);
        w.q = L.rq + o; w.id = L.rid + o; w.x = L.rx + o; w.y = L.ry + o; w.z = L.rz + o;
        w.tab = L.tab + s * kTab;
    } else {
        const int k = kmod(P, u);
        const int g0 = uni(S.mo[k]);
        w.n = uni(S.mo[k + 1]) - g0;
        const int g = hb + g0;
        w.q = W.sq + g; w.id = W.sid + g; w.x = W.sx + g; w.y = W.sy + g; w.z = W.sz + g;
        w.tab = nullptr;
    }
    return w;
}

// registers holding one module on its way into the ring
template <int B>
struct RingStage {
    static constexpr int PF = (512 + B - 1) / B;
    uint16_t q[PF], qp[PF], id[PF];
    float x[PF], y[PF], z[PF];
};

// coarse-index entries owned by position i of an n-hit slot whose phi16 is
// q (qp: phi16 of position i-1): every high byte b with
// high(qp) < b <= high(q) starts at i; the last position also closes the
// table with n
__device__ __forceinline__ void tab_fill(uint16_t *tab, int i, int n, uint16_t q, uint16_t qp)
{
    const int b_lo = i == 0 ? 0 : (qp >> 8) + 1;
    const int b_hi = q >> 8;
    for (int b = b_lo; b <= b_hi; ++b) tab[b] = (uint16_t)i;
    if (i == n - 1)
        for (int b = b_hi + 1; b < kTab; ++b) tab[b] = (uint16_t)n;
}

template <int B>
__device__ __forceinline__ void ring_load(const sbt_params &P, const Work &W, int hb, int u, const Shared<B> &S,
                                          const Lds &L, RingStage<B> &R)
{
    const int k = kmod(P, u);
    const int g = uni(S.mo[k]), n = uni(S.mo[k + 1]) - g;
#pragma unroll
    for (int j = 0; j < RingStage<B>::PF; ++j) {
        const int i = (int)threadIdx.x + j * B;
        if (i < n) {
            R.q[j] = W.sq[hb + g + i];
            R.qp[j] = i > 0 ? W.sq[hb + g + i - 1] : (uint16_t)0;
            R.id[j] = W.sid[hb + g + i];
            R.x[j] = W.sx[hb + g + i];
            R.y[j] = W.sy[hb + g + i];
            R.z[j] = W.sz[hb + g + i];
        }
    }
}

template <int B>
__device__ __forceinline__ void ring_store(const sbt_params &P, const Work &W, int hb, int u, Shared<B> &S,
                                           const Lds &L, const RingStage<B> &R)
{
    const int k = kmod(P, u);
    const int g = uni(S.mo[k]), n = uni(S.mo[k + 1]) - g;
    const int s = u & 3;
    if (threadIdx.x == 0) S.slot_n[s] = n;
    const int o = s * L.cap;
    uint16_t *tab = L.tab + s * kTab;
    if (n == 0)
        for (int b = threadIdx.x; b < kTab; b += B) tab[b] = 0;
#pragma unroll
    for (int j = 0; j < RingStage<B>::PF; ++j) {
        const int i = (int)threadIdx.x + j * B;
        if (i < n) {
            L.rq[o + i] = R.q[j];
            L.rid[o + i] = R.id[j];
            L.rx[o + i] = R.x[j];
            L.ry[o + i] = R.y[j];
            L.rz[o + i] = R.z[j];
            tab_fill(tab, i, n, R.q[j], R.qp[j]);
        }
    }
    for (int i = (int)threadIdx.x + RingStage<B>::PF * B; i < n; i += B) {
        const uint16_t q = W.sq[hb + g + i];
        L.rq[o + i] = q;
        L.rid[o + i] = W.sid[hb + g + i];
        L.rx[o + i] = W.sx[hb + g + i];
        L.ry[o + i] = W.sy[hb + g + i];
        L.rz[o + i] = W.sz[hb + g + i];
        tab_fill(tab, i, n, q, W.sq[hb + g + i - 1]);
    }
}

// ---------------------------------------------------------------- active lists
// A list of record indices whose first cap entries live in LDS and the rest
// in memory (cap = 0 in the memory instantiation).
struct AList {
    uint16_t *lds, *mem;
    int cap;
    __device__ __forceinline__ uint16_t get(int a) const { return a < cap ? lds[a] : mem[a]; }
    __device__ __forceinline__ void put(int a, uint16_t v) const
    {
        if (a < cap) lds[a] = v;
        else mem[a] = v;
    }
};

// ---------------------------------------------------------------- seeding
// The pendulum search visits the doublet module's phi-sorted positions in
// the order s0, s0-1, s0+1, s0-2, s0+2, ... (wrapping, at most n visits) and
// keeps the first K unflagged ones.  Here the unflagged positions are first
// compacted in order; the K kept ones are then the K of smallest visit rank
// (offset o >= 0 -> 2o, o < 0 -> -2o-1), found by merging the walks up and
// down from s0 through the compacted list.  Returns the position of the
// c-th kept partner, or -1.
__device__ __forceinline__ int pendulum_pick(const uint16_t *F, int nf, int j, int s0, int na, int hu, int hd, int c)
{
    int su = 0, sd = 0, pos = -1;
    for (int step = 0; step <= c; ++step) {
        int vu = 0x7fffffff, vd = 0x7fffffff, pu = 0, pd = 0;
        if (su < nf) {
            int ix = j + su;
            if (ix >= nf) ix -= nf;
            pu = F[ix];
            int o = pu - s0;
            if (o < 0) o += na;
            if (o <= hu) vu = 2 * o;
        }
        if (sd < nf) {
            int ix = j - 1 - sd;
            if (ix < 0) ix += nf;
            pd = F[ix];
            int o = s0 - pd;
            if (o < 0) o += na;
            if (o >= 1 && o <= hd) vd = 2 * o - 1;
        }
        if (vu == 0x7fffffff && vd == 0x7fffffff) return -1;
        if (vd == 0x7fffffff || vu < vd) { pos = pu; ++su; }
        else { pos = pd; ++sd; }
    }
    return pos;
}

// best third hit for one doublet (h0 at wa position pos, h1 = middle hit)
struct SeedBest {
    float sc;
    uint16_t id0, id2;
    int pos0, pos2;
    bool found;
};

__device__ __forceinline__ bool seed_better(const SeedBest &a, const SeedBest &b)
{
    if (a.found != b.found) return a.found;
    if (!a.found) return false;
    if (a.sc != b.sc) return a.sc < b.sc;
    if (a.id0 != b.id0) return a.id0 < b.id0;
    return a.id2 < b.id2;
}

template <bool kLds>
__device__ __forceinline__ void seed_doublet(const Win &wa, const Win &wc, const uint32_t *own, int pos0, float x1,
                                             float y1, float z1, float Zc, float Ss, uint16_t Ws, uint16_t span,
                                             SeedBest &b)
{
    const uint16_t id0 = wa.id[pos0];
    const float x0 = wa.x[pos0], y0 = wa.y[pos0], z0 = wa.z[pos0];
    const float d01 = z1 - z0;
    const float tx = (x1 - x0) / d01;
    const float ty = (y1 - y0) / d01;
    const float dzc = Zc - z1;
    const uint16_t qe = phi16(x1 + tx * dzc, y1 + ty * dzc);
    const int nc = wc.n;
    if (nc == 0) return;
    const uint16_t lo = (uint16_t)(qe - Ws);
    int st = win_lower_bound<kLds>(wc, lo);
    if (st == nc) st = 0;
    for (int jj = 0; jj < nc; ++jj) {
        int pc = st + jj;
        if (pc >= nc) pc -= nc;
        const uint16_t qc = wc.q[pc];
        if ((uint16_t)(qc - lo) > span) break;
        const uint16_t id2 = wc.id[pc];
        if (!is_free(own, id2)) continue;
        const float dz = wc.z[pc] - z1;
        const float dx = (x1 + tx * dz) - wc.x[pc];
        const float dy = (y1 + ty * dz) - wc.y[pc];
        const float sc = (dx * dx) + (dy * dy);
        if (!(sc < Ss)) continue;
        if (!b.found || sc < b.sc || (sc == b.sc && (id0 < b.id0 || (id0 == b.id0 && id2 < b.id2)))) {
            b.found = true;
            b.sc = sc;
            b.id0 = id0;
            b.id2 = id2;
            b.pos0 = pos0;
            b.pos2 = pc;
        }
    }
}

// ---------------------------------------------------------------- following search
// Following search of one forming track into traversal index u (Section 3,
// "track following"): the last two hits extrapolated to the module's
// nominal z, the best unflagged hit of the inclusive phi window by
// (scatter, id) under the threshold, and claims on that hit (and on the
// three seed hits of a bare seed) keyed (scatter, key) for stage u.
// Returns the best hit's id | window position << 16, or ~0.
template <bool kLds>
__device__ __forceinline__ uint32_t follow_item(const sbt_params &P, const Win &wc, float Zc, const uint32_t *own,
                                                unsigned long long *claim, const Rec &R, int u, float &bsc_out)
{
    const float Sf = P.max_scatter_forwarding;
    const uint16_t Wf = (uint16_t)P.phi_window_forwarding;
    const uint16_t span = (uint16_t)(2 * P.phi_window_forwarding);
    const int nc = wc.n;
    uint16_t best = kNone;
    int bpos = 0;
    float bsc = 0.0f;
    bool elig = (u - (int)R.last_t) <= P.max_consecutive_misses + 1;
    if (elig && R.len == 3) elig = is_free(own, R.h0) && is_free(own, R.h1) && is_free(own, R.h2);
    if (elig && nc > 0) {
        const float dzc = Zc - R.zb;
        const uint16_t qe = phi16(R.xb + R.tx * dzc, R.yb + R.ty * dzc);
        const uint16_t lo = (uint16_t)(qe - Wf);
        int st = win_lower_bound<kLds>(wc, lo);
        if (st == nc) st = 0;
        for (int j = 0; j < nc; ++j) {
            int pc = st + j;
            if (pc >= nc) pc -= nc;
            const uint16_t qc = wc.q[pc];
            if ((uint16_t)(qc - lo) > span) break;
            const uint16_t id = wc.id[pc];
            if (!is_free(own, id)) continue;
            const float dz = wc.z[pc] - R.zb;
            const float dx = (R.xb + R.tx * dz) - wc.x[pc];
            const float dy = (R.yb + R.ty * dz) - wc.y[pc];
            const float sc = (dx * dx) + (dy * dy);
            if (!(sc < Sf)) continue;
            if (best == kNone || sc < bsc || (sc == bsc && id < best)) {
                best = id;
                bpos = pc;
                bsc = sc;
            }
        }
        if (best != kNone) {
            const unsigned long long kap = claim_key(bsc, R.key, u);
            atomicMin(&claim[best], kap);
            if (R.len == 3) {
                atomicMin(&claim[R.h0], kap);
                atomicMin(&claim[R.h1], kap);
                atomicMin(&claim[R.h2], kap);
            }
        }
    }
    bsc_out = bsc;
    return best == kNone ? 0xFFFFFFFFu : ((uint32_t)bpos << 16) | best;
}

// search result of active slot a (record r): LDS for the first cap slots
__device__ __forceinline__ void put_result(const Lds &L, const Work &W, int hb, int cap, int a, int r, uint32_t pb,
                                           float bsc)
{
    if (a < cap) {
        L.sbest[a] = pb;
        L.sbsc[a] = bsc;
    } else {
        W.rbest[hb + r] = pb;
        W.rbsc[hb + r] = bsc;
    }
}

// Seeding(t), t >= 2 (Section 3), fused with the following search into
// t+1.  Seeding: modules A = kmod(t-2), Bm = kmod(t-1), C = kmod(t); work
// items are (unflagged middle hit, partner rank c) -- with K a power of two
// up to 16, the K doublets of a middle hit run on K adjacent lanes and their
// best triplets are reduced with lane shuffles, otherwise one lane handles
// all K.  A new seed's following search into t+1 runs on the lane that made
// it.  The tracks kept by the last resolution (active slots [0, n_keep))
// search t+1 on waves of their own.  Both read the flags as the resolution
// of t left them, which is the state the following of t+1 starts from.
template <int B, bool kLds>
__device__ void stage_seed_follow(const sbt_params &P, const Work &W, int hb, int t, Shared<B> &S, const Lds &L,
                                  const uint32_t *own, const AList &nxt, int *n_nxt, int n_keep, bool follow_next)
{
    const Win wa = window<B, kLds>(P, L, S, W, hb, t - 2);
    const Win wb = window<B, kLds>(P, L, S, W, hb, t - 1);
    const Win wc = window<B, kLds>(P, L, S, W, hb, t);
    Win wn = wc;
    float Zn = 0.0f;
    if (follow_next) {
        wn = window<B, kLds>(P, L, S, W, hb, t + 1);
        Zn = P.module_z[kmod(P, t + 1)];
    }
    unsigned long long *__restrict__ claim = W.claim + hb;
    const int na = wa.n, nbm = wb.n;
    const float Zc = P.module_z[kmod(P, t)];
    const float Ss = P.max_scatter_seeding;
    const int K = P.max_doublet_candidates;
    const uint16_t Ws = (uint16_t)P.phi_window_seeding;
    const uint16_t span = (uint16_t)(2 * P.phi_window_seeding);

    // unflagged positions of the doublet module and of the middle module, ascending
    uint16_t *F, *FR, *FM;
    if (kLds) {
        F = L.freel; FR = L.frank; FM = L.freem;
    } else {
        const int ga = hb + uni(S.mo[kmod(P, t - 2)]), gb = hb + uni(S.mo[kmod(P, t - 1)]);
        F = W.freel + ga; FR = W.frank + ga; FM = W.freem + gb;
    }
    int nf = 0, nfm = 0;
    const int nmax = na > nbm ? na : nbm;
    for (int base = 0; base < nmax; base += B) {
        const int p = base + (int)threadIdx.x;
        const bool fa = p < na && is_free(own, wa.id[p]);
        const bool fb = p < nbm && is_free(own, wb.id[p]);
        int total;
        const int idx = block_excl_scan<B>((fa ? 1 : 0) | (fb ? 0x10000 : 0), S.scan, &total);
        if (p < na) FR[p] = (uint16_t)(nf + (idx & 0xFFFF));
        if (fa) F[nf + (idx & 0xFFFF)] = (uint16_t)p;
        if (fb) FM[nfm + (idx >> 16)] = (uint16_t)p;
        nf += total & 0xFFFF;
        nfm += total >> 16;
    }
    // the lists are in LDS in the LDS instantiation, in memory otherwise
    if (kLds) lds_barrier();
    else __syncthreads();
    const int hd = na >> 1, hu = na - hd - 1;   // offsets visited: [-hd, hu]
    const int G = (K == 1 || K == 2 || K == 4 || K == 8 || K == 16) ? K : 1;
    const int per_lane = G == 1 ? K : 1;
    const int seed_items = (nf > 0 && nfm > 0) ? nfm * G : 0;
    const int seed_pad = (seed_items + 63) & ~63;      // seeding and following never share a wave
    const int follow_items = follow_next ? n_keep : 0;
    const int total = seed_pad + follow_items;

    for (int base = 0; base < total; base += B) {
        const int g = base + (int)threadIdx.x;
        const int g_wave = uni(base + ((int)threadIdx.x & ~63));
        if (g_wave >= seed_pad) {
            const int a = g - seed_pad;
            if (a < follow_items) {
                const int r = nxt.get(a);
                const Rec R = W.rec[hb + r];
                float bsc;
                const uint32_t pb = follow_item<kLds>(P, wn, Zn, own, claim, R, t + 1, bsc);
                put_result(L, W, hb, nxt.cap, a, r, pb, bsc);
            }
            continue;
        }
        const int i = g / G, c = g - i * G;
        SeedBest best;
        best.found = false;
        best.sc = 0.0f;
        best.id0 = kNone;
        best.id2 = kNone;
        best.pos0 = 0;
        best.pos2 = 0;
        int p1 = 0;
        float x1 = 0.0f, y1 = 0.0f, z1 = 0.0f;
        if (g < seed_items) {
            p1 = FM[i];
            x1 = wb.x[p1]; y1 = wb.y[p1]; z1 = wb.z[p1];
            int s0 = win_lower_bound<kLds>(wa, wb.q[p1]);
            if (s0 == na) s0 = 0;
            const int j = FR[s0];   // first unflagged position >= s0, as an index into F
            for (int cc = 0; cc < per_lane; ++cc) {
                const int pos0 = pendulum_pick(F, nf, j, s0, na, hu, hd, c + cc);
                if (pos0 < 0) break;
                seed_doublet<kLds>(wa, wc, own, pos0, x1, y1, z1, Zc, Ss, Ws, span, best);
            }
        }
        // minimum over the G lanes of a middle hit
        for (int m = 1; m < G; m <<= 1) {
            SeedBest o;
            o.found = __shfl_xor((int)best.found, m) != 0;
            o.sc = __shfl_xor(best.sc, m);
            o.id0 = (uint16_t)__shfl_xor((int)best.id0, m);
            o.id2 = (uint16_t)__shfl_xor((int)best.id2, m);
            o.pos0 = __shfl_xor(best.pos0, m);
            o.pos2 = __shfl_xor(best.pos2, m);
            if (seed_better(o, best)) best = o;
        }
        const bool emit = best.found && c == 0 && g < seed_items;
        const int r = wave_append(emit, &S.cnt[0]);
        const int l = wave_append(emit, n_nxt);
        if (emit) {
            const float x0b = wa.x[best.pos0], y0b = wa.y[best.pos0], z0b = wa.z[best.pos0];
            const float x2b = wc.x[best.pos2], y2b = wc.y[best.pos2], z2b = wc.z[best.pos2];
            const uint16_t id1 = wb.id[p1];
            Rec R;
            const float d12 = z2b - z1;
            R.xb = x2b; R.yb = y2b; R.zb = z2b;
            R.tx = (x2b - x1) / d12;
            R.ty = (y2b - y1) / d12;
            R.key = id1; R.h0 = best.id0; R.h1 = id1; R.h2 = best.id2; R.last = best.id2;
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
            nxt.put(l, (uint16_t)r);
            if (follow_next) {
                float bsc;
                const uint32_t pb = follow_item<kLds>(P, wn, Zn, own, claim, R, t + 1, bsc);
                put_result(L, W, hb, nxt.cap, l, r, pb, bsc);
            }
        }
    }
}

// A track wins iff its key is the minimum on every hit it claimed; winners
// append their best hit and flag their claim set.  Tracks that have now missed
// more than max_consecutive_misses modules in a row become final; the others
// stay active for the next module.
template <int B, bool kLds>
__device__ void stage_follow_resolve(const sbt_params &P, const Work &W, int hb, int t, Shared<B> &S,
                                     const Lds &L, uint32_t *own, const AList &act, int n_act, const AList &nxt,
                                     int *n_nxt)
{
    const Win wc = window<B, kLds>(P, L, S, W, hb, t);
    const unsigned long long *__restrict__ claim = W.claim + hb;
    for (int base = 0; base < n_act; base += B) {
        const int a = base + (int)threadIdx.x;
        bool done = false, keep = false;
        int r = 0;
        if (a < n_act) {
            r = act.get(a);
            const bool in_lds = a < act.cap;
            const uint32_t pb = in_lds ? L.sbest[a] : W.rbest[hb + r];
            Rec R = W.rec[hb + r];
            int last_t = R.last_t;
            if (pb != 0xFFFFFFFFu) {
                const uint16_t best = (uint16_t)(pb & 0xFFFF);
                const int bpos = (int)(pb >> 16);
                const unsigned long long kap = claim_key(in_lds ? L.sbsc[a] : W.rbsc[hb + r], R.key, t);
                bool win = claim[best] == kap;
                if (R.len == 3) win = win && claim[R.h0] == kap && claim[R.h1] == kap && claim[R.h2] == kap;
                if (win) {
                    set_flag(own, best);
                    if (R.len == 3) {
                        set_flag(own, R.h0);
                        set_flag(own, R.h1);
                        set_flag(own, R.h2);
                    }
                    W.prev[hb + best] = R.last;
                    const float xn = wc.x[bpos], yn = wc.y[bpos], zn = wc.z[bpos];
                    const float dab = zn - R.zb;
                    R.tx = (xn - R.xb) / dab;
                    R.ty = (yn - R.yb) / dab;
                    R.xb = xn; R.yb = yn; R.zb = zn;
                    R.last = best;
                    R.len = (uint8_t)(R.len + 1);
                    R.last_t = (uint8_t)t;
                    W.rec[hb + r] = R;
                    last_t = t;
                }
            }
            done = (t - last_t) >= P.max_consecutive_misses + 1;
            keep = !done;
        }
        const int f = wave_append(done, &S.cnt[3]);
        if (done) W.fin[hb + f] = (uint16_t)r;
        const int l = wave_append(keep, n_nxt);
        if (keep) nxt.put(l, (uint16_t)r);
    }
}

// The owner flags of an event: in LDS when the event fits, else in memory.
__device__ __forceinline__ uint32_t *owner_words(const Work &W, int e, int hb) { return W.owner + (hb >> 5) + e; }

// whether an event runs the LDS instantiation of the tracking stages
template <int B>
__device__ __forceinline__ bool event_in_lds(const Shared<B> &S, const Lds &L, int N)
{
    return uni(S.maxmod) <= L.cap && N <= L.own_cap;
}

template <int B>
__device__ __forceinline__ uint32_t *owner_ptr(const Shared<B> &S, const Lds &L, const Work &W, int e, int hb, int N)
{
    return event_in_lds<B>(S, L, N) ? L.own : owner_words(W, e, hb);
}

// Seeding and following over all modules.  Leaves the final record list in
// W.fin and its length in S.cnt[3]; with writeback the owner flags are also
// copied to memory.
template <int B, bool kLds>
__device__ void stage_track_impl(const sbt_params &P, const Work &W, int e, int hb, int N, Shared<B> &S,
                                 const Lds &L, bool writeback)
{
    const int M = P.n_modules;
    uint32_t *own = kLds ? L.own : owner_words(W, e, hb);
    const int nw = (N + 31) >> 5;
    for (int i = threadIdx.x; i < nw; i += B) own[i] = 0u;
    for (int i = threadIdx.x; i < N; i += B) {
        W.claim[hb + i] = kNoClaim;
        W.key2rec[hb + i] = kNone;
    }
    if (threadIdx.x == 0) {
        S.cnt[0] = 0; S.cnt[1] = 0; S.cnt[2] = 0; S.cnt[3] = 0;
    }
    RingStage<B> R;
    if (kLds)
        for (int u = 0; u < 4 && u < M; ++u) {
            ring_load<B>(P, W, hb, u, S, L, R);
            ring_store<B>(P, W, hb, u, S, L, R);
        }
    __syncthreads();
    const AList l0 = {kLds ? L.al0 : nullptr, W.act0 + hb, kLds ? L.cap : 0};
    const AList l1 = {kLds ? L.al1 : nullptr, W.act1 + hb, kLds ? L.cap : 0};
    int par = 0;
    stage_seed_follow<B, kLds>(P, W, hb, 2, S, L, own, l0, &S.cnt[1], 0, M > 3);
    __syncthreads();
    for (int t = 3; t < M; ++t) {
        // act (n_act tracks) holds every forming track with its search into
        // t done: resolve t keeping the survivors in nxt, then seed t and
        // search t+1
        const int n_act = uni(S.cnt[1 + par]);
        const AList &act = par ? l1 : l0;
        const AList &nxt = par ? l0 : l1;
        const bool more = t + 1 < M;
        if (kLds && more) ring_load<B>(P, W, hb, t + 1, S, L, R);
        stage_follow_resolve<B, kLds>(P, W, hb, t, S, L, own, act, n_act, nxt, &S.cnt[1 + (par ^ 1)]);
        if (kLds && more) ring_store<B>(P, W, hb, t + 1, S, L, R);
        __syncthreads();
        const int n_keep = uni(S.cnt[1 + (par ^ 1)]);
        if (threadIdx.x == 0) S.cnt[1 + par] = 0;   // act becomes the next step's nxt
        stage_seed_follow<B, kLds>(P, W, hb, t, S, L, own, nxt, &S.cnt[1 + (par ^ 1)], n_keep, more);
        __syncthreads();
        par ^= 1;
    }
    const int n_act = uni(S.cnt[1 + par]);
    const int nf = uni(S.cnt[3]);
    const AList &act = par ? l1 : l0;
    for (int a = threadIdx.x; a < n_act; a += B) W.fin[hb + nf + a] = act.get(a);
    if (kLds && writeback) {
        uint32_t *g = owner_words(W, e, hb);
        for (int i = threadIdx.x; i < nw; i += B) g[i] = own[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) S.cnt[3] = nf + n_act;
    __syncthreads();
}

template <int B>
__device__ void stage_track(const sbt_params &P, const Work &W, int e, int hb, int N, Shared<B> &S, const Lds &L,
                            bool writeback)
{
    if (event_in_lds<B>(S, L, N)) stage_track_impl<B, true>(P, W, e, hb, N, S, L, writeback);
    else stage_track_impl<B, false>(P, W, e, hb, N, S, L, writeback);
}

// ---------------------------------------------------------------- tracklet filter
// Tracks of >= 4 hits are accepted; a three-hit track is a candidate when its
// fit chi2 is under the threshold and none of its hits is flagged; candidates
// sharing hits keep the one with the minimum (chi2, key).
template <int B>
__device__ void stage_filter(const sbt_params &P, const Work &W, int hb, int n_fin, const uint32_t *own)
{
    const float X = P.max_tracklet_chi2;
    unsigned long long *__restrict__ claim = W.claim + hb;
    for (int a = threadIdx.x; a < n_fin; a += B) {
        const int r = W.fin[hb + a];
        const Rec R = W.rec[hb + r];
        uint8_t fl = 0;
        if (R.len >= 4) {
            fl = kFlagAccepted;
        } else {
            const float c2 = W.rchi2[hb + r];
            if (c2 < X && is_free(own, R.h0) && is_free(own, R.h1) && is_free(own, R.h2)) {
                const unsigned long long kap = claim_key(c2, R.key, kFilterStage);
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
            const unsigned long long kap = claim_key(W.rchi2[hb + r], R.key, kFilterStage);
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
