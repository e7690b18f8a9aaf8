// Device-side stages of Search by triplet for gfx950 (wave64).
//
// One event is processed by one workgroup of B lanes.  Every stage is a pure
// function of the event state at the stage start (the paper's barrier between
// seeding and following, Section 3) and every choice is a minimum over unique
// keys, so the parallel evaluation order never changes the result.
//
// Per-event state lives in the workspace, in regions indexed by the event's
// absolute hit offset hb (capacity N = hits of the event):
//   hs      16-byte sorted hits {x, y, z, phi16 | id << 16} by sorted position
//   owner   one bit per hit id: set once a track has taken the hit (the
//           method only ever asks whether a hit is flagged; which track
//           holds it is settled by the claim keys)
//   claim   u64 per hit id: minimum claim key of the current stage (the LDS
//           instantiation keeps the claims on followers' best hits in LDS,
//           by window position, and only the seed hits' claims here)
//   link    two u16 per hit id: the previous hit of the owning track, and
//           the record of the accepted track whose key is this id
//   rec     32-byte forming-track records (one per seed; <= N) and a 16-byte
//           auxiliary record each (search result, seed fit, filter outcome)
//   lists   six u16 lists of the memory instantiation (active tracks x2,
//           final tracks, unflagged positions x2, unflagged ranks)
// Hit ids, keys and record indices are 16-bit (events hold <= 65,535 hits).
// Per-event bases are uniform; per-lane offsets are 32-bit.
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

// per-record auxiliary data
struct RecAux {
    uint32_t best;      // memory instantiation: search result (best id | position << 16, or ~0)
    float bsc;          // its scatter
    float chi2;         // tracklet fit of the seed
    uint32_t flag;      // filter outcome
};
static_assert(sizeof(RecAux) == 16, "auxiliary record layout");

// sorted hit: coordinates and phi16 | id << 16
struct alignas(16) Hit16 {
    float x, y, z;
    uint32_t qid;
};

// per-event counters
struct EvInfo {
    int32_t nt, nh;     // accepted tracks and their hits
    int32_t out_h;      // first output hit position (batch scan)
    int32_t st;         // SBT_EV_* status
    int32_t nfin;       // final records (plain form)
    int32_t out_t;      // first output track position (batch scan)
    int32_t pad[2];
};

// record flags
constexpr uint32_t kFlagCandidate = 2;  // tracklet candidate
constexpr uint32_t kFlagAccepted = 4;

// memory lists (stride = workspace hit capacity)
constexpr int kListAct0 = 0, kListAct1 = 1, kListFin = 2, kListFreeL = 3, kListFreeM = 4, kListFRank = 5;
constexpr int kLists = 6;

// Workspace: one base pointer; every array sits at a fixed multiple of the
// hit capacity H (a multiple of 256) or, after the per-hit arrays, of the
// event capacity E.  Per hit: rec 32 B, hs 16, aux 16, claim 8, keys 4 (sort
// keys of events too large for the LDS sort), link 4, st_toff 4 (per-event
// track hit offsets), six u16 lists 12, st_hits 2 (per-event compacted hit
// ids).  Then the flag bitmaps (event e's starts at word (hb >> 5) + e), the
// per-event counters, the event order (largest first), the work counter (and
// beside it the count of events set aside) and the list of events set aside.
struct Work {
    char *base;
    uint32_t H, E;
};

constexpr uint32_t kOffRec = 0, kOffHs = 32, kOffAux = 48, kOffClaim = 64, kOffKeys = 72, kOffLink = 76,
                   kOffToff = 80, kOffLists = 84, kOffStHits = 96, kHitBytes = 98;

__host__ __device__ inline uint64_t ws_owner(uint32_t H) { return (uint64_t)H * kHitBytes; }
__host__ __device__ inline uint64_t ws_ev(uint32_t H, uint32_t E) { return ws_owner(H) + (((uint64_t)H / 32 + E + 2) * 4 + 255) / 256 * 256; }
__host__ __device__ inline uint64_t ws_order(uint32_t H, uint32_t E) { return ws_ev(H, E) + (uint64_t)E * 32; }
__host__ __device__ inline uint64_t ws_counter(uint32_t H, uint32_t E) { return ws_order(H, E) + (uint64_t)E * 4; }
// events a first pass set aside for a second one
__host__ __device__ inline uint64_t ws_defer(uint32_t H, uint32_t E) { return ws_counter(H, E) + 256; }
__host__ __device__ inline uint64_t ws_bytes(uint32_t H, uint32_t E) { return ws_defer(H, E) + ((uint64_t)E * 4 + 255) / 256 * 256; }

__host__ __device__ inline EvInfo *ws_evinfo(const Work &W) { return (EvInfo *)(W.base + ws_ev(W.H, W.E)); }
__host__ __device__ inline int32_t *ws_orderp(const Work &W) { return (int32_t *)(W.base + ws_order(W.H, W.E)); }
__host__ __device__ inline unsigned int *ws_counterp(const Work &W)
{
    return (unsigned int *)(W.base + ws_counter(W.H, W.E));
}
// the number of events set aside, beside the work counter
__host__ __device__ inline unsigned int *ws_defer_countp(const Work &W) { return ws_counterp(W) + 1; }
__host__ __device__ inline int32_t *ws_deferp(const Work &W) { return (int32_t *)(W.base + ws_defer(W.H, W.E)); }
__host__ __device__ inline Hit16 *ws_hs(const Work &W) { return (Hit16 *)(W.base + (uint64_t)W.H * kOffHs); }
__host__ __device__ inline int32_t *ws_toff(const Work &W) { return (int32_t *)(W.base + (uint64_t)W.H * kOffToff); }
__host__ __device__ inline uint16_t *ws_sthits(const Work &W)
{
    return (uint16_t *)(W.base + (uint64_t)W.H * kOffStHits);
}

struct HitsArgs {
    int32_t n_events;
    int32_t n_hits;
    const int32_t *eo;
    const int32_t *mo;
    const float *x, *y, *z;   // binary32 structure of arrays, or
    const uint2 *h16;         // binary16 x, y, z, unused per hit (null for binary32)
};

struct OutArgs {
    int32_t *eto;
    int32_t *tho;
    int32_t *th;
    int32_t *status;
};

// element i of an array with a uniform base, addressed with a 32-bit offset
template <class T>
__device__ __forceinline__ T &at(T *p, uint32_t i)
{
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(p) + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ const T &at(const T *p, uint32_t i)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + i * (uint32_t)sizeof(T));
}

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

// Lane index among the lanes that run one event.  An event of 64 lanes is
// one wave, and a workgroup may hold several of them, one event per wave;
// wider events have their workgroup to themselves.
template <int B>
__device__ __forceinline__ int tid()
{
    return B == 64 ? (int)(threadIdx.x & 63u) : (int)threadIdx.x;
}

// Barrier over the lanes of one event.  The lanes of a 64-lane event are one
// wave and run in lockstep, so only its memory operations have to complete
// (the fences); the workgroup's other waves run other events and are not
// waited for.
template <int B>
__device__ __forceinline__ void ev_sync()
{
    if (B == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
        __syncthreads();
    }
}

// The same for phases that exchange LDS data only (see lds_barrier).
template <int B>
__device__ __forceinline__ void ev_lds_sync()
{
    if (B == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    } else {
        lds_barrier();
    }
}

// The value, hidden from the optimiser at this point.  Stages re-read the
// scalar parameters and the workspace base through this at the start of
// every module step, so values derived from them are recomputed per step
// instead of being hoisted out of the event and step loops, where dozens of
// them would stay live in scalar registers (and spill) for the whole kernel.
// The "+s" operand must reach the asm in a scalar register: where a change
// elsewhere in a kernel leaves the compiler holding it in a vector register,
// compilation stops with an illegal VGPR-to-SGPR copy (a readfirstlane on
// the input resolves it, at the price of a different register allocation).
template <class T>
__device__ __forceinline__ T opq(T v)
{
    asm volatile("" : "+s"(v));
    return v;
}

// A workspace pointer hidden from the optimiser (see opq) that stays known
// as global memory, so its accesses remain global (not flat) instructions.
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ char *opq_global(char *p)
{
    uint64_t v = reinterpret_cast<uint64_t>(p);
    asm volatile("" : "+s"(v));
    return (char *)(gchar *)v;
}

// scalar parameters of the stages
struct Prm {
    int M, rev, K, Ws, Wf, misses;
    float Ss, Sf, X;
};

__device__ __forceinline__ Prm fresh(const sbt_params &P)
{
    Prm p;
    p.M = opq(P.n_modules);
    p.rev = opq(P.reverse);
    p.K = opq(P.max_doublet_candidates);
    p.Ws = opq(P.phi_window_seeding);
    p.Wf = opq(P.phi_window_forwarding);
    p.misses = opq(P.max_consecutive_misses);
    p.Ss = __int_as_float(opq(__float_as_int(P.max_scatter_seeding)));
    p.Sf = __int_as_float(opq(__float_as_int(P.max_scatter_forwarding)));
    p.X = __int_as_float(opq(__float_as_int(P.max_tracklet_chi2)));
    return p;
}

__device__ __forceinline__ int kmod(const Prm &p, int t) { return p.rev ? p.M - 1 - t : t; }
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
    return ((at(own, id >> 5) >> (id & 31u)) & 1u) == 0u;
}

__device__ __forceinline__ void set_flag(uint32_t *own, unsigned id)
{
    atomicOr(&at(own, id >> 5), 1u << (id & 31u));
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

// number of set bits of m below this lane
__device__ __forceinline__ int lane_rank(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Append under a predicate with one LDS atomic per wave; every lane of the
// wave must call it.  Returns the slot, or -1 where pred is false.
__device__ __forceinline__ int wave_append(bool pred, int *counter)
{
    const unsigned long long m = __ballot(pred);
    if (m == 0) return -1;
    int base = 0;
    if (lane_rank(__builtin_amdgcn_read_exec()) == 0) base = atomicAdd(counter, __popcll(m));
    base = __builtin_amdgcn_readfirstlane(base);
    return pred ? base + lane_rank(m) : -1;
}

// Two appends at once (their atomics overlap); every lane must call it.
__device__ __forceinline__ void wave_append2(bool p0, int *c0, bool p1, int *c1, int &r0, int &r1)
{
    const unsigned long long m0 = __ballot(p0), m1 = __ballot(p1);
    int b0 = 0, b1 = 0;
    if (lane_rank(__builtin_amdgcn_read_exec()) == 0) {
        if (m0) b0 = atomicAdd(c0, __popcll(m0));
        if (m1) b1 = atomicAdd(c1, __popcll(m1));
    }
    b0 = __builtin_amdgcn_readfirstlane(b0);
    b1 = __builtin_amdgcn_readfirstlane(b1);
    r0 = p0 ? b0 + lane_rank(m0) : -1;
    r1 = p1 ? b1 + lane_rank(m1) : -1;
}

// inclusive prefix sum over the wave: row shifts, then the row broadcasts
__device__ __forceinline__ int wave_incl_scan(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return v;
}

// Sum over the waves of the workgroup of per-wave values: returns the sum of
// the waves before this one and sets *total.  s_w holds B/64 ints.
template <int B>
__device__ __forceinline__ int waves_before(int wave_total, int *s_w, int *total)
{
    constexpr int NW = B / 64;
    const int w = uni((int)(tid<B>() >> 6));
    if ((tid<B>() & 63) == 0) s_w[w] = wave_total;
    lds_barrier();
    int before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const int t = s_w[i];
        before += i < w ? t : 0;
        all += t;
    }
    *total = all;
    return before;
}

// Exclusive scan over the workgroup.  s_w holds 2 * (B/64) ints; the two
// halves alternate with `phase` so back-to-back calls need one barrier each.
template <int B>
__device__ __forceinline__ int block_excl_scan(int v, int *s_w, int phase, int *total)
{
    const int inc = wave_incl_scan(v);
    const int wt = __builtin_amdgcn_readlane(inc, 63);
    if (B == 64) {
        *total = wt;
        return inc - v;
    }
    return waves_before<B>(wt, s_w + (phase & 1) * (B / 64), total) + inc - v;
}

// Exclusive counts of two predicates over the workgroup (ballots), packed as
// count_a | count_b << 16 like the totals.
template <int B>
__device__ __forceinline__ int block_count2(bool pa, bool pb, int *s_w, int phase, int *total)
{
    const unsigned long long ma = __ballot(pa), mb = __ballot(pb);
    const int mine = lane_rank(ma) | (lane_rank(mb) << 16);
    const int wt = __popcll(ma) | (__popcll(mb) << 16);
    if (B == 64) {
        *total = wt;
        return mine;
    }
    return waves_before<B>(wt, s_w + (phase & 1) * (B / 64), total) + mine;
}

// in-place exclusive scan of a[0..n) in LDS
template <int B>
__device__ void block_scan_inplace(int *a, int n, int *s_w)
{
    const int chunk = (n + B - 1) / B;
    const int beg = tid<B>() * chunk;
    const int end = beg + chunk < n ? beg + chunk : n;
    int sum = 0;
    for (int i = beg; i < end; ++i) sum += a[i];
    int total;
    int off = block_excl_scan<B>(sum, s_w, 0, &total);
    for (int i = beg; i < end; ++i) {
        int v = a[i];
        a[i] = off;
        off += v;
    }
}

// minimum over lanes lane ^ m, m = 1, 2, 4, 8 (quad permutes for 1 and 2)
__device__ __forceinline__ int lane_xor(int v, int m)
{
    if (m == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
    if (m == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
    return __shfl_xor(v, m);
}

// ---------------------------------------------------------------- LDS layout
// Dynamic LDS of one event workgroup, for a compile-time slot capacity CAP
// (hits per module slot).  The sort scratch (histogram, fill counters, the
// 32-bit sort keys and per-hit bins of events with at most sortcap/2 hits)
// aliases the tracking area, which is filled only after the sort.
//   ring   4 slots x CAP sorted hits (16 B each): traversal index u in slot
//          u mod 4; module t+1 is filled into the slot of t-3 while t is
//          being resolved
//   tab    coarse phi index of each slot: first position whose phi16 high
//          byte is >= b, b = 0..256
//   freel  unflagged positions of the seeding stage's doublet module
//   freem  unflagged positions of the middle module
//   frank  unflagged positions before each doublet-module position
//   al0/1  active-track lists (CAP entries; more sends the event to memory)
//   res    per active slot: the search result (best hit id | window position
//          << 16, scatter) and the claim set's inputs (key, seed hits)
//   cfree  unflagged-position bits of the seeding stage's third module
//   lclaim claim words of the module being searched by the following
//          stage, by window position (the claims on seed hits stay in memory)
//   own    hit-flag bitmap of the event when N <= own_cap
extern __shared__ __align__(16) char g_lds[];

constexpr int kTab = 257;
constexpr int kSlots = 4;   // ring slots: traversal indices t-2 .. t+1
__host__ __device__ constexpr uint32_t a16(uint32_t v) { return (v + 15u) & ~15u; }
__host__ __device__ constexpr uint32_t lay_tab(int cap) { return 16u * kSlots * (uint32_t)cap; }
__host__ __device__ constexpr uint32_t lay_freel(int cap) { return a16(lay_tab(cap) + 2u * kSlots * kTab); }
__host__ __device__ constexpr uint32_t lay_freem(int cap) { return lay_freel(cap) + a16(2u * cap); }
__host__ __device__ constexpr uint32_t lay_frank(int cap) { return lay_freem(cap) + a16(2u * cap); }
__host__ __device__ constexpr uint32_t lay_al0(int cap) { return lay_frank(cap) + a16(2u * cap); }
__host__ __device__ constexpr uint32_t lay_al1(int cap) { return lay_al0(cap) + a16(2u * cap); }
__host__ __device__ constexpr uint32_t lay_res(int cap) { return lay_al1(cap) + a16(2u * cap); }
__host__ __device__ constexpr uint32_t lay_cfree(int cap) { return lay_res(cap) + 16u * cap; }
__host__ __device__ constexpr uint32_t lay_lclaim(int cap) { return lay_cfree(cap) + a16(8u * (uint32_t)((cap + 63) / 64)); }
__host__ __device__ constexpr uint32_t lay_own(int cap) { return lay_lclaim(cap) + 8u * (uint32_t)cap; }

// sort bins: 1024 in total, a power of two per module
constexpr int kSortBins = 1024;
__host__ __device__ constexpr uint32_t lds_sort_head() { return a16((2u * kSortBins + 1u) * 4u); }

__host__ __device__ inline uint32_t lds_bytes(int cap, int own_cap)
{
    const uint32_t sort = lds_sort_head() + 4u * 1024u;   // keys of 1,024 hits at least
    const uint32_t track = cap > 0 ? lay_own(cap) + a16(4u * (uint32_t)((own_cap + 31) / 32)) : 0u;
    return sort > track ? sort : track;
}
__host__ __device__ inline int lds_sortcap(int cap, int own_cap)
{
    return (int)((lds_bytes(cap, own_cap) - lds_sort_head()) / 4u);
}

__host__ __device__ inline int sort_shift(int M)
{
    int bits = 4;                       // M <= 64 -> at least 16 bins per module
    while (bits < 12 && (M << (bits + 1)) <= kSortBins) ++bits;
    return 16 - bits;
}

template <int CAP>
struct Lay {
    static __device__ __forceinline__ Hit16 *ring(uint32_t lo, int s)
    {
        return reinterpret_cast<Hit16 *>(g_lds + lo) + s * CAP;
    }
    static __device__ __forceinline__ uint16_t *tab(uint32_t lo, int s)
    {
        return reinterpret_cast<uint16_t *>(g_lds + lo + lay_tab(CAP)) + s * kTab;
    }
    static __device__ __forceinline__ uint16_t *freel(uint32_t lo) { return reinterpret_cast<uint16_t *>(g_lds + lo + lay_freel(CAP)); }
    static __device__ __forceinline__ uint16_t *freem(uint32_t lo) { return reinterpret_cast<uint16_t *>(g_lds + lo + lay_freem(CAP)); }
    static __device__ __forceinline__ uint16_t *frank(uint32_t lo) { return reinterpret_cast<uint16_t *>(g_lds + lo + lay_frank(CAP)); }
    static __device__ __forceinline__ uint16_t *al(uint32_t lo, int i)
    {
        return reinterpret_cast<uint16_t *>(g_lds + lo + (i ? lay_al1(CAP) : lay_al0(CAP)));
    }
    static __device__ __forceinline__ uint4 *res(uint32_t lo) { return reinterpret_cast<uint4 *>(g_lds + lo + lay_res(CAP)); }
    static __device__ __forceinline__ uint32_t *own(uint32_t lo) { return reinterpret_cast<uint32_t *>(g_lds + lo + lay_own(CAP)); }
    static __device__ __forceinline__ unsigned long long *cfree(uint32_t lo)
    {
        return reinterpret_cast<unsigned long long *>(g_lds + lo + lay_cfree(CAP));
    }
    static __device__ __forceinline__ unsigned long long *lclaim(uint32_t lo)
    {
        return reinterpret_cast<unsigned long long *>(g_lds + lo + lay_lclaim(CAP));
    }
};

// static LDS shared by the stages of one event
template <int B>
struct Shared {
    int mo[SBT_MAX_MODULES + 1];
    int cnt[4];          // records, list[0], list[1], final
    int status;
    int e;
    int maxmod;          // hits of the event's largest module
    int ovf;             // an LDS list overflowed
    int scan[2 * (B / 64)];
    int slot_n[kSlots];  // hits of the module held by each ring slot
    uint8_t mtab[(SBT_MAX_EVENT_HITS + 64) / 64];   // module of every 64th hit (sort)
};

// Events of 64 lanes run one per wave, up to this many in a workgroup; each
// takes a region of the dynamic LDS: its Shared block, then its layout.
constexpr int kMaxEventsPerBlock = 16;
template <int B>
__host__ __device__ constexpr uint32_t shared_block_bytes()
{
    return a16((uint32_t)sizeof(Shared<B>));
}
template <int B>
__host__ __device__ inline uint32_t event_region_bytes(int cap, int own_cap)
{
    return shared_block_bytes<B>() + lds_bytes(cap, own_cap);
}

// per-event views of the workspace: pointers are derived on use from the
// base, the capacity H and the event's hit offset hb
struct Ev {
    char *base;
    uint32_t H, E;
    int e, hb, N;
    uint32_t lo;   // byte offset of the event's region in the workgroup's dynamic LDS
    template <class T>
    __device__ __forceinline__ T *arr(uint32_t off, uint32_t elem) const
    {
        return reinterpret_cast<T *>(base + (uint64_t)H * off + (uint64_t)(uint32_t)hb * elem);
    }
    __device__ __forceinline__ Rec *rec() const { return arr<Rec>(kOffRec, 32); }
    __device__ __forceinline__ Hit16 *hs() const { return arr<Hit16>(kOffHs, 16); }
    __device__ __forceinline__ RecAux *aux() const { return arr<RecAux>(kOffAux, 16); }
    __device__ __forceinline__ unsigned long long *claim() const { return arr<unsigned long long>(kOffClaim, 8); }
    __device__ __forceinline__ uint32_t *keys() const { return arr<uint32_t>(kOffKeys, 4); }
    __device__ __forceinline__ uint16_t *link() const { return arr<uint16_t>(kOffLink, 4); }   // [2i] prev, [2i+1] key -> record
    __device__ __forceinline__ int32_t *st_toff() const { return arr<int32_t>(kOffToff, 4); }
    __device__ __forceinline__ uint16_t *st_hits() const { return arr<uint16_t>(kOffStHits, 2); }
    __device__ __forceinline__ uint16_t *list(int k) const
    {
        return reinterpret_cast<uint16_t *>(base + (uint64_t)H * (kOffLists + 2u * k) + (uint64_t)(uint32_t)hb * 2);
    }
    __device__ __forceinline__ uint32_t *own() const
    {
        return reinterpret_cast<uint32_t *>(base + ws_owner(H)) + ((uint32_t)hb >> 5) + e;
    }
    __device__ __forceinline__ EvInfo &info() const
    {
        return reinterpret_cast<EvInfo *>(base + ws_ev(H, E))[e];
    }
};

__device__ __forceinline__ Ev event_view(const Work &W, int e, int hb, int N, uint32_t lo = 0)
{
    Ev v;
    v.base = opq_global(W.base);
    v.H = opq(W.H);
    v.E = W.E;
    v.e = e;
    v.hb = hb;
    v.N = N;
    v.lo = lo;
    return v;
}

// the view with its base hidden from the optimiser (see opq)
__device__ __forceinline__ Ev fresh(const Ev &v)
{
    Ev w = v;
    w.base = opq_global(v.base);
    w.H = opq(v.H);
    return w;
}

// ---------------------------------------------------------------- validation
// Loads the event-local module offsets into LDS and checks the offsets.
template <int B>
__device__ int load_event(const sbt_params &P, const HitsArgs &H, int e, Shared<B> &S,
                          int *hb_out, int *n_out)
{
    const int M = P.n_modules;
    int lo = H.eo[e], hi = H.eo[e + 1];
    if (tid<B>() == 0) {
        S.status = 0;
        S.maxmod = 0;
    }
    ev_sync<B>();
    unsigned st = 0;
    if (lo < 0 || hi > H.n_hits || hi < lo) st = SBT_EV_BAD_OFFSETS;
    else if (hi - lo > SBT_MAX_EVENT_HITS) st = SBT_EV_TOO_LARGE;
    else if (P.max_event_hits > 0 && hi - lo > P.max_event_hits) st = SBT_EV_CUT;
    if (st == 0) {
        const long long base = (long long)e * M;
        for (int k = tid<B>(); k <= M; k += B) {
            int v = H.mo[base + k];
            S.mo[k] = v - lo;
            bool bad = (k == 0 && v != lo) || (k == M && v != hi) || v < lo || v > hi;
            if (k > 0 && H.mo[base + k - 1] > v) bad = true;
            if (bad) atomicOr(&S.status, (int)SBT_EV_BAD_OFFSETS);
            if (k < M) atomicMax(&S.maxmod, H.mo[base + k + 1] - v);
        }
    } else if (tid<B>() == 0) {
        S.status = (int)st;
    }
    ev_sync<B>();
    *hb_out = uni(lo);
    *n_out = uni(hi - lo);
    return uni(S.status);
}

// ---------------------------------------------------------------- hit coordinates
// Coordinates of event-local hit i, from binary32 arrays or widened exactly
// from the binary16 array-of-structures form.
__device__ __forceinline__ float half_bits_to_float(uint32_t b)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xFFFFu));
}

struct HitSrc {
    const float *x, *y, *z;
    const uint2 *h16;
    __device__ __forceinline__ void xy(int i, float &px, float &py) const
    {
        if (h16) {
            const uint2 w = at(h16, i);
            px = half_bits_to_float(w.x);
            py = half_bits_to_float(w.x >> 16);
        } else {
            px = at(x, i);
            py = at(y, i);
        }
    }
    __device__ __forceinline__ void xyz(int i, float &px, float &py, float &pz) const
    {
        if (h16) {
            const uint2 w = at(h16, i);
            px = half_bits_to_float(w.x);
            py = half_bits_to_float(w.x >> 16);
            pz = half_bits_to_float(w.y);
        } else {
            px = at(x, i);
            py = at(y, i);
            pz = at(z, i);
        }
    }
};

__device__ __forceinline__ HitSrc hit_src(const HitsArgs &H, int hb)
{
    HitSrc s;
    s.h16 = H.h16 ? H.h16 + hb : nullptr;
    s.x = H.h16 ? nullptr : H.x + hb;
    s.y = H.h16 ? nullptr : H.y + hb;
    s.z = H.h16 ? nullptr : H.z + hb;
    return s;
}

// ---------------------------------------------------------------- sort by phi
// Counting sort on (module, top bits of phi16) into buckets of 32-bit keys
// phi16 << 16 | id, then each key's rank inside its bucket by counting the
// smaller keys of the bucket; ties in phi16 fall to the lower id because the
// id is the key's low half.  Three forms by event size against the LDS key
// capacity sortcap: keys and per-hit bins in LDS (2N <= sortcap); keys in
// LDS with the bins recomputed (N <= sortcap); both in memory.
// module of hit i from the module of its 64-hit chunk and a short forward scan
__device__ __forceinline__ int sort_bin(const int *mo, const uint8_t *mtab, int i, uint16_t q, int bpm, int shift)
{
    int m = mtab[i >> 6];
    while (mo[m + 1] <= i) ++m;
    return m * bpm + (q >> shift);
}

constexpr int kSortChunk = 8;

template <int B>
__device__ void stage_sort(const sbt_params &PP, const HitsArgs &H, const Ev &v0, Shared<B> &S, int sortcap)
{
    const Ev v = fresh(v0);
    const int M = fresh(PP).M, N = v.N;
    const int shift = sort_shift(M);
    const int bpm = 1 << (16 - shift);
    const int nb = M * bpm;
    int *hist = reinterpret_cast<int *>(g_lds + v.lo);
    int *fill = hist + kSortBins + 1;
    uint32_t *lkeys = reinterpret_cast<uint32_t *>(g_lds + v.lo + lds_sort_head());
    const int form = 2 * N <= sortcap ? 0 : (N <= sortcap ? 1 : 2);
    for (int i = tid<B>(); i <= nb; i += B) hist[i] = 0;
    for (int i = tid<B>(); i < nb; i += B) fill[i] = 0;
    for (int c = tid<B>(); c < (N + 63) / 64; c += B) S.mtab[c] = (uint8_t)module_of(S.mo, M, c * 64);
    ev_sync<B>();
    const HitSrc src = hit_src(H, v.hb);
    // memory form: bins in the claim words (not yet in use)
    uint32_t *bins_m = reinterpret_cast<uint32_t *>(v.claim());
    // the coordinates of a lane's next kSortChunk hits are loaded together
    for (int i0 = tid<B>(); i0 < N; i0 += kSortChunk * B) {
        float px[kSortChunk], py[kSortChunk];
#pragma unroll
        for (int j = 0; j < kSortChunk; ++j)
            if (i0 + j * B < N) src.xy(i0 + j * B, px[j], py[j]);
#pragma unroll
        for (int j = 0; j < kSortChunk; ++j) {
            const int i = i0 + j * B;
            if (i >= N) break;
            const uint16_t qi = phi16(px[j], py[j]);
            const int bin = sort_bin(S.mo, S.mtab, i, qi, bpm, shift);
            const uint32_t tb = (uint32_t)qi | ((uint32_t)bin << 16);
            if (form == 0) lkeys[N + i] = tb;
            else if (form == 2) at(bins_m, i) = tb;
            atomicAdd(&hist[bin], 1);
        }
    }
    ev_sync<B>();
    block_scan_inplace<B>(hist, nb + 1, S.scan);
    ev_sync<B>();
    // separate LDS and memory branches keep each access in its address space
    if (form == 0) {
        for (int i = tid<B>(); i < N; i += B) {
            const uint32_t tb = lkeys[N + i];
            const int bin = (int)(tb >> 16);
            lkeys[hist[bin] + atomicAdd(&fill[bin], 1)] = (tb << 16) | (uint32_t)i;
        }
    } else if (form == 1) {
        for (int i = tid<B>(); i < N; i += B) {
            float px, py;
            src.xy(i, px, py);
            const uint16_t qi = phi16(px, py);
            const int bin = sort_bin(S.mo, S.mtab, i, qi, bpm, shift);
            lkeys[hist[bin] + atomicAdd(&fill[bin], 1)] = ((uint32_t)qi << 16) | (uint32_t)i;
        }
    } else {
        for (int i = tid<B>(); i < N; i += B) {
            const uint32_t tb = at(bins_m, i);
            const int bin = (int)(tb >> 16);
            at(v.keys(), hist[bin] + atomicAdd(&fill[bin], 1)) = (tb << 16) | (uint32_t)i;
        }
    }
    ev_sync<B>();
    for (int s = tid<B>(); s < N; s += B) {
        uint32_t key;
        int i, rank;
        if (form != 2) {
            key = lkeys[s];
            i = (int)(key & 0xFFFFu);
            const int bin = form == 0 ? (int)(lkeys[N + i] >> 16)
                                      : sort_bin(S.mo, S.mtab, i, (uint16_t)(key >> 16), bpm, shift);
            const int lo = hist[bin], hi = hist[bin + 1];
            rank = lo;
            for (int m = lo; m < hi; ++m) rank += lkeys[m] < key;
        } else {
            key = at(v.keys(), s);
            i = (int)(key & 0xFFFFu);
            const int bin = (int)(at(bins_m, i) >> 16);
            const int lo = hist[bin], hi = hist[bin + 1];
            rank = lo;
            for (int m = lo; m < hi; ++m) rank += at(v.keys(), m) < key;
        }
        Hit16 h;
        src.xyz(i, h.x, h.y, h.z);
        h.qid = (key >> 16) | (key << 16);
        at(v.hs(), rank) = h;
    }
    ev_sync<B>();
}

// ---------------------------------------------------------------- module windows
// An event whose modules all fit the LDS slots (and whose hit flags fit the
// LDS bitmap) runs the LDS instantiation of the tracking stages: traversal
// index u lives in ring slot u mod 4 and every window access is an LDS access.
// Any other event runs the memory instantiation, which reads the sorted
// hits in memory directly.  Both compute the same thing.
struct Win {
    const Hit16 *h;
    const uint16_t *tab;   // coarse index (LDS instantiation)
    int n;
};

__device__ __forceinline__ uint16_t q_of(const Hit16 &h) { return (uint16_t)(h.qid & 0xFFFFu); }
__device__ __forceinline__ uint16_t id_of(const Hit16 &h) { return (uint16_t)(h.qid >> 16); }
__device__ __forceinline__ uint16_t win_q(const Win &w, int p) { return (uint16_t)(at(w.h, p).qid & 0xFFFFu); }
__device__ __forceinline__ uint16_t win_id(const Win &w, int p) { return (uint16_t)(at(w.h, p).qid >> 16); }

// first position of the window whose phi16 is >= v
template <bool kLds>
__device__ __forceinline__ int win_lower_bound(const Win &w, uint16_t v)
{
    if (kLds) {
        int p = at(w.tab, v >> 8);
        const int end = at(w.tab, (v >> 8) + 1);
        while (p < end && win_q(w, p) < v) ++p;
        return p;
    }
    int lo = 0, hi = w.n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (win_q(w, mid) < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <int B, bool kLds, int CAP>
__device__ __forceinline__ Win window(const Prm &P, const Shared<B> &S, const Ev &v, int u)
{
    Win w;
    if (kLds) {
        const int s = u % kSlots;
        w.n = uni(S.slot_n[s]);
        w.h = Lay<CAP>::ring(v.lo, s);
        w.tab = Lay<CAP>::tab(v.lo, s);
    } else {
        const int k = kmod(P, u);
        const int g0 = uni(S.mo[k]);
        w.n = uni(S.mo[k + 1]) - g0;
        w.h = v.hs() + g0;
        w.tab = nullptr;
    }
    return w;
}

// coarse-index entries owned by position i > 0 of a slot whose phi16 is q
// (qp: phi16 of position i-1): every high byte b with high(qp) < b <=
// high(q) starts at i.  The entries up to the first hit's high byte (0) and
// above the last hit's (n) are written by all lanes together.
__device__ __forceinline__ void tab_fill(uint16_t *tab, int i, uint16_t q, uint16_t qp)
{
    if (i == 0) return;
    for (int b = (qp >> 8) + 1; b <= (q >> 8); ++b) tab[b] = (uint16_t)i;
}

// Copies the sorted hits of traversal index u into its ring slot and builds
// the slot's coarse index, on lanes [l0, B) of the workgroup.
template <int B, int CAP>
__device__ __forceinline__ void ring_fill(const Prm &P, const Ev &v, int u, Shared<B> &S, int l0)
{
    const int lane = (int)tid<B>() - l0, nl = B - l0;
    if (lane < 0) return;
    const int k = kmod(P, u);
    const int g = uni(S.mo[k]), n = uni(S.mo[k + 1]) - g;
    const int s = u % kSlots;
    if (lane == 0) S.slot_n[s] = n;
    Hit16 *ring = Lay<CAP>::ring(v.lo, s);
    uint16_t *tab = Lay<CAP>::tab(v.lo, s);
    const Hit16 *src = v.hs() + g;
    // n == 0: every entry is 0
    int hi_first = kTab, hi_last = kTab;
    if (n > 0) {
        hi_first = q_of(at(src, 0)) >> 8;
        hi_last = q_of(at(src, n - 1)) >> 8;
    }
    for (int b = lane; b < kTab; b += nl) {
        if (b <= hi_first) tab[b] = 0;
        else if (b > hi_last) tab[b] = (uint16_t)n;
    }
    for (int i = lane; i < n; i += nl) {
        const Hit16 h = at(src, i);
        ring[i] = h;
        tab_fill(tab, i, q_of(h), i > 0 ? q_of(at(src, i - 1)) : (uint16_t)0);
    }
}

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
            pu = at(F, ix);
            int o = pu - s0;
            if (o < 0) o += na;
            if (o <= hu) vu = 2 * o;
        }
        if (sd < nf) {
            int ix = j - 1 - sd;
            if (ix < 0) ix += nf;
            pd = at(F, ix);
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

// The same picks for K = 4 with the four partner ranks of a middle hit on
// the four lanes of a quad (c = lane & 3): lane c loads the c-th unflagged
// position upwards from s0 and the c-th downwards below it and turns them
// into visit ranks; the quad exchanges the eight ranks, every lane merges
// the two ascending lists and keeps the c-th smallest, whose rank gives its
// position back (rank 2o: s0 + o, rank 2o - 1: s0 - o).  All four lanes of
// the quad must be active.
template <int CTRL>
__device__ __forceinline__ int quad_bcast(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, false);
}

__device__ __forceinline__ int pendulum_quad(const uint16_t *F, int nf, int j, int s0, int na, int hu, int hd, int c)
{
    constexpr int kInf = 0x7fffffff;
    int ru = kInf, rd = kInf;
    if (c < nf) {
        int iu = j + c;
        if (iu >= nf) iu -= nf;
        int id = j - 1 - c;
        if (id < 0) id += nf;
        const int pu = at(F, iu), pd = at(F, id);
        int o = pu - s0;
        if (o < 0) o += na;
        if (o <= hu) ru = 2 * o;
        int od = s0 - pd;
        if (od < 0) od += na;
        if (od >= 1 && od <= hd) rd = 2 * od - 1;
    }
    int u0 = quad_bcast<0x00>(ru), u1 = quad_bcast<0x55>(ru), u2 = quad_bcast<0xAA>(ru), u3 = quad_bcast<0xFF>(ru);
    int d0 = quad_bcast<0x00>(rd), d1 = quad_bcast<0x55>(rd), d2 = quad_bcast<0xAA>(rd), d3 = quad_bcast<0xFF>(rd);
    int pick = kInf;
#pragma unroll
    for (int step = 0; step < 4; ++step) {
        const bool up = u0 < d0;
        const int take = up ? u0 : d0;
        if (step == c) pick = take;
        if (up) { u0 = u1; u1 = u2; u2 = u3; u3 = kInf; }
        else { d0 = d1; d1 = d2; d2 = d3; d3 = kInf; }
    }
    if (pick == kInf) return -1;
    int pos;
    if ((pick & 1) == 0) {
        pos = s0 + (pick >> 1);
        if (pos >= na) pos -= na;
    } else {
        pos = s0 - ((pick + 1) >> 1);
        if (pos < 0) pos += na;
    }
    return pos;
}

// Best third hit for one doublet: the key orders like the comparison
// (found, scatter, id0, id2) -- scatter bits << 32 | id0 << 16 | id2, ~0 when
// nothing was found (scatters are >= +0, so their bits order like the
// values); pos holds the window positions pos0 | pos2 << 16.
template <bool kLds>
__device__ __forceinline__ void seed_doublet(const Win &wa, const Win &wc, const uint32_t *own,
                                             const unsigned long long *cfree, int pos0, float x1, float y1, float z1,
                                             float Zc, float Ss, uint16_t Ws, uint16_t span, unsigned long long &bkey,
                                             uint32_t &bpos)
{
    const Hit16 h0 = at(wa.h, pos0);
    const uint32_t id0 = id_of(h0);
    const float d01 = z1 - h0.z;
    const float tx = (x1 - h0.x) / d01;
    const float ty = (y1 - h0.y) / d01;
    const float dzc = Zc - z1;
    const uint16_t qe = phi16(x1 + tx * dzc, y1 + ty * dzc);
    const int nc = wc.n;
    if (nc == 0) return;
    const uint16_t lo = (uint16_t)(qe - Ws);
    int pc = win_lower_bound<kLds>(wc, lo);
    if (pc == nc) pc = 0;
    Hit16 h2n = at(wc.h, pc);
    for (int jj = 0; jj < nc; ++jj) {
        // LDS: the flag bit is addressed by position, so it loads alongside the hit
        const bool fpos = kLds ? ((at(cfree, (uint32_t)pc >> 6) >> (pc & 63)) & 1ull) != 0ull : true;
        const Hit16 h2 = h2n;
        const int pn = pc + 1 == nc ? 0 : pc + 1;
        h2n = at(wc.h, pn);   // the next position, loaded while this one is scored
        if ((uint16_t)(q_of(h2) - lo) > span) break;
        const uint32_t id2 = id_of(h2);
        const bool fr = kLds ? fpos : is_free(own, id2);
        const float dz = h2.z - z1;
        const float dx = (x1 + tx * dz) - h2.x;
        const float dy = (y1 + ty * dz) - h2.y;
        const float sc = (dx * dx) + (dy * dy);
        const unsigned long long k = ((unsigned long long)__float_as_uint(sc) << 32) | (id0 << 16) | id2;
        const bool better = fr && (sc < Ss) && (k < bkey);
        bkey = better ? k : bkey;
        bpos = better ? ((uint32_t)pos0 | ((uint32_t)pc << 16)) : bpos;
        pc = pn;
    }
}

// ---------------------------------------------------------------- following search
// Following search of one forming track into traversal index u (Section 3,
// "track following"): the last two hits extrapolated to the module's
// nominal z, the best unflagged hit of the inclusive phi window by
// (scatter, id) under the threshold, and claims on that hit (and on the
// three seed hits of a bare seed) keyed (scatter, key) for stage u.  The LDS
// instantiation claims the best hit in lclaim, by window position; seed
// hits are always claimed in memory.  Returns the best hit's id | window
// position << 16, or ~0.
template <bool kLds>
__device__ __forceinline__ uint32_t follow_item(const Prm &P, const Win &wc, float Zc, const uint32_t *own,
                                                unsigned long long *claim, unsigned long long *lclaim, const Rec &R,
                                                int u, float &bsc_out)
{
    const float Sf = P.Sf;
    const uint16_t Wf = (uint16_t)P.Wf;
    const uint16_t span = (uint16_t)(2 * P.Wf);
    const int nc = wc.n;
    uint16_t best = kNone;
    int bpos = 0;
    float bsc = 0.0f;
    bool elig = (u - (int)R.last_t) <= P.misses + 1;
    if (elig && R.len == 3) elig = is_free(own, R.h0) && is_free(own, R.h1) && is_free(own, R.h2);
    if (elig && nc > 0) {
        const float dzc = Zc - R.zb;
        const uint16_t qe = phi16(R.xb + R.tx * dzc, R.yb + R.ty * dzc);
        const uint16_t lo = (uint16_t)(qe - Wf);
        int pc = win_lower_bound<kLds>(wc, lo);
        if (pc == nc) pc = 0;
        // No hit of module u is flagged yet: flags are set only when a
        // module is resolved, and u is resolved after this search.  The
        // flag test of the method is therefore always passed here.
        // (scatter, id) packed so that one comparison orders both
        unsigned long long bk = ~0ull;
        Hit16 hn = at(wc.h, pc);
        for (int j = 0; j < nc; ++j) {
            const Hit16 h = hn;
            const int pn = pc + 1 == nc ? 0 : pc + 1;
            hn = at(wc.h, pn);   // the next position, loaded while this one is scored
            if ((uint16_t)(q_of(h) - lo) > span) break;
            const float dz = h.z - R.zb;
            const float dx = (R.xb + R.tx * dz) - h.x;
            const float dy = (R.yb + R.ty * dz) - h.y;
            const float sc = (dx * dx) + (dy * dy);
            const unsigned long long k = ((unsigned long long)__float_as_uint(sc) << 32) | id_of(h);
            const bool better = (sc < Sf) && (k < bk);
            bk = better ? k : bk;
            bpos = better ? pc : bpos;
            pc = pn;
        }
        if (bk != ~0ull) {
            best = (uint16_t)(bk & 0xFFFFu);
            bsc = __uint_as_float((uint32_t)(bk >> 32));
        }
        if (best != kNone) {
            const unsigned long long kap = claim_key(bsc, R.key, u);
            if (kLds) atomicMin(&lclaim[bpos], kap);
            else atomicMin(&at(claim, best), kap);
            if (R.len == 3) {
                atomicMin(&at(claim, R.h0), kap);
                atomicMin(&at(claim, R.h1), kap);
                atomicMin(&at(claim, R.h2), kap);
            }
        }
    }
    bsc_out = bsc;
    return best == kNone ? 0xFFFFFFFFu : ((uint32_t)bpos << 16) | best;
}

// Search result of active slot a (record r).  LDS instantiation: the slot's
// 16 bytes hold the result and what the resolution needs to test the claims
// without the record: {best | position << 16, scatter, key | h0 << 16,
// h1 | h2 << 16}, seed hits only for a bare seed (h0 = none otherwise).
// Memory instantiation: the record's auxiliary data.
template <bool kLds, int CAP>
__device__ __forceinline__ void put_result(const Ev &v, int a, int r, uint32_t pb, float bsc, const Rec &R)
{
    if (kLds) {
        uint4 w;
        w.x = pb;
        w.y = __float_as_uint(bsc);
        w.z = (uint32_t)R.key | ((uint32_t)(R.len == 3 ? R.h0 : kNone) << 16);
        w.w = (uint32_t)R.h1 | ((uint32_t)R.h2 << 16);
        Lay<CAP>::res(v.lo)[a] = w;
    } else {
        RecAux &x = at(v.aux(), r);
        x.best = pb;
        x.bsc = bsc;
    }
}

// Seeding(t), t >= 2 (Section 3), fused with the following search into
// t+1.  With kCand the pendulum start of every middle hit is read from the
// table a separate candidate pass wrote into the workspace (the paper's
// "Fill candidates" kernel) instead of being searched here.  Seeding: modules A = kmod(t-2), Bm = kmod(t-1), C = kmod(t); work
// items are (unflagged middle hit, partner rank c) -- with K a power of two
// up to 16, the K doublets of a middle hit run on K adjacent lanes and their
// best triplets are reduced across the lanes, otherwise one lane handles all
// K.  A new seed's following search into t+1 runs on the lane that made it.
// The tracks kept by the last resolution (active slots [0, n_keep)) search
// t+1 on waves of their own.  Both read the flags as the resolution of t
// left them, which is the state the following of t+1 starts from.
template <int B, bool kLds, int CAP, bool kCand = false>
__device__ void stage_seed_follow(const sbt_params &PP, const Ev &v0, int t, Shared<B> &S, const uint32_t *own,
                                  uint16_t *nxt, int *n_nxt, int n_keep, bool follow_next)
{
    const Prm P = fresh(PP);
    const Ev v = fresh(v0);
    const Win wa = window<B, kLds, CAP>(P, S, v, t - 2);
    const Win wb = window<B, kLds, CAP>(P, S, v, t - 1);
    const Win wc = window<B, kLds, CAP>(P, S, v, t);
    Win wn = wc;
    float Zn = 0.0f;
    if (follow_next) {
        wn = window<B, kLds, CAP>(P, S, v, t + 1);
        Zn = PP.module_z[kmod(P, t + 1)];
    }
    const int na = wa.n, nbm = wb.n;
    const float Zc = PP.module_z[kmod(P, t)];
    const float Ss = P.Ss;
    const int K = P.K;
    const uint16_t Ws = (uint16_t)P.Ws;
    const uint16_t span = (uint16_t)(2 * P.Ws);

    // unflagged positions of the doublet module and of the middle module, ascending
    uint16_t *F, *FR, *FM;
    if (kLds) {
        F = Lay<CAP>::freel(v.lo);
        FR = Lay<CAP>::frank(v.lo);
        FM = Lay<CAP>::freem(v.lo);
    } else {
        const int ga = uni(S.mo[kmod(P, t - 2)]), gb = uni(S.mo[kmod(P, t - 1)]);
        F = v.list(kListFreeL) + ga;
        FR = v.list(kListFRank) + ga;
        FM = v.list(kListFreeM) + gb;
    }
    int nf = 0, nfm = 0;
    int nmax = na > nbm ? na : nbm;
    if (kLds && wc.n > nmax) nmax = wc.n;
    unsigned long long *cfree = kLds ? Lay<CAP>::cfree(v.lo) : nullptr;
    unsigned long long *lclaim = kLds ? Lay<CAP>::lclaim(v.lo) : nullptr;
    if (kLds && follow_next)
        for (int p = tid<B>(); p < wn.n; p += B) lclaim[p] = kNoClaim;
    int phase = 0;
    for (int base = 0; base < nmax; base += B, ++phase) {
        const int p = base + (int)tid<B>();
        const bool fa = p < na && is_free(own, win_id(wa, p));
        const bool fb = p < nbm && is_free(own, win_id(wb, p));
        if (kLds) {
            const unsigned long long m = __ballot(p < wc.n && is_free(own, win_id(wc, p)));
            if ((tid<B>() & 63) == 0 && p < wc.n) at(cfree, (uint32_t)p >> 6) = m;
        }
        int total;
        const int idx = block_count2<B>(fa, fb, S.scan, phase, &total);
        if (p < na) at(FR, p) = (uint16_t)(nf + (idx & 0xFFFF));
        if (fa) at(F, nf + (idx & 0xFFFF)) = (uint16_t)p;
        if (fb) at(FM, nfm + (idx >> 16)) = (uint16_t)p;
        nf += total & 0xFFFF;
        nfm += total >> 16;
    }
    // the lists are in LDS in the LDS instantiation, in memory otherwise
    if (kLds) ev_lds_sync<B>();
    else ev_sync<B>();
    const int hd = na >> 1, hu = na - hd - 1;   // offsets visited: [-hd, hu]
    const int G = (K == 1 || K == 2 || K == 4 || K == 8 || K == 16) ? K : 1;
    const int per_lane = G == 1 ? K : 1;
    const int seed_items = (nf > 0 && nfm > 0) ? nfm * G : 0;
    const int seed_pad = (seed_items + 63) & ~63;      // seeding and following never share a wave
    const int follow_items = follow_next ? n_keep : 0;
    const int total = seed_pad + follow_items;

    for (int base = 0; base < total; base += B) {
        const int g = base + (int)tid<B>();
        const int g_wave = uni(base + ((int)tid<B>() & ~63));
        if (g_wave >= seed_pad) {
            const int a = g - seed_pad;
            if (a < follow_items) {
                const int r = at(nxt, a);
                const Rec R = at(v.rec(), r);
                float bsc;
                const uint32_t pb = follow_item<kLds>(P, wn, Zn, own, v.claim(), lclaim, R, t + 1, bsc);
                put_result<kLds, CAP>(v, a, r, pb, bsc, R);
            }
            continue;
        }
        // the seeding waves carry the longest dependency chain of the step
        __builtin_amdgcn_s_setprio(2);
        const int i = g / G, c = g - i * G;
        unsigned long long bkey = ~0ull;
        uint32_t bpos = 0;
        Hit16 h1;
        h1.x = h1.y = h1.z = 0.0f;
        h1.qid = 0;
        if (g < seed_items) {
            const int p1 = at(FM, i);
            h1 = at(wb.h, p1);
            int s0;
            if (kCand) {
                s0 = (int)at(v.keys(), (uint32_t)(uni(S.mo[kmod(P, t - 1)]) + p1));
            } else {
                s0 = win_lower_bound<kLds>(wa, q_of(h1));
                if (s0 == na) s0 = 0;
            }
            const int j = at(FR, s0);   // first unflagged position >= s0, as an index into F
            if (G == 4) {
                const int pos0 = pendulum_quad(F, nf, j, s0, na, hu, hd, c);
                if (pos0 >= 0)
                    seed_doublet<kLds>(wa, wc, own, cfree, pos0, h1.x, h1.y, h1.z, Zc, Ss, Ws, span, bkey, bpos);
            } else {
                for (int cc = 0; cc < per_lane; ++cc) {
                    const int pos0 = pendulum_pick(F, nf, j, s0, na, hu, hd, c + cc);
                    if (pos0 < 0) break;
                    seed_doublet<kLds>(wa, wc, own, cfree, pos0, h1.x, h1.y, h1.z, Zc, Ss, Ws, span, bkey, bpos);
                }
            }
        }
        // minimum over the G lanes of a middle hit (keys are unique or ~0)
        for (int m = 1; m < G; m <<= 1) {
            const uint32_t olo = (uint32_t)lane_xor((int)(uint32_t)bkey, m);
            const uint32_t ohi = (uint32_t)lane_xor((int)(uint32_t)(bkey >> 32), m);
            const uint32_t opos = (uint32_t)lane_xor((int)bpos, m);
            const unsigned long long o = ((unsigned long long)ohi << 32) | olo;
            if (o < bkey) {
                bkey = o;
                bpos = opos;
            }
        }
        const bool emit = bkey != ~0ull && c == 0 && g < seed_items;
        int r, l;
        wave_append2(emit, &S.cnt[0], emit, n_nxt, r, l);
        if (emit) {
            if (kLds && l >= CAP) {
                S.ovf = 1;
            } else {
                const int pos0 = (int)(bpos & 0xFFFFu), pos2 = (int)(bpos >> 16);
                const Hit16 h0 = at(wa.h, pos0);
                const Hit16 h2 = at(wc.h, pos2);
                const float x1 = h1.x, y1 = h1.y, z1 = h1.z;
                Rec R;
                const float d12 = h2.z - z1;
                R.xb = h2.x; R.yb = h2.y; R.zb = h2.z;
                R.tx = (h2.x - x1) / d12;
                R.ty = (h2.y - y1) / d12;
                R.key = id_of(h1); R.h0 = id_of(h0); R.h1 = id_of(h1); R.h2 = id_of(h2); R.last = id_of(h2);
                R.len = 3; R.last_t = (uint8_t)t;
                at(v.rec(), r) = R;
                // tracklet fit of the seed, hits in traversal order (Section 3,
                // "Tracklet filter"): chi2 = ((v.x)^2 + (v.y)^2) / (v.v) with
                // v = (z2-z1, z0-z2, z1-z0) orthogonal to (1,1,1) and to z
                const float v0 = h2.z - z1, v1 = h0.z - h2.z, v2 = z1 - h0.z;
                const float ssx = ((v0 * h0.x) + (v1 * x1)) + (v2 * h2.x);
                const float ssy = ((v0 * h0.y) + (v1 * y1)) + (v2 * h2.y);
                const float n2 = ((v0 * v0) + (v1 * v1)) + (v2 * v2);
                at(v.aux(), r).chi2 = ((ssx * ssx) + (ssy * ssy)) / n2;
                at(nxt, l) = (uint16_t)r;
                if (follow_next) {
                    float bsc;
                    const uint32_t pb = follow_item<kLds>(P, wn, Zn, own, v.claim(), lclaim, R, t + 1, bsc);
                    put_result<kLds, CAP>(v, l, r, pb, bsc, R);
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
    }
}

// A track wins iff its key is the minimum on every hit it claimed; winners
// append their best hit and flag their claim set.  Tracks that have now missed
// more than max_consecutive_misses modules in a row become final; the others
// stay active for the next module.
template <int B, bool kLds, int CAP>
__device__ void stage_follow_resolve(const sbt_params &PP, const Ev &v0, int t, Shared<B> &S, uint32_t *own,
                                     const uint16_t *act, int n_act, uint16_t *nxt, int *n_nxt)
{
    const Prm P = fresh(PP);
    const Ev v = fresh(v0);
    const Win wc = window<B, kLds, CAP>(P, S, v, t);
    const unsigned long long *__restrict__ claim = v.claim();
    uint16_t *fin = v.list(kListFin);
    for (int base = 0; base < n_act; base += B) {
        const int a = base + (int)tid<B>();
        bool done = false, keep = false;
        int r = 0;
        if (a < n_act) {
            r = at(act, a);
            uint32_t pb, k0 = 0, k12 = 0;
            float bsc;
            if (kLds) {
                const uint4 w = Lay<CAP>::res(v.lo)[a];
                pb = w.x;
                bsc = __uint_as_float(w.y);
                k0 = w.z;
                k12 = w.w;
            } else {
                const RecAux &x = at(v.aux(), r);
                pb = x.best;
                bsc = x.bsc;
            }
            Rec R = at(v.rec(), r);
            if (!kLds) {
                k0 = (uint32_t)R.key | ((uint32_t)(R.len == 3 ? R.h0 : kNone) << 16);
                k12 = (uint32_t)R.h1 | ((uint32_t)R.h2 << 16);
            }
            bool win = false;
            if (pb != 0xFFFFFFFFu) {
                const uint16_t best = (uint16_t)(pb & 0xFFFF);
                const unsigned long long kap = claim_key(bsc, (uint16_t)(k0 & 0xFFFFu), t);
                const uint16_t h0 = (uint16_t)(k0 >> 16);
                win = kLds ? Lay<CAP>::lclaim(v.lo)[pb >> 16] == kap : at(claim, best) == kap;
                if (h0 != kNone)
                    win = win && at(claim, h0) == kap && at(claim, (uint16_t)(k12 & 0xFFFFu)) == kap &&
                          at(claim, (uint16_t)(k12 >> 16)) == kap;
            }
            int last_t = R.last_t;
            if (win) {
                const uint16_t best = (uint16_t)(pb & 0xFFFF);
                const int bpos = (int)(pb >> 16);
                set_flag(own, best);
                if (R.len == 3) {
                    set_flag(own, R.h0);
                    set_flag(own, R.h1);
                    set_flag(own, R.h2);
                }
                at(v.link(), 2u * best) = R.last;
                const Hit16 hn = at(wc.h, bpos);
                const float dab = hn.z - R.zb;
                R.tx = (hn.x - R.xb) / dab;
                R.ty = (hn.y - R.yb) / dab;
                R.xb = hn.x; R.yb = hn.y; R.zb = hn.z;
                R.last = best;
                R.len = (uint8_t)(R.len + 1);
                R.last_t = (uint8_t)t;
                at(v.rec(), r) = R;
                last_t = t;
            }
            done = (t - last_t) >= P.misses + 1;
            keep = !done;
        }
        int f, l;
        wave_append2(done, &S.cnt[3], keep, n_nxt, f, l);
        if (done) at(fin, f) = (uint16_t)r;
        if (keep) {
            if (kLds && l >= CAP) S.ovf = 1;
            else at(nxt, l) = (uint16_t)r;
        }
    }
}

// whether an event fits the LDS instantiation of the tracking stages
template <int B, int CAP>
__device__ __forceinline__ bool event_fits_lds(const Shared<B> &S, int N, int own_cap)
{
    return CAP > 0 && uni(S.maxmod) <= CAP && N <= own_cap;
}

// Seeding and following over all modules.  Leaves the final record list in
// the final list and its length in S.cnt[3]; with writeback the LDS flags are
// copied to memory.  The LDS instantiation returns false when an active list
// outgrew its LDS capacity (the event is then run again from memory).
template <int B, bool kLds, int CAP, bool kCand = false>
__device__ bool stage_track_impl(const sbt_params &PP, const Ev &v, Shared<B> &S, bool writeback)
{
    const Prm P = fresh(PP);
    const int M = P.M, N = v.N;
    uint32_t *own = kLds ? Lay<CAP>::own(v.lo) : v.own();
    const int nw = (N + 31) >> 5;
    for (int i = tid<B>(); i < nw; i += B) at(own, i) = 0u;
    for (int i = tid<B>(); i < N; i += B) {
        at(v.claim(), i) = kNoClaim;
        at(v.link(), 2u * i + 1u) = kNone;
    }
    if (tid<B>() == 0) {
        S.cnt[0] = 0; S.cnt[1] = 0; S.cnt[2] = 0; S.cnt[3] = 0;
        S.ovf = 0;
    }
    if (kLds)
        for (int u = 0; u < 4 && u < M; ++u) ring_fill<B, CAP>(P, v, u, S, 0);
    ev_sync<B>();
    uint16_t *l0 = kLds ? Lay<CAP>::al(v.lo, 0) : v.list(kListAct0);
    uint16_t *l1 = kLds ? Lay<CAP>::al(v.lo, 1) : v.list(kListAct1);
    // the last traversal index whose seeding can make a seed: its modules
    // t-2, t-1 and t all hold hits (2 when no index can)
    int last_seed = 2;
    for (int u = M - 1; u > 2; --u) {
        const int k0 = kmod(P, u), k1 = kmod(P, u - 1), k2 = kmod(P, u - 2);
        if (S.mo[k0 + 1] > S.mo[k0] && S.mo[k1 + 1] > S.mo[k1] && S.mo[k2 + 1] > S.mo[k2]) {
            last_seed = u;
            break;
        }
    }
    last_seed = uni(last_seed);
    int par = 0;
    stage_seed_follow<B, kLds, CAP, kCand>(PP, v, 2, S, own, l0, &S.cnt[1], 0, M > 3);
    ev_sync<B>();
    if (kLds && uni(S.ovf)) return false;
    for (int t = 3; t < M; ++t) {
        // act (n_act tracks) holds every forming track with its search into
        // t done: resolve t keeping the survivors in nxt, then seed t and
        // search t+1
        const int n_act = uni(S.cnt[1 + par]);
        // with no forming track and no seed possible from here on, the
        // remaining steps change nothing
        if (n_act == 0 && t > last_seed) break;
        uint16_t *act = par ? l1 : l0;
        uint16_t *nxt = par ? l0 : l1;
        const bool more = t + 1 < M;
        stage_follow_resolve<B, kLds, CAP>(PP, v, t, S, own, act, n_act, nxt, &S.cnt[1 + (par ^ 1)]);
        if (kLds && more) {
            // module t+1 into the slot of t-3 (unused from here on), on the
            // waves the resolution leaves idle (the last wave at least)
            const int last = n_act > 0 ? n_act - ((n_act - 1) / B) * B : 0;
            int l0 = (last + 63) & ~63;
            if (l0 > B - 64) l0 = B - 64;
            ring_fill<B, CAP>(fresh(PP), fresh(v), t + 1, S, l0);
        }
        ev_sync<B>();
        const int n_keep = uni(S.cnt[1 + (par ^ 1)]);
        if (tid<B>() == 0) S.cnt[1 + par] = 0;   // act becomes the next step's nxt
        if (!(kLds && uni(S.ovf)))
            stage_seed_follow<B, kLds, CAP, kCand>(PP, v, t, S, own, nxt, &S.cnt[1 + (par ^ 1)], n_keep, more);
        ev_sync<B>();
        if (kLds && uni(S.ovf)) return false;
        par ^= 1;
    }
    const int n_act = uni(S.cnt[1 + par]);
    const int nf = uni(S.cnt[3]);
    const uint16_t *act = par ? l1 : l0;
    uint16_t *fin = v.list(kListFin);
    for (int a = tid<B>(); a < n_act; a += B) at(fin, nf + a) = at(act, a);
    if (kLds && writeback)
        for (int i = tid<B>(); i < nw; i += B) at(v.own(), i) = at(own, i);
    ev_sync<B>();
    if (tid<B>() == 0) S.cnt[3] = nf + n_act;
    ev_sync<B>();
    return true;
}

// Runs the tracking stages; returns true when the event's flags ended in LDS.
template <int B, int CAP, bool kCand = false>
__device__ bool stage_track(const sbt_params &P, const Ev &v, Shared<B> &S, int own_cap, bool writeback)
{
    if constexpr (CAP > 0) {
        if (event_fits_lds<B, CAP>(S, v.N, own_cap)) {
            if (stage_track_impl<B, true, CAP, kCand>(P, v, S, writeback)) return true;
        }
    }
    stage_track_impl<B, false, CAP, kCand>(P, v, S, false);
    return false;
}

// ---------------------------------------------------------------- candidate pass
// The paper's separate "Fill candidates" step, as an ablation of the fused
// search: for every hit of every module after the first in traversal order,
// the first position of the preceding module (in traversal order: the
// doublet module when this hit is a middle hit) whose phi16 is >= the hit's,
// 0 when there is none -- the pendulum start, which does not depend on the
// flags.  Written by sorted position into the keys array (free after the
// sort) for the seeding stage to read.
template <int B>
__device__ void stage_fill_candidates(const sbt_params &PP, const Ev &v0, const Shared<B> &S)
{
    const Ev v = fresh(v0);
    const Prm P = fresh(PP);
    for (int u = 1; u < P.M; ++u) {
        const int k = kmod(P, u), ka = kmod(P, u - 1);
        const int g0 = S.mo[k], n = S.mo[k + 1] - g0;
        Win wa;
        wa.h = v.hs() + S.mo[ka];
        wa.n = S.mo[ka + 1] - S.mo[ka];
        wa.tab = nullptr;
        for (int i = tid<B>(); i < n; i += B) {
            int s0 = wa.n > 0 ? win_lower_bound<false>(wa, q_of(at(v.hs(), (uint32_t)(g0 + i)))) : 0;
            if (s0 == wa.n) s0 = 0;
            at(v.keys(), (uint32_t)(g0 + i)) = (uint32_t)s0;
        }
    }
}

// ---------------------------------------------------------------- tracklet filter
// Tracks of >= 4 hits are accepted; a three-hit track is a candidate when its
// fit chi2 is under the threshold and none of its hits is flagged; candidates
// sharing hits keep the one with the minimum (chi2, key).
template <int B>
__device__ void stage_filter(const sbt_params &PP, const Ev &v0, int n_fin, const uint32_t *own)
{
    const Ev v = fresh(v0);
    const float X = fresh(PP).X;
    unsigned long long *__restrict__ claim = v.claim();
    const uint16_t *fin = v.list(kListFin);
    for (int a = tid<B>(); a < n_fin; a += B) {
        const int r = at(fin, a);
        const Rec R = at(v.rec(), r);
        uint32_t fl = 0;
        if (R.len >= 4) {
            fl = kFlagAccepted;
        } else {
            const float c2 = at(v.aux(), r).chi2;
            if (c2 < X && is_free(own, R.h0) && is_free(own, R.h1) && is_free(own, R.h2)) {
                const unsigned long long kap = claim_key(c2, R.key, kFilterStage);
                atomicMin(&at(claim, R.h0), kap);
                atomicMin(&at(claim, R.h1), kap);
                atomicMin(&at(claim, R.h2), kap);
                fl = kFlagCandidate;
            }
        }
        at(v.aux(), r).flag = fl;
    }
    ev_sync<B>();
    for (int a = tid<B>(); a < n_fin; a += B) {
        const int r = at(fin, a);
        const RecAux x = at(v.aux(), r);
        uint32_t fl = x.flag;
        const Rec R = at(v.rec(), r);
        if (fl == kFlagCandidate) {
            const unsigned long long kap = claim_key(x.chi2, R.key, kFilterStage);
            fl = (at(claim, R.h0) == kap && at(claim, R.h1) == kap && at(claim, R.h2) == kap) ? kFlagAccepted : 0;
        }
        if (fl == kFlagAccepted) at(v.link(), 2u * R.key + 1u) = (uint16_t)r;
    }
    ev_sync<B>();
}

// ---------------------------------------------------------------- per-event compaction
// The accepted tracks in key order (the id of the seed's middle hit), each as
// its three seed hits followed by the hits appended to it in traversal order:
// per-event track offsets and hit ids into the staging arrays, counts into
// the event's counters.
constexpr int kCompactBatch = 8;   // key rounds whose link loads are in flight together

// Whether the LDS form of the compaction fits: the previous-hit links (2 B
// per hit) and the record of each accepted track in key order (2 B per
// track; tracks are disjoint with at least three hits, so at most N / 3).
__host__ __device__ inline bool compact_fits_lds(int N, int lds_bytes)
{
    return (int)a16(2u * (uint32_t)N) + 2 * (N / 3 + 1) <= lds_bytes;
}

// LDS form.  Pass 1 takes the keys in rounds of B (key = round * B + lane,
// loads coalesced, kCompactBatch rounds in flight), copies each previous-hit
// link to LDS and ranks the keys that own a record with a ballot count over
// the workgroup, which lists the records in key order.  Pass 2 gives each
// listed track a lane: an exclusive scan of the lengths places its hits, and
// the lane writes them, walking the links in LDS.
template <int B>
__device__ void compact_lds(const Ev &v, int *s_scan, int lds_bytes)
{
    const int N = v.N;
    uint16_t *lprev = reinterpret_cast<uint16_t *>(g_lds + v.lo);
    uint16_t *lrec = reinterpret_cast<uint16_t *>(g_lds + v.lo + a16(2u * (uint32_t)N));
    const int rec_cap = (lds_bytes - (int)a16(2u * (uint32_t)N)) / 2;
    const uint32_t *link = reinterpret_cast<const uint32_t *>(v.link());   // prev | record << 16
    const int rounds = (N + B - 1) / B;
    bool bad = false;
    int nt = 0;
    for (int j0 = 0; j0 < rounds; j0 += kCompactBatch) {
        uint32_t w[kCompactBatch];
#pragma unroll
        for (int u = 0; u < kCompactBatch; ++u) {
            const int k = (j0 + u) * B + (int)tid<B>();
            w[u] = k < N ? at(link, (uint32_t)k) : ((uint32_t)kNone << 16);
        }
#pragma unroll
        for (int u = 0; u < kCompactBatch; ++u) {
            if (j0 + u >= rounds) break;
            const int k = (j0 + u) * B + (int)tid<B>();
            const uint16_t r = (uint16_t)(w[u] >> 16);
            if (k < N) lprev[k] = (uint16_t)(w[u] & 0xFFFFu);
            int tot;
            const int pos = nt + (block_count2<B>(r != kNone, false, s_scan, j0 + u, &tot) & 0xFFFF);
            if (r != kNone) {
                if (pos < rec_cap) lrec[pos] = r;
                else bad = true;
            }
            nt += tot & 0xFFFF;
        }
    }
    ev_sync<B>();   // links and the record list visible
    if (nt > rec_cap) nt = 0;
    int nh = 0;
    for (int t0 = 0; t0 < nt; t0 += B) {
        const int t = t0 + (int)tid<B>();
        Rec R;
        int len = 0;
        if (t < nt) {
            R = at(v.rec(), lrec[t]);
            len = R.len;
        }
        int tot;
        const int hi = nh + block_excl_scan<B>(len, s_scan, t0 / B, &tot);
        nh += tot;
        if (t < nt) {
            // tracks are disjoint, so hi + len <= N; the checks below only
            // keep a broken invariant from turning into a stray access
            if (hi + len > N) {
                bad = true;
            } else {
                at(v.st_toff(), t) = hi;
                uint16_t *out = v.st_hits() + hi;
                uint16_t p = R.last;
                for (int j = len - 1; j >= 3; --j) {
                    if (p >= N) { bad = true; break; }
                    out[j] = p;
                    p = lprev[p];
                }
                out[2] = R.h2;
                out[1] = R.h1;
                out[0] = R.h0;
            }
        }
    }
    if (bad) v.info().st = (int)SBT_EV_INTERNAL;
    if (tid<B>() == 0) {
        v.info().nt = nh <= N ? nt : 0;
        v.info().nh = nh <= N ? nh : 0;
    }
}

// Memory form (events whose links do not fit, and the plain kernel): each
// lane owns a contiguous range of keys; it counts their tracks and hits, one
// scan of each over the workgroup, then it writes them in key order.
template <int B>
__device__ void compact_mem(const Ev &v, int *s_scan)
{
    const int N = v.N;
    const int per = (N + B - 1) / B;
    const int k0 = min(N, (int)tid<B>() * per), k1 = min(N, k0 + per);
    int nt = 0, nh = 0;
    for (int k = k0; k < k1; ++k) {
        const uint16_t r = at(v.link(), 2u * k + 1u);
        if (r != kNone) {
            ++nt;
            nh += at(v.rec(), r).len;
        }
    }
    int tt, th;
    int ti = block_excl_scan<B>(nt, s_scan, 0, &tt);
    int hi = block_excl_scan<B>(nh, s_scan, 1, &th);
    bool bad = th > N;
    for (int k = k0; k < k1 && !bad; ++k) {
        const uint16_t r = at(v.link(), 2u * k + 1u);
        if (r == kNone) continue;
        const Rec R = at(v.rec(), r);
        if (hi + R.len > N) {
            bad = true;
            break;
        }
        at(v.st_toff(), ti) = hi;
        uint16_t *out = v.st_hits() + hi;
        uint16_t p = R.last;
        for (int j = R.len - 1; j >= 3; --j) {
            if (p >= N) { bad = true; break; }
            out[j] = p;
            p = at(v.link(), 2u * p);
        }
        out[2] = R.h2;
        out[1] = R.h1;
        out[0] = R.h0;
        ++ti;
        hi += R.len;
    }
    if (bad) v.info().st = (int)SBT_EV_INTERNAL;
    if (tid<B>() == 0) {
        v.info().nt = th <= N ? tt : 0;
        v.info().nh = th <= N ? th : 0;
    }
}

// lds_bytes: LDS free for the compaction (0: none)
template <int B>
__device__ void stage_compact(const Ev &v0, int *s_scan, int lds_bytes)
{
    const Ev v = fresh(v0);
    if (compact_fits_lds(v.N, lds_bytes)) compact_lds<B>(v, s_scan, lds_bytes);
    else compact_mem<B>(v, s_scan);
}

}  // namespace sbt
