// Serving loop: continuous batching of single events over resident device
// slots (the C ABI in include/sbt.h, "serving").
//
// Each slot owns, for the server's lifetime, device inputs and workspace for
// up to slot_events events / slot_hits hits, pinned host staging of the
// inputs, a stream (default priority) and a completion event.  Events queued
// by sbt_server_submit are packed into the slot that is open for admission; a
// slot is launched (one H2D copy, batched reconstruction, completion event,
// all on its stream) when it cannot take the next queued event, when its
// oldest event has waited max_wait_us, or at once when no other slot is on
// the device.  While slots are in flight, newly arriving events are admitted
// into free slots, so their work overlaps on the device.  An event's tracks
// depend only on its own hits, so a result is the same whether the event ran
// alone or in a mix.
//
// The reconstruction writes each event's tracks, as a CSR of its own, straight
// into a pinned host result block that the returned results point into; blocks
// are recycled once no result refers to them.  No copy engine runs after the
// kernels, so a slot's H2D copy never queues behind another slot's output
// copy waiting for its kernels, and the host does not copy results.  The hits
// of a slot's events are copied into its pinned staging at launch by a small
// pool of threads owned by the server, in parallel over events; with
// binary16 transfer the same threads round them to 8-byte records on the way.
#include <hip/hip_runtime.h>
#include <immintrin.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "sbt.h"
#include "sbt_internal.h"

namespace {

double now_us()
{
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

struct QueuedEvent {
    int64_t id;
    double t_submit;
    int32_t mo[SBT_MAX_MODULES + 1];   // local offsets
    std::vector<float> xyz;            // x[n], y[n], z[n] (owned copy)
    const float *bx, *by, *bz;         // borrowed hits (load replay), or null
    int32_t n;
};

// an admitted event: its hits are copied into the slot's staging at launch
struct SlotEvent {
    int64_t id;
    double t_submit;
    int32_t base;                      // first hit in the slot
    int32_t n;
    const float *x, *y, *z;
    std::vector<float> own;            // owned hits, if the event brought its own copy
};

// Runs fn(i), i in [0, n), on the pool's threads and the caller; returns when
// every index is done.
class Pool {
public:
    explicit Pool(int n_threads)
    {
        for (int i = 0; i < n_threads; ++i) th_.emplace_back([this] { work(); });
    }
    ~Pool()
    {
        {
            std::lock_guard<std::mutex> g(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto &t : th_) t.join();
    }
    void run(int n, const std::function<void(int)> &fn)
    {
        if (n <= 0) return;
        if (th_.empty() || n == 1) {
            for (int i = 0; i < n; ++i) fn(i);
            return;
        }
        {
            std::lock_guard<std::mutex> g(m_);
            fn_ = &fn;
            n_ = n;
            next_.store(0);
            finished_ = 0;
            ++gen_;
        }
        cv_.notify_all();
        for (int i; (i = next_.fetch_add(1)) < n;) fn(i);
        std::unique_lock<std::mutex> lk(m_);
        done_cv_.wait(lk, [this] { return finished_ == (int)th_.size(); });
        fn_ = nullptr;
    }

private:
    void work()
    {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int)> *fn;
            int n;
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                fn = fn_;
                n = n_;
            }
            for (int i; (i = next_.fetch_add(1)) < n;) (*fn)(i);
            {
                std::lock_guard<std::mutex> g(m_);
                ++finished_;
            }
            done_cv_.notify_one();
        }
    }
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_cv_;
    const std::function<void(int)> *fn_ = nullptr;
    int n_ = 0;
    std::atomic<int> next_{0};
    int finished_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

enum SlotState { kFree = 0, kOpen = 1, kInFlight = 2 };

// Tracks of one launch, in pinned host memory the device writes: per event
// its status, track count (eto), offsets from zero and hit ids.
struct ResultBlock {
    char *mem = nullptr;
    int32_t *eto = nullptr, *st = nullptr, *hoff = nullptr, *tho = nullptr, *th = nullptr;
    ~ResultBlock()
    {
        if (mem) (void)hipHostFree(mem);
    }
};

struct Slot {
    // device inputs (event and module offsets, then x, y, z packed for the
    // launch's hit count) and workspace
    char *dmem = nullptr;
    void *dwork = nullptr;
    // pinned host staging, same layout as the device inputs
    char *hin = nullptr;
    int32_t *heo = nullptr, *hmo = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    SlotState state = kFree;
    int32_t n_events = 0, n_hits = 0;
    double t_oldest = 0.0;
    std::vector<SlotEvent> events;
    std::shared_ptr<ResultBlock> block;   // written by the launch in flight
};

struct ReadyResult {
    sbt_server_result r;
    std::shared_ptr<ResultBlock> block;
    size_t tho_at, th_at;
};

}  // namespace

struct sbt_server {
    sbt_params params;
    sbt_tuning tuning;
    bool per_launch_tuning;  // no tuning given: chosen per launch from the slot's shape
    int cus;                 // compute units of the device
    sbt_server_config cfg;
    std::vector<Slot> slots;
    std::deque<QueuedEvent> queue;
    size_t max_queue;
    int open_slot;           // index of the slot admitting events, or -1
    std::vector<std::shared_ptr<ResultBlock>> store;   // blocks of the results last returned
    std::deque<ReadyResult> ready;                      // completed, not yet returned
    std::vector<std::shared_ptr<ResultBlock>> blocks;   // every result block (recycled)
    std::unique_ptr<Pool> pool;
};

namespace {

// byte layout of one slot's inputs (the same on the device and in the pinned
// staging) and of a result block
struct SlotLayout {
    size_t eo, mo, xyz, in_total;                  // inputs: x, y, z from xyz on
    size_t work, device_total;
    size_t r_eto, r_st, r_hoff, r_tho, r_th, r_total;   // result block
};

SlotLayout slot_layout(const sbt_server_config &c, int M)
{
    SlotLayout L;
    const size_t H = (size_t)c.slot_hits, E = (size_t)c.slot_events;
    size_t o = 0;
    L.eo = o; o += align_up(4 * (E + 1));
    L.mo = o; o += align_up(4 * (E * M + 1));
    L.xyz = o; o += c.coords_f16 ? align_up(8 * H) : 3 * align_up(4 * H);
    L.in_total = o;
    L.work = align_up(sbt::workspace_bytes(c.slot_events, c.slot_hits));
    L.device_total = L.in_total + L.work;
    size_t r = 0;
    L.r_eto = r; r += align_up(4 * (E + 1));
    L.r_st = r; r += align_up(4 * E);
    L.r_hoff = r; r += align_up(4 * E);
    L.r_tho = r; r += align_up(4 * (H / 3 + E + 1));   // tracks have >= 3 distinct hits
    L.r_th = r; r += align_up(4 * H);
    L.r_total = r;
    return L;
}

// bytes from one of x, y, z to the next for a launch of H hits
size_t xyz_stride(size_t H) { return align_up(4 * H); }

// Binary16 records of n hits, each x | y << 16 and z (upper half zero) in two
// 32-bit words, the layout of sbt_hits_f16; every coordinate is rounded to
// the nearest binary16, ties to even.  Eight hits per step with the F16C
// conversion, the rest one by one.
__attribute__((target("avx,f16c"))) void half_records_f16c(const float *x, const float *y, const float *z, int n,
                                                           uint16_t *out)
{
    const __m128i zero = _mm_setzero_si128();
    int i = 0;
    for (; i + 8 <= n; i += 8) {
        const __m128i hx = _mm256_cvtps_ph(_mm256_loadu_ps(x + i), _MM_FROUND_TO_NEAREST_INT);
        const __m128i hy = _mm256_cvtps_ph(_mm256_loadu_ps(y + i), _MM_FROUND_TO_NEAREST_INT);
        const __m128i hz = _mm256_cvtps_ph(_mm256_loadu_ps(z + i), _MM_FROUND_TO_NEAREST_INT);
        const __m128i xy_lo = _mm_unpacklo_epi16(hx, hy), xy_hi = _mm_unpackhi_epi16(hx, hy);
        const __m128i z_lo = _mm_unpacklo_epi16(hz, zero), z_hi = _mm_unpackhi_epi16(hz, zero);
        __m128i *o = reinterpret_cast<__m128i *>(out + 4 * (size_t)i);
        _mm_storeu_si128(o + 0, _mm_unpacklo_epi32(xy_lo, z_lo));
        _mm_storeu_si128(o + 1, _mm_unpackhi_epi32(xy_lo, z_lo));
        _mm_storeu_si128(o + 2, _mm_unpacklo_epi32(xy_hi, z_hi));
        _mm_storeu_si128(o + 3, _mm_unpackhi_epi32(xy_hi, z_hi));
    }
    for (; i < n; ++i) {
        out[4 * (size_t)i + 0] = _cvtss_sh(x[i], _MM_FROUND_TO_NEAREST_INT);
        out[4 * (size_t)i + 1] = _cvtss_sh(y[i], _MM_FROUND_TO_NEAREST_INT);
        out[4 * (size_t)i + 2] = _cvtss_sh(z[i], _MM_FROUND_TO_NEAREST_INT);
        out[4 * (size_t)i + 3] = 0;
    }
}

// the same without F16C
void half_records_portable(const float *x, const float *y, const float *z, int n, uint16_t *out)
{
    for (int i = 0; i < n; ++i) {
        out[4 * (size_t)i + 0] = __builtin_bit_cast(uint16_t, (_Float16)x[i]);
        out[4 * (size_t)i + 1] = __builtin_bit_cast(uint16_t, (_Float16)y[i]);
        out[4 * (size_t)i + 2] = __builtin_bit_cast(uint16_t, (_Float16)z[i]);
        out[4 * (size_t)i + 3] = 0;
    }
}

void half_records(const float *x, const float *y, const float *z, int n, uint16_t *out)
{
    static const bool f16c = __builtin_cpu_supports("f16c") && __builtin_cpu_supports("avx");
    if (f16c) half_records_f16c(x, y, z, n, out);
    else half_records_portable(x, y, z, n, out);
}

void free_slot(Slot &s)
{
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.dmem) (void)hipFree(s.dmem);
    if (s.hin) (void)hipHostFree(s.hin);
    s = Slot();
}

int init_slot(Slot &s, const SlotLayout &L)
{
    if (hipMalloc(&s.dmem, L.device_total) != hipSuccess) return SBT_ERR_NOMEM;
    if (hipHostMalloc(&s.hin, L.in_total, hipHostMallocDefault) != hipSuccess) return SBT_ERR_NOMEM;
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return SBT_ERR_HIP;
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return SBT_ERR_HIP;
    s.dwork = s.dmem + L.in_total;
    s.heo = (int32_t *)(s.hin + L.eo);
    s.hmo = (int32_t *)(s.hin + L.mo);
    s.state = kFree;
    return SBT_OK;
}

std::shared_ptr<ResultBlock> new_block(const SlotLayout &L)
{
    std::shared_ptr<ResultBlock> b(new (std::nothrow) ResultBlock());
    if (!b || hipHostMalloc(&b->mem, L.r_total, hipHostMallocDefault) != hipSuccess) return nullptr;
    b->eto = (int32_t *)(b->mem + L.r_eto);
    b->st = (int32_t *)(b->mem + L.r_st);
    b->hoff = (int32_t *)(b->mem + L.r_hoff);
    b->tho = (int32_t *)(b->mem + L.r_tho);
    b->th = (int32_t *)(b->mem + L.r_th);
    return b;
}

// Result blocks a server may hold: one per slot on the device, one per slot
// for results completed since the last poll and one per slot for the results
// that poll returned (valid until the next), and two more.  Past that, which
// only a caller leaving completed results unreturned reaches, launches wait
// until its polls release blocks.
size_t max_blocks(const sbt_server *srv) { return 3 * srv->slots.size() + 2; }

// A launch that has to wait for a result block (internal, never returned).
constexpr int kWaitForBlock = 1;

// a block no slot or result refers to any more, else a new one; nullptr with
// *rc = kWaitForBlock at the limit, SBT_ERR_NOMEM when allocation fails
std::shared_ptr<ResultBlock> free_block(sbt_server *srv, const SlotLayout &L, int *rc)
{
    *rc = SBT_OK;
    for (auto &b : srv->blocks)
        if (b.use_count() == 1) return b;
    if (srv->blocks.size() >= max_blocks(srv)) {
        *rc = kWaitForBlock;
        return nullptr;
    }
    std::shared_ptr<ResultBlock> b = new_block(L);
    if (b) srv->blocks.push_back(b);
    else *rc = SBT_ERR_NOMEM;
    return b;
}

// Admits a queued event into an open slot: offsets now, hits at launch.
void pack(sbt_server *srv, Slot &s, QueuedEvent &q)
{
    const int M = srv->params.n_modules;
    if (s.n_events == 0) {
        s.heo[0] = 0;
        s.hmo[0] = 0;
        s.t_oldest = q.t_submit;
    }
    const int32_t base = s.n_hits;
    for (int k = 1; k <= M; ++k) s.hmo[(size_t)s.n_events * M + k] = base + q.mo[k];
    s.n_hits += q.n;
    s.n_events += 1;
    s.heo[s.n_events] = s.n_hits;
    SlotEvent se;
    se.id = q.id;
    se.t_submit = q.t_submit;
    se.base = base;
    se.n = q.n;
    if (q.bx) {
        se.x = q.bx;
        se.y = q.by;
        se.z = q.bz;
    } else {
        se.own = std::move(q.xyz);
        se.x = se.own.data();
        se.y = se.own.data() + q.n;
        se.z = se.own.data() + 2 * (size_t)q.n;
    }
    s.events.push_back(std::move(se));
}

// Launch configuration of a slot: the caller's, or when none was given the
// library's choice for the slot's size (at most one event per compute unit,
// or two large ones, run 1,024 lanes per event, so that each finishes sooner,
// which is what a lightly loaded server needs).
sbt_tuning launch_tuning(const sbt_server *srv, int E, int H)
{
    return srv->per_launch_tuning ? sbt::batch_tuning(E, H, srv->cus) : srv->tuning;
}

int launch(sbt_server *srv, Slot &s)
{
    const int M = srv->params.n_modules;
    const SlotLayout L = slot_layout(srv->cfg, M);
    const size_t E = (size_t)s.n_events, H = (size_t)s.n_hits;
    const size_t stride = xyz_stride(H);
    hipStream_t st = s.stream;
    int brc;
    std::shared_ptr<ResultBlock> block = free_block(srv, L, &brc);
    if (!block) return brc;
    // hits into the pinned staging, packed for this launch, in parallel over
    // events: x, y, z arrays, or binary16 records
    const bool f16 = srv->cfg.coords_f16 != 0;
    float *hx = (float *)(s.hin + L.xyz), *hy = (float *)(s.hin + L.xyz + stride),
          *hz = (float *)(s.hin + L.xyz + 2 * stride);
    uint16_t *h16 = (uint16_t *)(s.hin + L.xyz);
    srv->pool->run((int)s.events.size(), [&](int i) {
        SlotEvent &ev = s.events[(size_t)i];
        if (ev.n > 0) {
            if (f16) {
                half_records(ev.x, ev.y, ev.z, ev.n, h16 + 4 * (size_t)ev.base);
            } else {
                memcpy(hx + ev.base, ev.x, sizeof(float) * ev.n);
                memcpy(hy + ev.base, ev.y, sizeof(float) * ev.n);
                memcpy(hz + ev.base, ev.z, sizeof(float) * ev.n);
            }
        }
        std::vector<float>().swap(ev.own);
    });
    // offsets and hits in one copy
    const size_t in_bytes = L.xyz + (f16 ? 8 * H : 3 * stride);
    if (hipMemcpyAsync(s.dmem, s.hin, in_bytes, hipMemcpyHostToDevice, st) != hipSuccess) return SBT_ERR_HIP;
    sbt::EventOut out;
    out.eto = block->eto;
    out.status = block->st;
    out.hoff = block->hoff;
    out.tho = block->tho;
    out.th = block->th;
    const sbt_tuning tuning = launch_tuning(srv, (int)E, (int)H);
    int rc;
    if (f16) {
        sbt_hits_f16 hits;
        hits.n_events = (int32_t)E;
        hits.n_hits = (int32_t)H;
        hits.event_offsets = (const int32_t *)(s.dmem + L.eo);
        hits.module_offsets = (const int32_t *)(s.dmem + L.mo);
        hits.xyzw = (const uint16_t *)(s.dmem + L.xyz);
        rc = sbt::launch_batched_events_f16(srv->params, tuning, hits, out, s.dwork, st);
    } else {
        sbt_hits hits;
        hits.n_events = (int32_t)E;
        hits.n_hits = (int32_t)H;
        hits.event_offsets = (const int32_t *)(s.dmem + L.eo);
        hits.module_offsets = (const int32_t *)(s.dmem + L.mo);
        hits.x = (const float *)(s.dmem + L.xyz);
        hits.y = (const float *)(s.dmem + L.xyz + stride);
        hits.z = (const float *)(s.dmem + L.xyz + 2 * stride);
        rc = sbt::launch_batched_events(srv->params, tuning, hits, out, s.dwork, st);
    }
    if (rc) return rc;
    if (hipEventRecord(s.done, st) != hipSuccess) return SBT_ERR_HIP;
    s.block = std::move(block);
    s.state = kInFlight;
    return SBT_OK;
}

// Moves a completed slot's events to the ready queue; their results point
// into the slot's result block.
void collect(sbt_server *srv, Slot &s)
{
    const double t = now_us();
    const int32_t E = s.n_events;
    const ResultBlock &b = *s.block;
    for (int32_t i = 0; i < E; ++i) {
        ReadyResult rr;
        const int32_t t0 = b.eto[i], t1 = b.eto[i + 1];
        rr.r.request_id = s.events[(size_t)i].id;
        rr.r.status = b.st[i];
        rr.r.n_tracks = t1 - t0;
        rr.r.track_hit_offsets = nullptr;
        rr.r.track_hits = nullptr;
        rr.r.t_submit_us = s.events[(size_t)i].t_submit;
        rr.r.t_done_us = t;
        rr.block = s.block;
        rr.tho_at = (size_t)t0 + (size_t)i;
        rr.th_at = (size_t)b.hoff[i];
        srv->ready.push_back(std::move(rr));
    }
    s.block.reset();
    s.events.clear();
    s.n_events = 0;
    s.n_hits = 0;
    s.state = kFree;
}

int step(sbt_server *srv)
{
    // 1. collect completed slots
    int in_flight = 0;
    for (auto &s : srv->slots) {
        if (s.state != kInFlight) continue;
        hipError_t q = hipEventQuery(s.done);
        if (q == hipSuccess) collect(srv, s);
        else if (q == hipErrorNotReady) ++in_flight;
        else return SBT_ERR_HIP;
    }
    // 2. admit queued events into the open slot, opening free slots as needed
    const double t = now_us();
    while (!srv->queue.empty()) {
        if (srv->open_slot < 0) {
            for (size_t i = 0; i < srv->slots.size(); ++i)
                if (srv->slots[i].state == kFree) {
                    srv->open_slot = (int)i;
                    srv->slots[i].state = kOpen;
                    break;
                }
            if (srv->open_slot < 0) break;   // every slot is busy: events wait on the host
        }
        Slot &s = srv->slots[(size_t)srv->open_slot];
        QueuedEvent &q = srv->queue.front();
        if (s.n_events + 1 > srv->cfg.slot_events || s.n_hits + q.n > srv->cfg.slot_hits) {
            int rc = launch(srv, s);        // full: launch it and open another
            if (rc == kWaitForBlock) break;   // events wait on the host
            if (rc) return rc;
            ++in_flight;
            srv->open_slot = -1;
            continue;
        }
        pack(srv, s, q);
        srv->queue.pop_front();
    }
    // 3. launch the open slot when it waited long enough or the device is idle
    if (srv->open_slot >= 0) {
        Slot &s = srv->slots[(size_t)srv->open_slot];
        if (s.n_events > 0 && (in_flight == 0 || t - s.t_oldest >= (double)srv->cfg.max_wait_us)) {
            int rc = launch(srv, s);
            if (rc == kWaitForBlock) return SBT_OK;   // launched once a poll releases a block
            if (rc) return rc;
            srv->open_slot = -1;
        }
    }
    return SBT_OK;
}

}  // namespace

extern "C" {

int sbt_debug_half_records(const float *x, const float *y, const float *z, int32_t n, uint16_t *out)
{
    if (!x || !y || !z || !out || n < 0) return SBT_ERR_INVALID_ARG;
    half_records(x, y, z, n, out);
    return SBT_OK;
}

double sbt_now_us(void) { return now_us(); }

int sbt_server_create(const sbt_params *params, const sbt_tuning *tuning, const sbt_server_config *config,
                      sbt_server **out)
{
    int rc = sbt_params_validate(params);
    if (rc) return rc;
    if (!config || !out) return SBT_ERR_INVALID_ARG;
    const sbt_server_config &c = *config;
    if (c.n_slots < 1 || c.slot_events < 1 || c.slot_hits < SBT_MAX_EVENT_HITS || c.max_wait_us < 0 ||
        (c.coords_f16 != 0 && c.coords_f16 != 1))
        return SBT_ERR_INVALID_ARG;
    sbt_tuning t = tuning ? *tuning : sbt::default_tuning_config();
    if ((rc = sbt::tuning_valid(t))) return rc;
    const SlotLayout L = slot_layout(c, params->n_modules);
    if ((size_t)c.n_slots * L.device_total > c.device_budget_bytes) return SBT_ERR_WORKSPACE;
    sbt_server *srv = new (std::nothrow) sbt_server();
    if (!srv) return SBT_ERR_NOMEM;
    srv->params = *params;
    srv->tuning = t;
    srv->per_launch_tuning = tuning == nullptr;
    {
        int dev = 0;
        srv->cus = 256;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&srv->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            delete srv;
            return SBT_ERR_HIP;
        }
    }
    srv->cfg = c;
    srv->max_queue = (size_t)c.n_slots * (size_t)c.slot_events * 4;
    srv->open_slot = -1;
    {
        const unsigned hw = std::thread::hardware_concurrency();
        const int workers = (int)std::min(7u, hw > 1 ? hw - 1 : 0u);
        srv->pool.reset(new (std::nothrow) Pool(workers));
        if (!srv->pool) {
            delete srv;
            return SBT_ERR_NOMEM;
        }
    }
    srv->slots.resize((size_t)c.n_slots);
    for (auto &s : srv->slots) {
        if ((rc = init_slot(s, L))) {
            for (auto &x : srv->slots) free_slot(x);
            delete srv;
            return rc;
        }
    }
    // one result block per slot and one for the results last returned; more
    // (up to max_blocks) are added while callers leave results unreturned
    for (int i = 0; i <= c.n_slots; ++i) {
        std::shared_ptr<ResultBlock> b = new_block(L);
        if (!b) {
            for (auto &x : srv->slots) free_slot(x);
            delete srv;
            return SBT_ERR_NOMEM;
        }
        srv->blocks.push_back(std::move(b));
    }
    *out = srv;
    return SBT_OK;
}

void sbt_server_destroy(sbt_server *srv)
{
    if (!srv) return;
    for (auto &s : srv->slots)
        if (s.stream) (void)hipStreamSynchronize(s.stream);
    for (auto &s : srv->slots) free_slot(s);
    delete srv;
}

int sbt_server_submit(sbt_server *srv, int64_t request_id, int32_t n_hits, const int32_t *module_offsets,
                      const float *x, const float *y, const float *z)
{
    if (!srv || n_hits < 0 || !module_offsets) return SBT_ERR_INVALID_ARG;
    if (n_hits > 0 && (!x || !y || !z)) return SBT_ERR_INVALID_ARG;
    if (n_hits > SBT_MAX_EVENT_HITS) return SBT_ERR_EVENT_TOO_LARGE;
    const int M = srv->params.n_modules;
    if (module_offsets[0] != 0 || module_offsets[M] != n_hits) return SBT_ERR_INVALID_ARG;
    for (int k = 0; k < M; ++k)
        if (module_offsets[k + 1] < module_offsets[k]) return SBT_ERR_INVALID_ARG;
    if (srv->queue.size() >= srv->max_queue) return SBT_ERR_NOT_READY;
    QueuedEvent q;
    q.id = request_id;
    q.t_submit = now_us();
    q.bx = q.by = q.bz = nullptr;
    q.n = n_hits;
    for (int k = 0; k <= M; ++k) q.mo[k] = module_offsets[k];
    q.xyz.resize(3 * (size_t)n_hits);
    if (n_hits > 0) {
        memcpy(q.xyz.data(), x, sizeof(float) * n_hits);
        memcpy(q.xyz.data() + n_hits, y, sizeof(float) * n_hits);
        memcpy(q.xyz.data() + 2 * (size_t)n_hits, z, sizeof(float) * n_hits);
    }
    srv->queue.push_back(std::move(q));
    return SBT_OK;
}

int sbt_server_poll(sbt_server *srv, sbt_server_result *results, int32_t max_results, int32_t wait_us)
{
    if (!srv || (max_results > 0 && !results) || max_results < 0) return SBT_ERR_INVALID_ARG;
    srv->store.clear();
    const double t_end = now_us() + (wait_us > 0 ? (double)wait_us : 0.0);
    for (;;) {
        int rc = step(srv);
        if (rc) return rc;
        if (!srv->ready.empty() || now_us() >= t_end) break;
        std::this_thread::yield();
    }
    int32_t n = 0;
    while (n < max_results && !srv->ready.empty()) {
        ReadyResult &rr = srv->ready.front();
        results[n] = rr.r;
        results[n].track_hit_offsets = rr.block->tho + rr.tho_at;
        results[n].track_hits = rr.block->th + rr.th_at;
        if (srv->store.empty() || srv->store.back() != rr.block) srv->store.push_back(rr.block);
        srv->ready.pop_front();
        ++n;
    }
    return n;
}

int sbt_server_replay(sbt_server *srv, int32_t n_arrivals, const double *arrival_us, const int32_t *picks,
                      int32_t pool_events, const int32_t *event_offsets, const int32_t *module_offsets,
                      const float *x, const float *y, const float *z, double *latency_us, int32_t *n_tracks,
                      double *wall_us)
{
    if (!srv || n_arrivals < 0 || pool_events < 1 || !arrival_us || !picks || !event_offsets || !module_offsets ||
        !x || !y || !z || !latency_us || !wall_us)
        return SBT_ERR_INVALID_ARG;
    const int M = srv->params.n_modules;
    // results are indexed by arrival, so nothing submitted earlier may still
    // be pending: its request id could be any value
    int32_t queued = 0, in_flight = 0;
    sbt_server_pending(srv, &queued, &in_flight);
    if (queued != 0 || in_flight != 0) return SBT_ERR_NOT_READY;
    for (int32_t i = 0; i < n_arrivals; ++i) {
        if (picks[i] < 0 || picks[i] >= pool_events) return SBT_ERR_INVALID_ARG;
        const int32_t n = event_offsets[picks[i] + 1] - event_offsets[picks[i]];
        if (n < 0) return SBT_ERR_INVALID_ARG;
        if (n > SBT_MAX_EVENT_HITS) return SBT_ERR_EVENT_TOO_LARGE;
    }
    // room for every result the slots can complete at once, so that each
    // poll returns all of them and their result blocks are released promptly
    std::vector<sbt_server_result> res(
        std::max<size_t>(512, srv->slots.size() * (size_t)srv->cfg.slot_events));
    const double t0 = now_us();
    int32_t next = 0, done = 0;
    while (done < n_arrivals) {
        const double t = now_us() - t0;
        while (next < n_arrivals && arrival_us[next] <= t && srv->queue.size() < srv->max_queue) {
            const int32_t e = picks[next];
            const int32_t lo = event_offsets[e], hi = event_offsets[e + 1];
            QueuedEvent q;
            q.id = next;
            q.t_submit = t0 + arrival_us[next];
            q.n = hi - lo;
            for (int k = 0; k <= M; ++k) q.mo[k] = module_offsets[(size_t)e * M + k] - lo;
            q.bx = x + lo;
            q.by = y + lo;
            q.bz = z + lo;
            srv->queue.push_back(std::move(q));
            ++next;
        }
        int n = sbt_server_poll(srv, res.data(), (int32_t)res.size(), 0);
        if (n < 0) return n;
        for (int i = 0; i < n; ++i) {
            const int64_t id = res[(size_t)i].request_id;
            if (id < 0 || id >= n_arrivals) return SBT_ERR_INVALID_ARG;   // never expected: the server was idle
            latency_us[id] = res[(size_t)i].t_done_us - (t0 + arrival_us[id]);
            if (n_tracks) n_tracks[id] = res[(size_t)i].n_tracks;
            ++done;
        }
    }
    *wall_us = now_us() - t0;
    return SBT_OK;
}

int sbt_server_result_blocks(const sbt_server *srv, int32_t *n_blocks, int32_t *limit)
{
    if (!srv) return SBT_ERR_INVALID_ARG;
    if (n_blocks) *n_blocks = (int32_t)srv->blocks.size();
    if (limit) *limit = (int32_t)max_blocks(srv);
    return SBT_OK;
}

int sbt_server_pending(const sbt_server *srv, int32_t *queued, int32_t *in_flight)
{
    if (!srv) return SBT_ERR_INVALID_ARG;
    int32_t q = (int32_t)srv->queue.size(), f = 0;
    for (const auto &s : srv->slots)
        if (s.state != kFree) f += s.n_events;
    if (queued) *queued = q;
    if (in_flight) *in_flight = f + (int32_t)srv->ready.size();
    return SBT_OK;
}

}  // extern "C"
