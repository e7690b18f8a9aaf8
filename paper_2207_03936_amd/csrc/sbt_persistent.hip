// Batched form: a persistent work-stealing kernel that runs every stage of an
// event inside one workgroup and then takes the next event (largest first)
// from a device counter.  Built once per workgroup width (SBT_TPE).
#include <hip/hip_runtime.h>

#include "sbt.h"
#include "sbt_device.h"
#include "sbt_kernels.h"

#ifndef SBT_TPE
#error "SBT_TPE (workgroup width) must be defined"
#endif

using namespace sbt;

// One event per group of B lanes.  For B > 64 the group is the workgroup and
// its static LDS holds the event's Shared block.  For B = 64 a workgroup of
// any number of waves runs one event per wave, each with its own region of
// the dynamic LDS (the Shared block, then the layout of lds_bytes(CAP,
// own_cap) bytes), and no wave ever waits for another.
template <int B, int CAP>
__global__ __launch_bounds__(B == 64 ? 64 * kMaxEventsPerBlock : B) void k_persistent(sbt_params P, HitsArgs H,
                                                                                     Work W0, int own_cap,
                                                                                     int sortcap)
{
    uint32_t lo = 0;
    Shared<B> *sp;
    if constexpr (B == 64) {
        const uint32_t region = event_region_bytes<B>(CAP, own_cap);
        const uint32_t r0 = (uint32_t)uni((int)(threadIdx.x >> 6)) * region;
        sp = reinterpret_cast<Shared<B> *>(g_lds + r0);
        lo = r0 + shared_block_bytes<B>();
    } else {
        __shared__ Shared<B> S_wg;
        sp = &S_wg;
    }
    Shared<B> &S = *sp;
    for (;;) {
        // the workspace base is hidden from the optimiser per event, so the
        // pointers derived from it are not hoisted out of this loop
        Work W = W0;
        W.base = opq_global(W0.base);
        W.H = opq(W0.H);
        W.E = opq(W0.E);
        if (tid<B>() == 0) {
            const int idx = (int)atomicAdd(ws_counterp(W), 1u);
            S.e = idx < H.n_events ? ws_orderp(W)[idx] : -1;
        }
        ev_sync<B>();
        const int e = uni(S.e);
        if (e < 0) break;
        int hb, N;
        const int st = load_event<B>(P, H, e, S, &hb, &N);
        if (tid<B>() == 0) ws_evinfo(W)[e].st = st;
        if (st == 0) {
            const Ev v = event_view(W, e, hb, N, lo);
            stage_sort<B>(P, H, v, S, sortcap);
            const bool in_lds = stage_track<B, CAP>(P, v, S, own_cap, false);
            const int n_fin = uni(S.cnt[3]);
            if (CAP > 0 && in_lds) stage_filter<B>(P, v, n_fin, Lay<CAP>::own(v.lo));
            else stage_filter<B>(P, v, n_fin, v.own());
            stage_compact<B>(v, S.scan, (int)lds_sort_head() + 4 * sortcap);
        } else if (tid<B>() == 0) {
            ws_evinfo(W)[e].nt = 0;
            ws_evinfo(W)[e].nh = 0;
        }
        ev_sync<B>();
    }
}

#if SBT_TPE == 512
// The 512-lane kernel held to six waves per SIMD (at most 80 VGPRs), so that
// three workgroups with 448-hit slots (49.5 KB of LDS each) share a compute
// unit: more events in flight for long batches.  With defer, events whose
// busiest module or flag count does not fit the LDS form are not run from
// memory but listed for a second pass.  The body is otherwise k_persistent's
// for B = 512, written out again: routing both kernels through one inlined
// function changes the default kernel's generated code, which is kept as it
// was measured.
template <int CAP>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6))) void k_persistent_dense(
    sbt_params P, HitsArgs H, Work W0, int own_cap, int sortcap, int defer)
{
    constexpr int B = 512;
    constexpr uint32_t lo = 0;
    __shared__ Shared<B> S;
    for (;;) {
        // the workspace base is hidden from the optimiser per event, so the
        // pointers derived from it are not hoisted out of this loop
        Work W = W0;
        W.base = opq_global(W0.base);
        W.H = opq(W0.H);
        W.E = opq(W0.E);
        if (tid<B>() == 0) {
            const int idx = (int)atomicAdd(ws_counterp(W), 1u);
            S.e = idx < H.n_events ? ws_orderp(W)[idx] : -1;
        }
        ev_sync<B>();
        const int e = uni(S.e);
        if (e < 0) break;
        int hb, N;
        const int st = load_event<B>(P, H, e, S, &hb, &N);
        if (defer && st == 0 && !event_fits_lds<B, CAP>(S, N, own_cap)) {
            // with defer, an event that does not fit the LDS slots is set
            // aside for a second pass with larger slots
            if (tid<B>() == 0) ws_deferp(W)[atomicAdd(ws_defer_countp(W), 1u)] = e;
        } else {
            if (tid<B>() == 0) ws_evinfo(W)[e].st = st;
            if (st == 0) {
                const Ev v = event_view(W, e, hb, N, lo);
                stage_sort<B>(P, H, v, S, sortcap);
                const bool in_lds = stage_track<B, CAP>(P, v, S, own_cap, false);
                const int n_fin = uni(S.cnt[3]);
                if (CAP > 0 && in_lds) stage_filter<B>(P, v, n_fin, Lay<CAP>::own(v.lo));
                else stage_filter<B>(P, v, n_fin, v.own());
                stage_compact<B>(v, S.scan, (int)lds_sort_head() + 4 * sortcap);
            } else if (tid<B>() == 0) {
                ws_evinfo(W)[e].nt = 0;
                ws_evinfo(W)[e].nh = 0;
            }
        }
        ev_sync<B>();
    }
}

#endif

#define SBT_CAT2(a, b) a##b
#define SBT_CAT(a, b) SBT_CAT2(a, b)

namespace sbt {

const void *SBT_CAT(persistent_kernel_, SBT_TPE)(int cap)
{
    switch (cap) {
    case 0: return reinterpret_cast<const void *>(k_persistent<SBT_TPE, 0>);
    case 256: return reinterpret_cast<const void *>(k_persistent<SBT_TPE, 256>);
    case 448: return reinterpret_cast<const void *>(k_persistent<SBT_TPE, 448>);
    case 672: return reinterpret_cast<const void *>(k_persistent<SBT_TPE, 672>);
    case 768: return reinterpret_cast<const void *>(k_persistent<SBT_TPE, 768>);
    case 1024: return reinterpret_cast<const void *>(k_persistent<SBT_TPE, 1024>);
    case 1536: return reinterpret_cast<const void *>(k_persistent<SBT_TPE, 1536>);
    default: return nullptr;
    }
}

#if SBT_TPE == 512
const void *persistent_kernel_512_dense(int cap)
{
    return cap == 448 ? reinterpret_cast<const void *>(k_persistent_dense<448>) : nullptr;
}
#endif

}  // namespace sbt
