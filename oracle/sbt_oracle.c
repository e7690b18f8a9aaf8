/*
 * Search by triplet -- plain, single-threaded CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the HIP library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it; the product
 * path never does.  It shares no code, header or constant table with the HIP
 * library: every constant below is written out here.
 *
 * What is computed (paper, Section 3, "Sort by phi", "Track seeding and track
 * following", "Tracklet filter"), one event at a time:
 *
 *   1. phi of every hit as a 16-bit unsigned integer on the full circle
 *      (the simplified two-argument arctangent, mapped onto [0, 2^16) so that
 *      differences wrap modulo 2^16).
 *   2. hits of every module ordered by (phi16, hit id).
 *   3. seeding and following alternate over consecutive modules, the
 *      following stage flagging the hits it takes; seeding never uses a
 *      flagged hit.
 *   4. forming tracks that miss two consecutive modules, or reach the last
 *      module, become final: three hits make a tracklet, four or more a track.
 *   5. tracklets pass a least-squares straight-line fit threshold and must be
 *      made of unflagged hits.
 *   6. output: tracks and accepted tracklets ordered by the id of the middle
 *      hit of their seed, each as its hit ids in traversal order.
 *
 * Readings of points the paper leaves open (each also stated where used):
 *   - traversal: t = 0..M-1 visits module kmod(t) = reverse ? M-1-t : t.
 *   - every stage is a pure function of the state at its start (the paper's
 *     barrier between seeding and following); every choice is a minimum over
 *     a total order with unique keys, so the result does not depend on the
 *     order in which candidates are visited.
 *   - flags are owner keys: owner[h] is FREE or the key (seed middle-hit id)
 *     of the track that took h.  "Flagged" means owner != FREE.
 *   - thresholds are strict (<), phi windows inclusive (<=).
 *
 * Arithmetic: IEEE binary32, round to nearest even, operations in the
 * written order, no contraction into fused multiply-add (build with
 * -ffp-contract=off), correctly rounded division, no flush of denormals.
 *
 * Parity pins live in the test suite: phi16 against a float64 arctangent,
 * the sort against numpy.lexsort, the tracklet chi2 against a float64
 * least-squares fit, the search mechanics against exhaustive enumeration on
 * tiny events, and the physics indicators on generated straight tracks.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#include "sbt_oracle_abi.h"

#define ORC_OK 0
#define ORC_ERR_INVALID_ARG (-1)
#define ORC_ERR_NOMEM (-5)

#define ORC_FREE 0xFFFFFFFFu
#define ORC_MAX_MODULES 64

/* ---- phi16: simplified atan2 mapped onto 16 bits (Section 3, "Sort by phi") ----
 * atan(r) for r in [0,1] is r * P(r^2) with P of degree 4; the coefficients
 * were fitted in float64 (iteratively reweighted least squares towards the
 * minimax solution) and rounded to binary32.  Maximum error of the binary32
 * evaluation is 1.2e-5 rad, i.e. 0.12 phi16 units.  The angle is then
 * scaled by 32768/pi and rounded to nearest even, so -pi and +pi both map to
 * 0x8000 and the 16-bit value is a point on the circle. */
static const float ORC_C0 = 0x1.ffee7ap-1f;
static const float ORC_C1 = -0x1.523b6cp-2f;
static const float ORC_C2 = 0x1.70f766p-3f;
static const float ORC_C3 = -0x1.5ccd12p-4f;
static const float ORC_C4 = 0x1.55871cp-6f;
static const float ORC_HALF_PI = 0x1.921fb6p+0f;  /* binary32 nearest to pi/2 */
static const float ORC_PI = 0x1.921fb6p+1f;       /* binary32 nearest to pi */
static const float ORC_PHI_SCALE = 0x1.45f306p+13f; /* binary32 nearest to 32768/pi */

uint16_t sbt_oracle_phi16(float x, float y)
{
    float a = x < 0.0f ? -x : x;
    float b = y < 0.0f ? -y : y;
    if (a == 0.0f && b == 0.0f) return 0;
    float mn = a < b ? a : b;
    float mx = a < b ? b : a;
    float r = mn / mx;
    float s = r * r;
    float p = ORC_C4;
    p = p * s + ORC_C3;
    p = p * s + ORC_C2;
    p = p * s + ORC_C1;
    p = p * s + ORC_C0;
    float at = r * p;
    if (b > a) at = ORC_HALF_PI - at;
    if (x < 0.0f) at = ORC_PI - at;
    if (y < 0.0f) at = -at;
    int32_t q = (int32_t)rintf(at * ORC_PHI_SCALE);   /* nearest, ties to even */
    return (uint16_t)(q & 0xFFFF);
}

void sbt_oracle_phi16_array(int64_t n, const float *x, const float *y, uint16_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = sbt_oracle_phi16(x[i], y[i]);
}

/* signed modular difference of two phi16 values, in [-32768, 32767] */
static int orc_dphi(uint16_t a, uint16_t b)
{
    int d = (int)a - (int)b;
    d &= 0xFFFF;
    if (d >= 32768) d -= 65536;
    return d;
}

static int orc_in_window(uint16_t q, uint16_t centre, int w)
{
    int d = orc_dphi(q, centre);
    if (d < 0) d = -d;
    return d <= w;
}

/* exported for the window-membership pin */
int sbt_oracle_in_window(uint16_t q, uint16_t centre, int32_t w)
{
    return orc_in_window(q, centre, (int)w);
}

/* ---- per-module phi sort (Section 3, "Sort by phi") ----
 * Ties in phi16 are broken by the lower hit id. */
static const uint16_t *orc_sort_q;
static int orc_cmp_hits(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    if (orc_sort_q[a] != orc_sort_q[b]) return orc_sort_q[a] < orc_sort_q[b] ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* mo: M+1 event-local module offsets; out: hit ids, module by module, each
 * module ordered by (phi16, id). */
static void orc_sort_event(int M, const int32_t *mo, const uint16_t *q, int32_t *out)
{
    for (int k = 0; k < M; ++k) {
        for (int32_t i = mo[k]; i < mo[k + 1]; ++i) out[i] = i;
        orc_sort_q = q;
        qsort(out + mo[k], (size_t)(mo[k + 1] - mo[k]), sizeof(int32_t), orc_cmp_hits);
    }
}

void sbt_oracle_sort_event(int M, const int32_t *mo, const float *x, const float *y,
                           int32_t *sorted_ids)
{
    int32_t n = mo[M];
    uint16_t *q = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) q[i] = sbt_oracle_phi16(x[i], y[i]);
    orc_sort_event(M, mo, q, sorted_ids);
    free(q);
}

/* ---- pendulum search (Section 3, "Track seeding and track following") ----
 * Over a module's phi-sorted list of n hits: start at the first position whose
 * phi16 is >= the target (or position 0 if there is none), then alternate one
 * step down, one step up, two down, two up, ... with wrap-around, for at most
 * n visits, collecting unflagged hits until k of them are found.  Flagged hits
 * are skipped and not counted.  Returns the number collected; positions are
 * written in visit order. */
int sbt_oracle_pendulum(int32_t n, const uint16_t *q_sorted, const uint8_t *flagged,
                        uint16_t target, int32_t k, int32_t *out_pos)
{
    if (n <= 0) return 0;
    int32_t s0 = 0;
    while (s0 < n && q_sorted[s0] < target) ++s0;
    if (s0 == n) s0 = 0;
    int32_t got = 0;
    for (int32_t v = 0; v < n && got < k; ++v) {
        int32_t off = (v & 1) ? -((v + 1) / 2) : (v / 2);
        int32_t pos = (int32_t)(((int64_t)s0 + off) % n);
        if (pos < 0) pos += n;
        if (!flagged[pos]) out_pos[got++] = pos;
    }
    return got;
}

/* ---- tracklet fit (Section 3, "Tracklet filter") ----
 * Sum of squared residuals of separate least-squares lines x(z) and y(z)
 * through three hits.  With v = (z2-z1, z0-z2, z1-z0), v is orthogonal to
 * (1,1,1) and to z, so the residual of each fit is the projection on v:
 * chi2 = ((v.x)^2 + (v.y)^2) / (v.v). */
float sbt_oracle_tracklet_chi2(const float *x3, const float *y3, const float *z3)
{
    float v0 = z3[2] - z3[1];
    float v1 = z3[0] - z3[2];
    float v2 = z3[1] - z3[0];
    float sx = ((v0 * x3[0]) + (v1 * x3[1])) + (v2 * x3[2]);
    float sy = ((v0 * y3[0]) + (v1 * y3[1])) + (v2 * y3[2]);
    float n2 = ((v0 * v0) + (v1 * v1)) + (v2 * v2);
    return ((sx * sx) + (sy * sy)) / n2;
}

/* ---- parameters ---- */
typedef struct {
    int M;
    const float *module_z;
    int reverse;
    int K;           /* pendulum candidates per middle hit */
    int Ws, Wf;      /* inclusive phi16 half-windows */
    float Ss, Sf;    /* scatter thresholds (mm^2), strict */
    float X;         /* tracklet chi2 threshold (mm^2), strict */
    int misses;      /* consecutive modules a forming track may miss */
} orc_params;

typedef struct {
    int32_t hits[ORC_MAX_MODULES];  /* event-local hit ids, traversal order */
    int32_t n;
    int32_t last_t;
    uint32_t key;                   /* id of the seed's middle hit */
    int final;
    /* following-stage scratch */
    int has_best;
    int32_t best;
    float best_sc;
    int wins;
} orc_track;

typedef struct {
    int N, M;
    const int32_t *mo;       /* M+1 event-local module offsets */
    const float *x, *y, *z;  /* event-local */
    uint16_t *q;             /* phi16 per hit id */
    int32_t *sorted;         /* ids, per module phi-sorted */
    uint32_t *owner;         /* FREE or owner key, per hit id */
    uint64_t *claim;         /* per hit id */
    orc_track *trk;
    int32_t n_trk;
    uint8_t *flag_scratch;
    int32_t *pos_scratch;
} orc_event;

static int orc_kmod(const orc_params *p, int t) { return p->reverse ? p->M - 1 - t : t; }

static uint32_t orc_float_bits(float f)
{
    uint32_t u;
    memcpy(&u, &f, sizeof u);
    return u;
}

/* Seeding(t), t >= 2: modules A = kmod(t-2), B = kmod(t-1), C = kmod(t).
 * For every unflagged middle hit h1 in B: up to K unflagged doublet partners h0
 * in A by the pendulum search around phi16(h1); each doublet extrapolated
 * (from h1, the nearer hit) to C's nominal z; the unflagged hits h2 of C
 * inside the inclusive phi window around the extrapolated phi16 are scored by
 * the scatter dx^2 + dy^2 at h2's own z; the kept seed is the minimum of
 * (scatter, id0, id2) among those with scatter < Ss.  Writes no flags. */
static void orc_seeding(const orc_params *p, orc_event *ev, int t)
{
    int A = orc_kmod(p, t - 2), B = orc_kmod(p, t - 1), C = orc_kmod(p, t);
    float Zc = p->module_z[C];
    int32_t a0 = ev->mo[A], na = ev->mo[A + 1] - ev->mo[A];
    const int32_t *PA = ev->sorted + a0;
    if (na <= 0) return;
    /* the flag state of module A is fixed during this stage */
    uint16_t *qa = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)na);
    for (int32_t s = 0; s < na; ++s) {
        qa[s] = ev->q[PA[s]];
        ev->flag_scratch[s] = ev->owner[PA[s]] != ORC_FREE;
    }
    int32_t n_new = 0;
    orc_track *fresh = (orc_track *)malloc(sizeof(orc_track) * (size_t)(ev->mo[B + 1] - ev->mo[B] + 1));
    for (int32_t h1 = ev->mo[B]; h1 < ev->mo[B + 1]; ++h1) {
        if (ev->owner[h1] != ORC_FREE) continue;
        int32_t nc = sbt_oracle_pendulum(na, qa, ev->flag_scratch, ev->q[h1], p->K, ev->pos_scratch);
        int found = 0;
        float bsc = 0.0f;
        int32_t b0 = -1, b2 = -1;
        float x1 = ev->x[h1], y1 = ev->y[h1], z1 = ev->z[h1];
        for (int32_t c = 0; c < nc; ++c) {
            int32_t h0 = PA[ev->pos_scratch[c]];
            float x0 = ev->x[h0], y0 = ev->y[h0], z0 = ev->z[h0];
            float d01 = z1 - z0;
            float tx = (x1 - x0) / d01;
            float ty = (y1 - y0) / d01;
            float dzc = Zc - z1;
            uint16_t qe = sbt_oracle_phi16(x1 + tx * dzc, y1 + ty * dzc);
            for (int32_t h2 = ev->mo[C]; h2 < ev->mo[C + 1]; ++h2) {
                if (ev->owner[h2] != ORC_FREE) continue;
                if (!orc_in_window(ev->q[h2], qe, p->Ws)) continue;
                float dz = ev->z[h2] - z1;
                float dx = (x1 + tx * dz) - ev->x[h2];
                float dy = (y1 + ty * dz) - ev->y[h2];
                float sc = (dx * dx) + (dy * dy);
                if (!(sc < p->Ss)) continue;
                int better = !found || sc < bsc ||
                             (sc == bsc && (h0 < b0 || (h0 == b0 && h2 < b2)));
                if (better) { found = 1; bsc = sc; b0 = h0; b2 = h2; }
            }
        }
        if (found) {
            orc_track *f = &fresh[n_new++];
            memset(f, 0, sizeof *f);
            f->hits[0] = b0; f->hits[1] = h1; f->hits[2] = b2;
            f->n = 3;
            f->last_t = t;
            f->key = (uint32_t)h1;
        }
    }
    for (int32_t i = 0; i < n_new; ++i) ev->trk[ev->n_trk++] = fresh[i];
    free(fresh);
    free(qa);
}

/* Following(t), t >= 3, module C = kmod(t).
 * Eligible: not final, missed at most `misses` modules since its last hit, and
 * every hit either unflagged or flagged by this very track.  Search: the last
 * two hits (a, b) extrapolated from b to C's nominal z; the unflagged hits of C
 * inside the phi window scored by the scatter at their own z; best = minimum
 * (scatter, id) under Sf.  Claims: the claim set is {best}, plus the three
 * hits when the track is still a bare seed; key = (scatter bits << 32) | track
 * key; a track wins iff its key is the minimum claimed on every hit of its
 * claim set.  Winners append best and flag their claim set; everybody else
 * counts a miss.  Tracks that have now missed more than `misses` consecutive
 * modules become final. */
static void orc_following(const orc_params *p, orc_event *ev, int t)
{
    int C = orc_kmod(p, t);
    float Zc = p->module_z[C];
    /* search against the flag state at stage start */
    for (int32_t i = 0; i < ev->n_trk; ++i) {
        orc_track *f = &ev->trk[i];
        f->has_best = 0;
        f->wins = 0;
        if (f->final) continue;
        if (t - f->last_t > p->misses + 1) continue;
        int ok = 1;
        for (int32_t j = 0; j < f->n; ++j) {
            uint32_t o = ev->owner[f->hits[j]];
            if (o != ORC_FREE && o != f->key) ok = 0;
        }
        if (!ok) continue;
        int32_t ha = f->hits[f->n - 2], hb = f->hits[f->n - 1];
        float xa = ev->x[ha], ya = ev->y[ha], za = ev->z[ha];
        float xb = ev->x[hb], yb = ev->y[hb], zb = ev->z[hb];
        float dab = zb - za;
        float tx = (xb - xa) / dab;
        float ty = (yb - ya) / dab;
        float dzc = Zc - zb;
        uint16_t qe = sbt_oracle_phi16(xb + tx * dzc, yb + ty * dzc);
        for (int32_t h = ev->mo[C]; h < ev->mo[C + 1]; ++h) {
            if (ev->owner[h] != ORC_FREE) continue;
            if (!orc_in_window(ev->q[h], qe, p->Wf)) continue;
            float dz = ev->z[h] - zb;
            float dx = (xb + tx * dz) - ev->x[h];
            float dy = (yb + ty * dz) - ev->y[h];
            float sc = (dx * dx) + (dy * dy);
            if (!(sc < p->Sf)) continue;
            if (!f->has_best || sc < f->best_sc || (sc == f->best_sc && h < f->best)) {
                f->has_best = 1;
                f->best_sc = sc;
                f->best = h;
            }
        }
    }
    /* claims: minimum key per claimed hit */
    for (int32_t h = 0; h < ev->N; ++h) ev->claim[h] = UINT64_MAX;
    for (int32_t i = 0; i < ev->n_trk; ++i) {
        orc_track *f = &ev->trk[i];
        if (!f->has_best) continue;
        uint64_t kappa = ((uint64_t)orc_float_bits(f->best_sc) << 32) | f->key;
        if (kappa < ev->claim[f->best]) ev->claim[f->best] = kappa;
        if (f->n == 3)
            for (int j = 0; j < 3; ++j)
                if (kappa < ev->claim[f->hits[j]]) ev->claim[f->hits[j]] = kappa;
    }
    for (int32_t i = 0; i < ev->n_trk; ++i) {
        orc_track *f = &ev->trk[i];
        if (!f->has_best) continue;
        uint64_t kappa = ((uint64_t)orc_float_bits(f->best_sc) << 32) | f->key;
        int w = ev->claim[f->best] == kappa;
        if (f->n == 3)
            for (int j = 0; j < 3; ++j) w = w && ev->claim[f->hits[j]] == kappa;
        f->wins = w;
    }
    /* apply */
    for (int32_t i = 0; i < ev->n_trk; ++i) {
        orc_track *f = &ev->trk[i];
        if (!f->wins) continue;
        if (f->n == 3)
            for (int j = 0; j < 3; ++j) ev->owner[f->hits[j]] = f->key;
        ev->owner[f->best] = f->key;
        f->hits[f->n++] = f->best;
        f->last_t = t;
    }
    /* termination */
    for (int32_t i = 0; i < ev->n_trk; ++i) {
        orc_track *f = &ev->trk[i];
        if (!f->final && t - f->last_t >= p->misses + 1) f->final = 1;
    }
}

static int orc_cmp_u32(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Reconstruct one event.  Writes its accepted tracks, ordered by key, as
 * lengths (trk_len) and hit ids (hits_out); returns the number of tracks or a
 * negative error. */
static int32_t orc_event_run(const orc_params *p, int N, const int32_t *mo,
                             const float *x, const float *y, const float *z,
                             int32_t *trk_len, int32_t *hits_out, int32_t *n_hits_out)
{
    *n_hits_out = 0;
    if (N == 0) return 0;
    orc_event ev;
    memset(&ev, 0, sizeof ev);
    ev.N = N; ev.M = p->M; ev.mo = mo; ev.x = x; ev.y = y; ev.z = z;
    ev.q = (uint16_t *)calloc((size_t)N, sizeof(uint16_t));   /* every entry is written below */
    ev.sorted = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    ev.owner = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)N);
    ev.claim = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
    ev.trk = (orc_track *)malloc(sizeof(orc_track) * (size_t)N);
    ev.flag_scratch = (uint8_t *)malloc((size_t)N);
    ev.pos_scratch = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!ev.q || !ev.sorted || !ev.owner || !ev.claim || !ev.trk || !ev.flag_scratch || !ev.pos_scratch) {
        free(ev.q); free(ev.sorted); free(ev.owner); free(ev.claim); free(ev.trk);
        free(ev.flag_scratch); free(ev.pos_scratch);
        return ORC_ERR_NOMEM;
    }
    for (int32_t i = 0; i < N; ++i) ev.q[i] = sbt_oracle_phi16(x[i], y[i]);
    orc_sort_event(p->M, mo, ev.q, ev.sorted);
    for (int32_t i = 0; i < N; ++i) ev.owner[i] = ORC_FREE;

    orc_seeding(p, &ev, 2);
    for (int t = 3; t < p->M; ++t) {
        orc_following(p, &ev, t);
        orc_seeding(p, &ev, t);
    }
    for (int32_t i = 0; i < ev.n_trk; ++i) ev.trk[i].final = 1;

    /* tracklet filter: candidates, then claims among candidates */
    int32_t nt = ev.n_trk;
    float *chi2 = (float *)malloc(sizeof(float) * (size_t)(nt > 0 ? nt : 1));
    uint8_t *accept = (uint8_t *)malloc((size_t)(nt > 0 ? nt : 1));
    for (int32_t h = 0; h < N; ++h) ev.claim[h] = UINT64_MAX;
    for (int32_t i = 0; i < nt; ++i) {
        orc_track *f = &ev.trk[i];
        accept[i] = 0;
        if (f->n >= 4) { accept[i] = 1; continue; }
        float x3[3], y3[3], z3[3];
        for (int j = 0; j < 3; ++j) { x3[j] = x[f->hits[j]]; y3[j] = y[f->hits[j]]; z3[j] = z[f->hits[j]]; }
        chi2[i] = sbt_oracle_tracklet_chi2(x3, y3, z3);
        int cand = chi2[i] < p->X;
        for (int j = 0; j < 3; ++j) cand = cand && ev.owner[f->hits[j]] == ORC_FREE;
        accept[i] = cand ? 2 : 0;   /* 2: candidate, decided by claims below */
        if (cand) {
            uint64_t kappa = ((uint64_t)orc_float_bits(chi2[i]) << 32) | f->key;
            for (int j = 0; j < 3; ++j)
                if (kappa < ev.claim[f->hits[j]]) ev.claim[f->hits[j]] = kappa;
        }
    }
    for (int32_t i = 0; i < nt; ++i) {
        if (accept[i] != 2) continue;
        orc_track *f = &ev.trk[i];
        uint64_t kappa = ((uint64_t)orc_float_bits(chi2[i]) << 32) | f->key;
        int w = 1;
        for (int j = 0; j < 3; ++j) w = w && ev.claim[f->hits[j]] == kappa;
        accept[i] = (uint8_t)w;
    }

    /* output ordered by key (keys are unique) */
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * 2 * (size_t)(nt > 0 ? nt : 1));
    int32_t na = 0;
    for (int32_t i = 0; i < nt; ++i)
        if (accept[i]) { order[2 * na] = ev.trk[i].key; order[2 * na + 1] = (uint32_t)i; ++na; }
    qsort(order, (size_t)na, 2 * sizeof(uint32_t), orc_cmp_u32);
    int32_t w = 0;
    for (int32_t a = 0; a < na; ++a) {
        orc_track *f = &ev.trk[order[2 * a + 1]];
        trk_len[a] = f->n;
        for (int32_t j = 0; j < f->n; ++j) hits_out[w++] = f->hits[j];
    }
    *n_hits_out = w;

    free(order); free(accept); free(chi2);
    free(ev.q); free(ev.sorted); free(ev.owner); free(ev.claim); free(ev.trk);
    free(ev.flag_scratch); free(ev.pos_scratch);
    return na;
}

/* Full batch reconstruction.
 *   module_z[M], event_offsets[E+1], module_offsets[E*M+1] (absolute), x/y/z[H]
 *   max_event_hits > 0: the global event cut of the paper's sequence
 *   (Section 4): an event with more hits is not reconstructed (no tracks).
 *   outputs: event_track_offsets[E+1], track_hit_offsets[floor(H/3)+1],
 *            track_hits[H] (event-local ids, traversal order).
 * Returns 0 or a negative error. */
int sbt_oracle_reconstruct(int32_t n_modules, const float *module_z, int32_t reverse,
                           int32_t max_doublet_candidates,
                           int32_t phi_window_seeding, int32_t phi_window_forwarding,
                           float max_scatter_seeding, float max_scatter_forwarding,
                           float max_tracklet_chi2, int32_t max_consecutive_misses,
                           int32_t max_event_hits,
                           int32_t n_events, const int32_t *event_offsets,
                           const int32_t *module_offsets,
                           const float *x, const float *y, const float *z,
                           int32_t *event_track_offsets, int32_t *track_hit_offsets,
                           int32_t *track_hits)
{
    if (n_modules < 3 || n_modules > ORC_MAX_MODULES || !module_z || n_events < 0) return ORC_ERR_INVALID_ARG;
    if (max_doublet_candidates < 1 || max_consecutive_misses < 0 || max_event_hits < 0) return ORC_ERR_INVALID_ARG;
    if (phi_window_seeding < 0 || phi_window_seeding > 32767) return ORC_ERR_INVALID_ARG;
    if (phi_window_forwarding < 0 || phi_window_forwarding > 32767) return ORC_ERR_INVALID_ARG;
    orc_params p;
    p.M = n_modules; p.module_z = module_z; p.reverse = reverse ? 1 : 0;
    p.K = max_doublet_candidates; p.Ws = phi_window_seeding; p.Wf = phi_window_forwarding;
    p.Ss = max_scatter_seeding; p.Sf = max_scatter_forwarding; p.X = max_tracklet_chi2;
    p.misses = max_consecutive_misses;

    int32_t mo[ORC_MAX_MODULES + 1];
    int32_t n_tracks = 0, n_out_hits = 0;
    event_track_offsets[0] = 0;
    track_hit_offsets[0] = 0;
    for (int32_t e = 0; e < n_events; ++e) {
        int32_t base = event_offsets[e];
        int32_t N = event_offsets[e + 1] - base;
        if (max_event_hits > 0 && N > max_event_hits) {
            event_track_offsets[e + 1] = n_tracks;
            continue;
        }
        for (int k = 0; k <= n_modules; ++k) mo[k] = module_offsets[(int64_t)e * n_modules + k] - base;
        int32_t nh = 0;
        int32_t nt = orc_event_run(&p, N, mo, x + base, y + base, z + base,
                                   track_hit_offsets + n_tracks + 1, track_hits + n_out_hits, &nh);
        if (nt < 0) return nt;
        for (int32_t i = 0; i < nt; ++i)
            track_hit_offsets[n_tracks + 1 + i] += track_hit_offsets[n_tracks + i];
        n_tracks += nt;
        n_out_hits += nh;
        event_track_offsets[e + 1] = n_tracks;
    }
    return ORC_OK;
}

/* Batch entry with the structure layouts of sbt_oracle_abi.h: the per-event
 * status checks stated there, then the same per-event reconstruction as
 * sbt_oracle_reconstruct for every event that passes them. */
int sbt_reconstruct_cpu(const orc_abi_params *params, const orc_abi_hits *hits, orc_abi_tracks *tracks)
{
    if (!params || !hits || !tracks) return ORC_ERR_INVALID_ARG;
    const orc_abi_params *q = params;
    const int32_t M = q->n_modules, E = hits->n_events, H = hits->n_hits;
    if (M < 3 || M > ORC_MAX_MODULES || E < 0 || H < 0) return ORC_ERR_INVALID_ARG;
    if (q->max_doublet_candidates < 1 || q->max_consecutive_misses < 0 || q->max_event_hits < 0)
        return ORC_ERR_INVALID_ARG;
    if (q->phi_window_seeding < 0 || q->phi_window_seeding > 32767) return ORC_ERR_INVALID_ARG;
    if (q->phi_window_forwarding < 0 || q->phi_window_forwarding > 32767) return ORC_ERR_INVALID_ARG;
    if (!tracks->event_track_offsets || !tracks->track_hit_offsets || (H > 0 && !tracks->track_hits))
        return ORC_ERR_INVALID_ARG;
    if (E > 0 && (!hits->event_offsets || !hits->module_offsets)) return ORC_ERR_INVALID_ARG;
    if (H > 0 && (!hits->x || !hits->y || !hits->z)) return ORC_ERR_INVALID_ARG;
    orc_params p;
    p.M = M; p.module_z = q->module_z; p.reverse = q->reverse ? 1 : 0;
    p.K = q->max_doublet_candidates; p.Ws = q->phi_window_seeding; p.Wf = q->phi_window_forwarding;
    p.Ss = q->max_scatter_seeding; p.Sf = q->max_scatter_forwarding; p.X = q->max_tracklet_chi2;
    p.misses = q->max_consecutive_misses;

    const int32_t *eo = hits->event_offsets, *mog = hits->module_offsets;
    int32_t mo[ORC_MAX_MODULES + 1];
    int32_t n_tracks = 0, n_out_hits = 0;
    tracks->event_track_offsets[0] = 0;
    tracks->track_hit_offsets[0] = 0;
    for (int32_t e = 0; e < E; ++e) {
        const int32_t lo = eo[e], hi = eo[e + 1];
        int32_t st = 0;
        if (lo < 0 || hi > H || hi < lo) st = ORC_EV_BAD_OFFSETS;
        else if (hi - lo > 65535) st = ORC_EV_TOO_LARGE;
        else if (q->max_event_hits > 0 && hi - lo > q->max_event_hits) st = ORC_EV_CUT;
        else {
            const int64_t b = (int64_t)e * M;
            for (int32_t k = 0; k <= M; ++k) {
                const int32_t v = mog[b + k];
                if ((k == 0 && v != lo) || (k == M && v != hi) || v < lo || v > hi || (k > 0 && mog[b + k - 1] > v))
                    st = ORC_EV_BAD_OFFSETS;
            }
        }
        if (tracks->event_status) tracks->event_status[e] = st;
        if (st == 0) {
            for (int32_t k = 0; k <= M; ++k) mo[k] = mog[(int64_t)e * M + k] - lo;
            int32_t nh = 0;
            const int32_t nt = orc_event_run(&p, hi - lo, mo, hits->x + lo, hits->y + lo, hits->z + lo,
                                             tracks->track_hit_offsets + n_tracks + 1,
                                             tracks->track_hits + n_out_hits, &nh);
            if (nt < 0) return nt;
            for (int32_t i = 0; i < nt; ++i)
                tracks->track_hit_offsets[n_tracks + 1 + i] += tracks->track_hit_offsets[n_tracks + i];
            n_tracks += nt;
            n_out_hits += nh;
        }
        tracks->event_track_offsets[e + 1] = n_tracks;
    }
    return ORC_OK;
}
