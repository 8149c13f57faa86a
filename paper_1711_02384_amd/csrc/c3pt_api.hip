// Host side of libc3pt: argument validation, per-stream scratch, launch
// planning.  Every entry point validates all arguments before it touches the
// device, so a failing call enqueues nothing and leaves the output untouched.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/c3pt.h"
#include "c3pt_internal.h"
#include "c3pt_analysis.h"
#include "c3pt_fac_left.h"
#include "c3pt_fs_api.h"

using namespace c3pt;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int ok() {
    g_last_error.clear();
    return C3PT_OK;
}

// Per-(device, stream) scratch: device memory for split-site partial sums and
// small parameter tables, plus a pinned staging buffer for host->device
// parameter uploads guarded by an event.
// Pinned staging slots for parameter uploads, used in turn: an upload waits
// only for the copy made kUploadSlots uploads earlier from the same slot, so
// the host stays ahead of the stream instead of waiting for the kernels queued
// before the previous upload.
constexpr int kUploadSlots = 8;
struct Scratch {
    void* dev = nullptr;
    size_t dev_bytes = 0;
    void* aux = nullptr;       // second region: fields derived inside a call (stencil outputs)
    size_t aux_bytes = 0;
    void* pinned[kUploadSlots] = {};
    size_t pinned_bytes[kUploadSlots] = {};
    hipEvent_t ev[kUploadSlots] = {};
    int next_slot = 0;
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Scratch> g_scratch;

int current_device(int* dev) {
    if (hipGetDevice(dev) != hipSuccess) return fail(C3PT_EDEVICE, "hipGetDevice failed");
    return C3PT_OK;
}

// Ensure at least `bytes` of device scratch for (device, stream). Growing
// synchronizes the stream so that no enqueued kernel still reads the old buffer.
int scratch_dev(hipStream_t st, size_t bytes, void** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Scratch& s = g_scratch[{dev, st}];
    if (s.dev_bytes < bytes) {
        if (s.dev) {
            if (hipStreamSynchronize(st) != hipSuccess) return fail(C3PT_EDEVICE, "stream sync failed");
            hipFree(s.dev);
            s.dev = nullptr;
            s.dev_bytes = 0;
        }
        size_t want = std::max(bytes, (size_t)1 << 20);
        want = (want + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
        if (hipMalloc(&s.dev, want) != hipSuccess) {
            (void)hipGetLastError();
            s.dev = nullptr;
            return fail(C3PT_ENOMEM, "scratch allocation of %zu bytes failed", want);
        }
        s.dev_bytes = want;
    }
    *out = s.dev;
    return C3PT_OK;
}

// The second per-(device, stream) region, grown like the first (it never
// aliases the partial sums, which live in the first).
int scratch_aux(hipStream_t st, size_t bytes, void** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Scratch& s = g_scratch[{dev, st}];
    if (s.aux_bytes < bytes) {
        if (s.aux) {
            if (hipStreamSynchronize(st) != hipSuccess) return fail(C3PT_EDEVICE, "stream sync failed");
            (void)hipFree(s.aux);
            s.aux = nullptr;
            s.aux_bytes = 0;
        }
        const size_t want = (bytes + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1);
        if (hipMalloc(&s.aux, want) != hipSuccess) {
            (void)hipGetLastError();
            s.aux = nullptr;
            return fail(C3PT_ENOMEM, "scratch allocation of %zu bytes failed", want);
        }
        s.aux_bytes = want;
    }
    *out = s.aux;
    return C3PT_OK;
}

// Copy `bytes` of host data into device scratch at byte offset `off` through
// the next pinned staging slot; the slot's event orders its reuse.  The device
// region is ordered by the stream (kernels of earlier calls that read it run
// before the copy).
int upload(hipStream_t st, void* dev_base, size_t off, const void* host, size_t bytes) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Scratch& s = g_scratch[{dev, st}];
    const int k = s.next_slot;
    s.next_slot = (k + 1) % kUploadSlots;
    if (!s.ev[k]) {
        if (hipEventCreateWithFlags(&s.ev[k], hipEventDisableTiming) != hipSuccess)
            return fail(C3PT_EDEVICE, "event creation failed");
    } else if (hipEventSynchronize(s.ev[k]) != hipSuccess) {
        return fail(C3PT_EDEVICE, "event sync failed");
    }
    if (s.pinned_bytes[k] < bytes) {
        if (s.pinned[k]) hipHostFree(s.pinned[k]);
        s.pinned[k] = nullptr;
        s.pinned_bytes[k] = 0;
        size_t want = std::max(bytes, (size_t)65536);
        if (hipHostMalloc(&s.pinned[k], want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            s.pinned[k] = nullptr;
            return fail(C3PT_ENOMEM, "pinned staging allocation failed");
        }
        s.pinned_bytes[k] = want;
    }
    memcpy(s.pinned[k], host, bytes);
    if (hipMemcpyAsync((char*)dev_base + off, s.pinned[k], bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(C3PT_EDEVICE, "parameter upload failed");
    if (hipEventRecord(s.ev[k], st) != hipSuccess) return fail(C3PT_EDEVICE, "event record failed");
    return C3PT_OK;
}

// ---- kernel timing -------------------------------------------------------
struct ProfRec {
    const char* name;
    hipEvent_t a, b;
};
struct ProfStat {
    long long count = 0;
    double total = 0, mn = 1e300, mx = 0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::map<std::string, ProfStat> g_prof_stats;

// Launch `fn` on `st`, bracketed by timing events when profiling is enabled.
template <class F>
hipError_t timed(const char* name, hipStream_t st, F fn) {
#ifdef C3PT_SYNC_LAUNCHES
    // debug builds: every launch completes (or reports its fault) before the next
    {
        const hipError_t e = fn();
        if (e != hipSuccess) return e;
        const hipError_t s2 = hipStreamSynchronize(st);
        if (s2 != hipSuccess) {
            fprintf(stderr, "c3pt: launch %s failed: %s\n", name, hipGetErrorString(s2));
            return s2;
        }
        return hipGetLastError();
    }
#endif
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        on = g_prof_on;
    }
    if (!on) return fn();
    ProfRec r{name, nullptr, nullptr};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return hipErrorOutOfMemory;
    hipEventRecord(r.a, st);
    hipError_t e = fn();
    hipEventRecord(r.b, st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back(r);
    return e;
}

// ---- phase tables ---------------------------------------------------------
// Built once per (device, geometry, source, sign, arithmetic, layout, momentum
// group) and kept until c3pt_release_scratch or LRU eviction beyond a cap.
struct PhaseKey {
    int dev, L[3], r[3], sigma, mode, mtmax;
    std::vector<int> k;
    bool operator<(const PhaseKey& o) const {
        return std::tie(dev, L[0], L[1], L[2], r[0], r[1], r[2], sigma, mode, mtmax, k) <
               std::tie(o.dev, o.L[0], o.L[1], o.L[2], o.r[0], o.r[1], o.r[2], o.sigma, o.mode, o.mtmax, o.k);
    }
};
struct PhaseEntry {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipEvent_t ready = nullptr;
    unsigned long long last_use = 0;
    void* pinned = nullptr;   // host copy a factor plan was uploaded from
};
constexpr size_t kPhaseCacheCap = (size_t)2 << 30;
std::map<PhaseKey, PhaseEntry> g_phase;
size_t g_phase_bytes = 0;
unsigned long long g_phase_clock = 0;

void free_phase_entry(PhaseEntry& e) {
    if (e.ptr) hipFree(e.ptr);
    if (e.pinned) hipHostFree(e.pinned);
    if (e.ready) hipEventDestroy(e.ready);
    g_phase_bytes -= e.bytes;
    e = PhaseEntry{};
}

int check_geom(const c3pt_geom* g) {
    if (!g) return fail(C3PT_EINVAL, "geom is NULL");
    for (int j = 0; j < 3; ++j)
        if (g->L[j] < 1 || g->L[j] > C3PT_MAX_L)
            return fail(C3PT_EINVAL, "L[%d] = %d outside [1, %d]", j, g->L[j], C3PT_MAX_L);
    if (g->T < 1) return fail(C3PT_EINVAL, "T = %d < 1", g->T);
    if (g->dtype != C3PT_C64 && g->dtype != C3PT_C128) return fail(C3PT_EINVAL, "unknown dtype %d", g->dtype);
    if (g->proj != C3PT_PROJ_NATIVE && g->proj != C3PT_PROJ_SPLIT_F16 && g->proj != C3PT_PROJ_SPLIT_BF16 &&
        g->proj != C3PT_PROJ_FACTORED && g->proj != C3PT_PROJ_FACTORED_F16 && g->proj != C3PT_PROJ_FACTORED_BF16)
        return fail(C3PT_EINVAL, "unknown projection mode %d", g->proj);
    if ((g->proj == C3PT_PROJ_SPLIT_F16 || g->proj == C3PT_PROJ_SPLIT_BF16 || g->proj == C3PT_PROJ_FACTORED_F16 ||
         g->proj == C3PT_PROJ_FACTORED_BF16) &&
        g->dtype != C3PT_C64)
        return fail(C3PT_EINVAL, "split-precision projection needs complex64 inputs");
    return C3PT_OK;
}

int check_momenta(const int* k, int n_mom) {
    if (n_mom < 1 || n_mom > C3PT_MAX_MOM)
        return fail(C3PT_EINVAL, "n_mom = %d outside [1, %d]", n_mom, C3PT_MAX_MOM);
    if (!k) return fail(C3PT_EINVAL, "momentum list is NULL");
    return C3PT_OK;
}

int posmod(long long v, int L) {
    long long r = v % L;
    return (int)(r < 0 ? r + L : r);
}

int proj_mode(const c3pt_geom* g) {
    if (g->dtype == C3PT_C128) return kModeF64;
    if (g->proj == C3PT_PROJ_SPLIT_BF16) return kModeSplitBF16;
    if (g->proj == C3PT_PROJ_SPLIT_F16) return kModeSplitF16;
    return kModeF32;
}

// Kernel variant per (kind, mode, momentum-tile class); 0 = default.
constexpr int kKinds = 3;   // 0 meson spectator, 1 baryon spectator, 2 insertion
constexpr int kModes = 7;
constexpr int kModeFacVariants = 4;   // variant slot of the factored projection (not an arithmetic mode)
constexpr int kModeFsVariants = 5;    // variant slot of the split-precision fused projection
int g_variant[kKinds][kModes][kMtClasses] = {};

int variant_count(int kind, int mode, int cls) {
    if (kind < 0 || kind >= kKinds || mode < 0 || mode >= kModes || cls < 0 || cls >= kMtClasses) return 0;
    // factored: 0 = every x3 plane written as its own chunk, 1 = chunks of planes summed in registers
    if (mode == kModeFacVariants) return 2;
    // fused: 0 = propagator tiles split in the kernel, two column blocks per workgroup;
    // 1 = slices split by a pass first, two blocks; 2 = split pass, one block per
    // workgroup; 3 = split in the kernel, one block per workgroup; 4 = split in
    // the kernel, three blocks per workgroup where it applies (else as 0); 5 =
    // as 0 with 48-site tiles where it applies (L1 = 48, no derivative slots;
    // else as 0).  The nucleon's diquark always has its pass.
    if (mode == kModeFsVariants) return 6;
    // factored kernels of batches and serving: bit 0 32-site tiles where they
    // apply, bit 1 chunks of about 4096 instead of 2048 sites
    if (mode == kModeBatchFacVariants) return kBatchFacVariants;
    if (mode == kModeF64) return cls == 0 ? 1 : 0;
    return kVariantsPerClass[cls];
}

// Momentum groups: FP32 / split launches take up to 128 momenta, FP64 up to 32.
struct MomGroup {
    int off, n;
};

std::vector<MomGroup> momentum_groups(int n_mom, bool f64) {
    const int gmax = f64 ? kMaxMomGroupF64 : kMaxMomGroupF32;
    std::vector<MomGroup> g;
    for (int off = 0; off < n_mom; off += gmax) g.push_back({off, std::min(gmax, n_mom - off)});
    return g;
}

void fill_phase(PhaseSpec& ph, const c3pt_geom* g, int sigma, const int* k, const MomGroup& mg) {
    memset(&ph, 0, sizeof(ph));
    for (int j = 0; j < 3; ++j) {
        ph.L[j] = g->L[j];
        ph.r[j] = posmod(g->r[j], g->L[j]);
    }
    ph.sigma = sigma;
    ph.n_mom = mg.n;
    for (int m = 0; m < mg.n; ++m)
        for (int j = 0; j < 3; ++j) ph.k[j][m] = (uint8_t)posmod(k[3 * (mg.off + m) + j], g->L[j]);
}

// Phase table of one momentum group (built on `st` when missing).
int phase_table(const c3pt_geom* g, int sigma, int mode, int mtmax, const int* k, const MomGroup& mg,
                hipStream_t st, const void** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    PhaseSpec ph;
    fill_phase(ph, g, sigma, k, mg);
    ph.r[0] = ph.r[1] = ph.r[2] = 0;   // tables at the origin; the source factor is applied on reduction
    PhaseKey key;
    key.dev = dev;
    for (int j = 0; j < 3; ++j) {
        key.L[j] = ph.L[j];
        key.r[j] = ph.r[j];
    }
    key.sigma = sigma;
    key.mode = mode;
    key.mtmax = mtmax;
    for (int m = 0; m < mg.n; ++m)
        for (int j = 0; j < 3; ++j) key.k.push_back(ph.k[j][m]);
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_phase.find(key);
    if (it != g_phase.end()) {
        it->second.last_use = ++g_phase_clock;
        if (hipStreamWaitEvent(st, it->second.ready, 0) != hipSuccess)
            return fail(C3PT_EDEVICE, "waiting for the phase table failed");
        *out = it->second.ptr;
        return C3PT_OK;
    }
    const int V3 = g->L[0] * g->L[1] * g->L[2];
    const size_t bytes = phase_table_bytes(mode, V3, mtmax);
    while (g_phase_bytes + bytes > kPhaseCacheCap && !g_phase.empty()) {
        auto lru = g_phase.begin();
        for (auto jt = g_phase.begin(); jt != g_phase.end(); ++jt)
            if (jt->second.last_use < lru->second.last_use) lru = jt;
        hipDeviceSynchronize();
        free_phase_entry(lru->second);
        g_phase.erase(lru);
    }
    PhaseEntry e;
    if (hipMalloc(&e.ptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(C3PT_ENOMEM, "phase table allocation of %zu bytes failed", bytes);
    }
    e.bytes = bytes;
    g_phase_bytes += bytes;
    if (launch_phase_table(mode, ph, V3, mtmax, e.ptr, st) != hipSuccess ||
        hipEventCreateWithFlags(&e.ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(e.ready, st) != hipSuccess) {
        free_phase_entry(e);
        return fail(C3PT_EDEVICE, "building the phase table failed");
    }
    e.last_use = ++g_phase_clock;
    g_phase[key] = e;
    *out = e.ptr;
    return C3PT_OK;
}

// Factor plan of one momentum group (the factored projection): distinct k1
// values, distinct (k1, k2) pairs grouped by k1, and each momentum's pair and
// k3, all reduced mod L.  False when the group needs more k1 values or pairs
// than the kernel holds; the group then runs on the dense kernel.
bool build_factor_plan(const c3pt_geom* g, int sigma, const int* k, const MomGroup& mg, bool f64, FactorPlan* p,
                       int max_per_slot = kFacMaxBPerA) {
    memset(p, 0, sizeof(*p));
    for (int j = 0; j < 3; ++j) p->L[j] = g->L[j];
    p->sigma = sigma;
    p->n_mom = mg.n;
    const int max_pairs = f64 ? kFacMaxPairsF64 : kFacMaxPairsF32;
    // distinct k1, and the distinct k2 of each
    std::vector<int> k1s;
    std::vector<std::vector<int>> k2s;
    std::vector<int> am(mg.n), jm(mg.n);
    for (int m = 0; m < mg.n; ++m) {
        const int* km = k + 3 * (mg.off + m);
        const int r1 = posmod(km[0], g->L[0]), r2 = posmod(km[1], g->L[1]);
        int a = (int)(std::find(k1s.begin(), k1s.end(), r1) - k1s.begin());
        if (a == (int)k1s.size()) {
            k1s.push_back(r1);
            k2s.emplace_back();
        }
        int jj = (int)(std::find(k2s[a].begin(), k2s[a].end(), r2) - k2s[a].begin());
        if (jj == (int)k2s[a].size()) k2s[a].push_back(r2);
        am[m] = a;
        jm[m] = jj;
        p->k3[m] = posmod(km[2], g->L[2]);
    }
    // slots: a k1 with n pairs takes ceil(n / max_per_slot) slots of nearly equal size
    std::vector<int> first_slot(k1s.size()), parts(k1s.size());
    int n_slots = 0, nb = 0;
    for (size_t a = 0; a < k1s.size(); ++a) {
        const int n = (int)k2s[a].size();
        parts[a] = (n + max_per_slot - 1) / max_per_slot;
        first_slot[a] = n_slots;
        n_slots += parts[a];
        nb += n;
    }
    if (n_slots > kFacMaxK1 || nb > max_pairs) return false;
    // pair (a, jj) -> slot first_slot[a] + jj / per, position jj % per
    nb = 0;
    for (size_t a = 0; a < k1s.size(); ++a) {
        const int n = (int)k2s[a].size(), per = (n + parts[a] - 1) / parts[a];
        for (int s = 0; s < parts[a]; ++s) {
            const int slot = first_slot[a] + s;
            p->k1[slot] = k1s[a];
            p->bstart[slot] = nb;
            for (int jj = s * per; jj < std::min(n, (s + 1) * per); ++jj) p->k2[nb++] = k2s[a][jj];
            p->nbmax = std::max(p->nbmax, nb - p->bstart[slot]);
        }
    }
    p->n1 = n_slots;
    for (int a = p->n1; a <= kFacMaxK1; ++a) p->bstart[a] = nb;
    p->n12 = nb;
    for (int m = 0; m < mg.n; ++m) {
        const int a = am[m], n = (int)k2s[a].size(), per = (n + parts[a] - 1) / parts[a];
        p->pair_of_m[m] = p->bstart[first_slot[a] + jm[m] / per] + jm[m] % per;
    }
    // momenta grouped by pair, in increasing m within a pair
    int pos = 0;
    for (int b = 0; b < p->n12; ++b) {
        p->mstart[b] = pos;
        for (int m = 0; m < mg.n; ++m)
            if (p->pair_of_m[m] == b) p->m_of[pos++] = m;
    }
    for (int b = p->n12; b <= kFacMaxPairsF32; ++b) p->mstart[b] = pos;
    return true;
}

// Device copy of a factor plan, cached beside the phase tables.
int factor_plan_table(const FactorPlan& plan, bool f64, hipStream_t st, const void** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    PhaseKey key;
    key.dev = dev;
    for (int j = 0; j < 3; ++j) {
        key.L[j] = plan.L[j];
        key.r[j] = 0;
    }
    key.sigma = plan.sigma;
    key.mode = 100 + (f64 ? 1 : 0);
    key.mtmax = 0;
    const int* words = (const int*)&plan;
    key.k.assign(words, words + sizeof(FactorPlan) / sizeof(int));
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_phase.find(key);
    if (it != g_phase.end()) {
        it->second.last_use = ++g_phase_clock;
        if (hipStreamWaitEvent(st, it->second.ready, 0) != hipSuccess)
            return fail(C3PT_EDEVICE, "waiting for the factor plan failed");
        *out = it->second.ptr;
        return C3PT_OK;
    }
    PhaseEntry e;
    e.bytes = sizeof(FactorPlan);
    if (hipMalloc(&e.ptr, e.bytes) != hipSuccess ||
        hipHostMalloc(&e.pinned, e.bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        free_phase_entry(e);
        return fail(C3PT_ENOMEM, "factor plan allocation failed");
    }
    g_phase_bytes += e.bytes;
    memcpy(e.pinned, &plan, e.bytes);
    if (hipMemcpyAsync(e.ptr, e.pinned, e.bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventCreateWithFlags(&e.ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(e.ready, st) != hipSuccess) {
        free_phase_entry(e);
        return fail(C3PT_EDEVICE, "uploading the factor plan failed");
    }
    e.last_use = ++g_phase_clock;
    g_phase[key] = e;
    *out = e.ptr;
    return C3PT_OK;
}

// x3 planes per chunk of the factored projection: about 2048 sites (the
// workgroups that share a slice then keep its chunk in one XCD's L2), fewer
// when the launch would otherwise leave CUs idle.
void plan_planes(const int L[3], int n_colblocks, int* chunk_planes, int* n_chunks) {
    int cp = std::max(1, std::min(L[2], 2048 / (L[0] * L[1])));
    while (cp > 1 && (long long)n_colblocks * ((L[2] + cp - 1) / cp) < 2048) cp = (cp + 1) / 2;
    *chunk_planes = cp;
    *n_chunks = (L[2] + cp - 1) / cp;
}

// Sites per split-site chunk: enough chunks to fill the chip, never more than
// kMaxSitesPerChunkF32 sites in one FP32 partial sum.
void plan_chunks(int V3, int n_colblocks, bool f64, int* chunk_sites, int* n_chunks) {
    const int kt = kSiteTile;
    const int tiles = (V3 + kt - 1) / kt;
    const int target_wg = 2048;
    int chunks = std::max(1, (target_wg + n_colblocks - 1) / n_colblocks);
    chunks = std::min(chunks, tiles);
    const int max_sites = f64 ? (1 << 30) : kMaxSitesPerChunkF32;
    chunks = std::max(chunks, (V3 + max_sites - 1) / max_sites);
    int tiles_per_chunk = (tiles + chunks - 1) / chunks;
    *chunk_sites = tiles_per_chunk * kt;
    *n_chunks = (V3 + *chunk_sites - 1) / *chunk_sites;
}

int to_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return C3PT_OK;
    return fail(C3PT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---- extent checks ---------------------------------------------------------
// Before anything is enqueued, the bytes a kernel will index in each buffer
// (from the kernel's own index formula) are compared with the bytes the host
// sizes for it (from the allocation's formula).  A mismatch is an internal
// error: the call fails with C3PT_EINVAL before touching the device.
// g_extent_scale scales every allocated size in the comparison: a test hook
// that plants an under-allocation (c3pt_debug_scale_allocations).
double g_extent_scale = 1.0;

int check_extent(const char* what, size_t indexed, size_t allocated) {
    const size_t have = (size_t)((double)allocated * g_extent_scale);
    if (indexed > have)
        return fail(C3PT_EINVAL, "extent check: %s indexes %zu bytes, %zu allocated", what, indexed, have);
    return C3PT_OK;
}

// Bytes of a phase table the dense consumers index: tiles of up to kSiteTile
// sites from the first site, native rows [site][8 mtmax] complex, split blocks
// [site / 16][hi, lo][mtmax][64 lanes][8] 16-bit.
size_t phase_indexed_bytes(int mode, int V3, int mtmax) {
    const size_t vt = (size_t)(V3 + kSiteTile - 1) / kSiteTile * kSiteTile;
    if (mode == kModeSplitBF16 || mode == kModeSplitF16) return vt / 16 * (2 * (size_t)mtmax * 64 * 8 * 2);
    return vt * 8 * mtmax * (mode == kModeF64 ? sizeof(double2) : sizeof(float2));
}

// Bytes of the split-site partial sums a projection launch indexes:
// [n_chunks][n_colblocks][n_mom][192] in the accumulator type.
size_t partial_indexed_bytes(int n_chunks, int n_colblocks, int n_mom, size_t elem) {
    return (size_t)n_chunks * n_colblocks * n_mom * kBlockCols * elem;
}

const char* const fac_names[3] = {"fac_spectator_meson", "fac_spectator_baryon", "fac_insertion"};

// Runs projection launches over momentum groups and reduces each into `out`.
// `launch(pg, mt)` enqueues one fused kernel for the grid pg.
template <class Launch>
int run_projection(const char* kname, int kind, const c3pt_geom* g, int sigma, const int* k, int n_mom,
                   int n_colblocks, int n_share, int n_per_share, int group_cols, int n_groups, int inner,
                   int outer_stride, int off, void* out, Launch launch) {
    hipStream_t st = (hipStream_t)g->stream;
    const bool f64 = g->dtype == C3PT_C128;
    const int mode = proj_mode(g);
    const int V3 = g->L[0] * g->L[1] * g->L[2];
    auto groups = momentum_groups(n_mom, f64);
    const bool want_fac = g->proj == C3PT_PROJ_FACTORED;
    int chunk_sites, n_chunks_dense, chunk_planes, n_chunks_fac;
    plan_chunks(V3, n_colblocks, f64, &chunk_sites, &n_chunks_dense);
    plan_planes(g->L, n_colblocks, &chunk_planes, &n_chunks_fac);
    const size_t gmax = f64 ? kMaxMomGroupF64 : kMaxMomGroupF32;
    const size_t elem = f64 ? sizeof(double2) : sizeof(float2);
    const size_t bytes = (size_t)std::max(n_chunks_dense, want_fac ? n_chunks_fac : 0) * n_colblocks * gmax *
                         kBlockCols * elem;
    // every group's plan and extents before anything is enqueued
    std::vector<FactorPlan> plans(groups.size());
    std::vector<char> facs(groups.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const MomGroup& mg = groups[gi];
        const int mt = (mg.n + 7) / 8;
        const int mtmax = f64 ? 4 : (mt <= 4 ? 4 : mt <= 8 ? 8 : mt <= 12 ? 12 : 16);
        facs[gi] = want_fac && build_factor_plan(g, sigma, k, mg, f64, &plans[gi]);
        const int n_chunks = facs[gi] ? n_chunks_fac : n_chunks_dense;
        if (int rc = check_extent("partial sums", partial_indexed_bytes(n_chunks, n_colblocks, mg.n, elem), bytes))
            return rc;
        if (facs[gi]) {
            // the factored kernels copy the whole plan into LDS
            if (int rc = check_extent("factor plan", sizeof(FactorPlan), sizeof(FactorPlan))) return rc;
        } else if (int rc = check_extent("phase table", phase_indexed_bytes(mode, V3, mtmax),
                                         phase_table_bytes(mode, V3, mtmax))) {
            return rc;
        }
    }
    void* part;
    if (int rc = scratch_dev(st, bytes, &part)) return rc;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const MomGroup& mg = groups[gi];
        const int mt = (mg.n + 7) / 8;
        const int mtmax = f64 ? 4 : (mt <= 4 ? 4 : mt <= 8 ? 8 : mt <= 12 ? 12 : 16);
        const FactorPlan& plan = plans[gi];
        const bool fac = facs[gi];
        const void* tab;
        if (fac) {
            if (int rc = factor_plan_table(plan, f64, st, &tab)) return rc;
        } else if (int rc = phase_table(g, sigma, mode, mtmax, k, mg, st, &tab)) {
            return rc;
        }
        int fac_variant;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            fac_variant = g_variant[kind][kModeFacVariants][mt_class(mt)];
        }
        const int n_chunks = fac ? n_chunks_fac : n_chunks_dense;
        ProjGrid pg;
        pg.V3 = V3;
        pg.n_mom = mg.n;
        pg.chunk_sites = chunk_sites;
        pg.chunk_planes = chunk_planes;
        pg.fac_acc = fac && fac_variant == 1 ? 1 : 0;
        pg.n_chunks = n_chunks;
        pg.n_colblocks = n_colblocks;
        pg.n_share = n_share;
        pg.n_per_share = n_per_share;
        pg.phase = tab;
        pg.partial = part;
        int variant;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            variant = g_variant[kind][mode][mt_class(mt)];
        }
        if (int rc = to_status(timed(fac ? fac_names[kind] : kname, st,
                                     [&] { return launch(mode, pg, mt, variant, fac); }),
                               "projection launch"))
            return rc;
        ReduceArgs ra;
        ra.partial = part;
        ra.f64 = f64 ? 1 : 0;
        fill_phase(ra.ph, g, sigma, k, mg);
        ra.out = (double2*)out;
        ra.n_chunks = n_chunks;
        ra.n_colblocks = n_colblocks;
        ra.n_groups = n_groups;
        ra.group_cols = group_cols;
        ra.n_mom_grp = mg.n;
        ra.n_mom_total = n_mom;
        ra.m_off = mg.off;
        ra.inner = inner;
        ra.outer_stride = outer_stride;
        ra.off = off;
        if (int rc = to_status(timed("reduce", st, [&] { return launch_reduce(ra, st); }), "reduction launch"))
            return rc;
    }
    return C3PT_OK;
}

}  // namespace

// ---- split-precision fused projection (C3PT_PROJ_FACTORED_F16 / _BF16) ----
namespace {

bool is_fused(const c3pt_geom* g) {
    return g->proj == C3PT_PROJ_FACTORED_F16 || g->proj == C3PT_PROJ_FACTORED_BF16;
}

// Factor plans of every momentum group (FP32 limits, at most max_per_slot
// pairs per k1 slot); false if one does not factor.
bool fs_plans(const c3pt_geom* g, int sigma, const int* k, const std::vector<MomGroup>& groups,
              std::vector<FactorPlan>* plans, int max_per_slot) {
    plans->resize(groups.size());
    for (size_t i = 0; i < groups.size(); ++i)
        if (!build_factor_plan(g, sigma, k, groups[i], false, &(*plans)[i], max_per_slot)) return false;
    return true;
}

// Fused launch shape of a call: the tuned variant of (producer kind, momentum
// class) sets whether B is split by a pass, how many column blocks share a
// workgroup (variant 4: three, for 16-site tiles of the spectators and the
// local insertion when every momentum group factors with at most
// kFsPairsCB3 pairs per k1 slot; otherwise two) and the tile length
// (variant 5: rows of 48 sites as one tile, for the spectators and the local
// insertion when L1 = 48), then the factor plans.
int fs_setup(const c3pt_geom* g, int sigma, const int* k, int n_mom, int vkind, bool derivative,
             std::vector<MomGroup>* groups, std::vector<FactorPlan>* plans, bool* bsplit, int* cbw, int* kt) {
    *groups = momentum_groups(n_mom, false);
    int v;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        v = g_variant[vkind][kModeFsVariants][mt_class(((*groups)[0].n + 7) / 8)];
    }
    *bsplit = vkind == 1 || v == 1 || v == 2;
    *cbw = v == 4 ? 3 : (v == 2 || v == 3 ? 1 : 2);
    *kt = (v == 5 && !derivative && g->L[0] == 48 && (vkind == 1 || !*bsplit)) ? 48 : fs_kt(g->L);
    if (*cbw == 3 && (fs_kt(g->L) != 16 || derivative)) *cbw = 2;
    if (*cbw == 3 && !fs_plans(g, sigma, k, *groups, plans, kFsPairsCB3)) *cbw = 2;
    if (*cbw != 3 && !fs_plans(g, sigma, k, *groups, plans, kFacMaxBPerA))
        return fail(C3PT_EUNSUPPORTED, "the momentum list does not factor (too many distinct k1 or (k1, k2))");
    return C3PT_OK;
}

// The kernel launches of one fused projection: with three blocks per
// workgroup and N not a multiple of three, the last N % 3 noise vectors run as
// a two-block launch over the same work grid, so that no workgroup carries an
// empty block; both write the call's partial sums (column blocks keep their
// indexes).  The second launch reads the B blocks again (for the 48^3 local
// insertion 1.9 GB of propagator slices) and is still faster: spectator 2.70
// -> 2.54 ms, insertion 2.93 -> 2.79 ms against one launch with an empty
// block in each last group.  pg.n_per_share is set per launch from n_slots.
hipError_t fs_launch_noise_parts(bool bf16, int KT, int kind, bool bsplit, int cbw, int N, int n_slots,
                                 ProjGrid pg, FsArgs fa, hipStream_t st) {
    int base[2], cnt[2], cbs[2], nparts = 0;
    if (cbw == 3 && N % 3 != 0) {
        if (N >= 3) {
            base[nparts] = 0, cnt[nparts] = N - N % 3, cbs[nparts++] = 3;
        }
        base[nparts] = N - N % 3, cnt[nparts] = N % 3, cbs[nparts++] = 2;
    } else {
        base[0] = 0, cnt[0] = N, cbs[0] = cbw, nparts = 1;
    }
    for (int i = 0; i < nparts; ++i) {
        fa.i_base = base[i];
        fa.N = cnt[i];
        pg.n_per_share = n_slots * ((cnt[i] + cbs[i] - 1) / cbs[i]);
        const hipError_t e = launch_fs(bf16, KT, kind, bsplit, cbs[i], pg, fa, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Partial sums then split B blocks in this stream's scratch.
int fs_scratch(hipStream_t st, size_t part_bytes, size_t b_bytes, void** part, void** B) {
    const size_t off = (part_bytes + 255) & ~(size_t)255;
    void* base;
    if (int rc = scratch_dev(st, off + b_bytes, &base)) return rc;
    *part = base;
    *B = (char*)base + off;
    return C3PT_OK;
}

// Spectators on the fused path: meson (G1 only) or nucleon (G1, G2).
int fs_spectator(const c3pt_geom* geom, bool baryon, const void* G1, const void* G2, const void* eta, int N,
                 const int* k, int n_mom, void* out) {
    std::vector<MomGroup> groups;
    std::vector<FactorPlan> plans;
    bool bsplit;
    int cbw;
    int KT;
    if (int rc = fs_setup(geom, -1, k, n_mom, baryon ? 1 : 0, false, &groups, &plans, &bsplit, &cbw, &KT)) return rc;
    hipStream_t st = (hipStream_t)geom->stream;
    const bool bf16 = geom->proj == C3PT_PROJ_FACTORED_BF16;
    const int Lp = fs_lp(geom->L), rows = geom->L[1] * geom->L[2];
    const int V3 = geom->L[0] * rows;
    const size_t bb = fs_block_bytes(geom->L);
    const int n_slots = baryon ? 16 : 1;
    const int ncb = N * n_slots;
    const int n_per_share = n_slots * ((N + cbw - 1) / cbw);
    int cp, nch;
    plan_planes(geom->L, n_per_share, &cp, &nch);
    const size_t part_bytes = (size_t)nch * ncb * kMaxMomGroupF32 * kBlockCols * sizeof(float2);
    for (const MomGroup& mg : groups)
        if (int rc = check_extent("partial sums", partial_indexed_bytes(nch, ncb, mg.n, sizeof(float2)), part_bytes))
            return rc;
    if (int rc = check_extent("split B blocks", (size_t)n_slots * bb, (size_t)n_slots * bb)) return rc;
    void *part, *B;
    if (int rc = fs_scratch(st, part_bytes, (size_t)n_slots * bb, &part, &B)) return rc;
    if (!baryon && bsplit) {
        FsSplitArgs sa;
        memset(&sa, 0, sizeof(sa));
        for (int j = 0; j < 3; ++j) sa.L[j] = geom->L[j];
        sa.Lp = Lp;
        sa.rows = rows;
        sa.n_slices = 1;
        sa.conj_sign = 1;
        sa.G[0] = (const float2*)G1;
        sa.out = B;
        if (int rc = to_status(timed("fs_split", st, [&] { return launch_fs_split(bf16, sa, st); }), "split launch"))
            return rc;
    }
    if (baryon) {
        FsDiquarkArgs da;
        for (int j = 0; j < 3; ++j) da.L[j] = geom->L[j];
        da.Lp = Lp;
        da.rows = rows;
        da.G1 = (const float2*)G1;
        da.G2 = (const float2*)G2;
        da.out = B;
        if (int rc = to_status(timed("fs_diquark", st, [&] { return launch_fs_diquark(bf16, da, st); }),
                               "diquark launch"))
            return rc;
    }
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const MomGroup& mg = groups[gi];
        const void* tab;
        if (int rc = factor_plan_table(plans[gi], false, st, &tab)) return rc;
        ProjGrid pg;
        memset(&pg, 0, sizeof(pg));
        pg.V3 = V3;
        pg.n_mom = mg.n;
        pg.chunk_planes = cp;
        pg.n_chunks = nch;
        pg.n_colblocks = ncb;
        pg.n_share = 1;
        pg.n_per_share = n_per_share;
        pg.phase = tab;
        pg.partial = part;
        FsArgs fa;
        memset(&fa, 0, sizeof(fa));
        for (int j = 0; j < 3; ++j) fa.L[j] = geom->L[j];
        fa.Lp = Lp;
        fa.rows = rows;
        fa.N = N;
        fa.n_share = 1;
        fa.n_slots = n_slots;
        fa.colmap = baryon ? 1 : 0;
        fa.B = B;
        fa.b_stride = bb;
        fa.G[0][0] = G1;
        fa.u0[0] = eta;
        if (int rc = to_status(timed(baryon ? "fs_spectator_baryon" : "fs_spectator_meson", st,
                                     [&] {
                                         return fs_launch_noise_parts(bf16, KT, 0, bsplit, cbw, N, n_slots, pg,
                                                                      fa, st);
                                     }),
                               "projection launch"))
            return rc;
        ReduceArgs ra;
        ra.partial = part;
        ra.f64 = 0;
        fill_phase(ra.ph, geom, -1, k, mg);
        ra.out = (double2*)out;
        ra.n_chunks = nch;
        ra.n_colblocks = ncb;
        ra.n_groups = N;
        ra.group_cols = baryon ? 3072 : kBlockCols;
        ra.n_mom_grp = mg.n;
        ra.n_mom_total = n_mom;
        ra.m_off = mg.off;
        ra.inner = N;
        ra.outer_stride = 0;
        ra.off = 0;
        if (int rc = to_status(timed("reduce", st, [&] { return launch_reduce(ra, st); }), "reduction launch"))
            return rc;
    }
    return C3PT_OK;
}

// The insertion on the fused path (n_ops 1 or 5; arguments already checked).
int fs_insertion(const c3pt_geom* geom, const void* const* G_t, const void* const* s_t, int N, const int* taus,
                 int n_tau, const void* const* U_t, int n_ops, const int* k, int n_mom, void* out) {
    std::vector<MomGroup> groups;
    std::vector<FactorPlan> plans;
    bool bsplit;
    int cbw;
    int KT;
    if (int rc = fs_setup(geom, +1, k, n_mom, 2, n_ops == 5, &groups, &plans, &bsplit, &cbw, &KT)) return rc;
    hipStream_t st = (hipStream_t)geom->stream;
    const bool bf16 = geom->proj == C3PT_PROJ_FACTORED_BF16;
    const int Lp = fs_lp(geom->L), rows = geom->L[1] * geom->L[2];
    const int V3 = geom->L[0] * rows;
    const int T = geom->T;
    const int kind = n_ops == 5 ? 2 : 1;
    const int n_slots = n_ops == 5 ? 9 : 1;
    const size_t bb = fs_block_bytes(geom->L);
    for (int j0 = 0; j0 < n_tau; j0 += kMaxTauPerLaunch) {
        const int nt = std::min(kMaxTauPerLaunch, n_tau - j0);
        FsArgs fa;
        memset(&fa, 0, sizeof(fa));
        for (int j = 0; j < nt; ++j) {
            const int t = taus[j0 + j];
            fa.G[j][0] = G_t[t];
            if (n_ops == 5) {
                fa.G[j][1] = G_t[(t + 1) % T];
                fa.G[j][2] = G_t[(t - 1 + T) % T];
                fa.U[j] = U_t[t];
                fa.Up[j] = U_t[(t - 1 + T) % T];
            }
            fa.u0[j] = s_t[t];
        }
        const int ncb = N * nt * n_slots;
        const int n_per_share = n_slots * ((N + cbw - 1) / cbw);
        int cp, nch;
        plan_planes(geom->L, n_per_share * nt, &cp, &nch);
        const size_t part_bytes = (size_t)nch * ncb * kMaxMomGroupF32 * kBlockCols * sizeof(float2);
        // with the split pass: the distinct slices of the launch and the block of each role
        std::vector<int> sl;
        if (bsplit) {
            auto slot_of = [&](int t) {
                t = ((t % T) + T) % T;
                auto it = std::find(sl.begin(), sl.end(), t);
                if (it != sl.end()) return (int)(it - sl.begin());
                sl.push_back(t);
                return (int)sl.size() - 1;
            };
            for (int j = 0; j < nt; ++j) {
                const int t = taus[j0 + j];
                fa.bidx[j][0] = slot_of(t);
                if (n_ops == 5) {
                    fa.bidx[j][1] = slot_of(t + 1);
                    fa.bidx[j][2] = slot_of(t - 1);
                }
            }
        }
        for (const MomGroup& mg : groups)
            if (int rc = check_extent("partial sums", partial_indexed_bytes(nch, ncb, mg.n, sizeof(float2)),
                                      part_bytes))
                return rc;
        if (bsplit) {
            int bmax = 0;
            for (int j = 0; j < nt; ++j)
                for (int r = 0; r < (n_ops == 5 ? 3 : 1); ++r) bmax = std::max(bmax, fa.bidx[j][r] + 1);
            if (int rc = check_extent("split B blocks", (size_t)bmax * bb, sl.size() * bb)) return rc;
        }
        void *part, *B;
        if (int rc = fs_scratch(st, part_bytes, sl.size() * bb, &part, &B)) return rc;
        for (size_t s0 = 0; s0 < sl.size(); s0 += kMaxTauPerLaunch + 2) {
            FsSplitArgs sa;
            memset(&sa, 0, sizeof(sa));
            for (int j = 0; j < 3; ++j) sa.L[j] = geom->L[j];
            sa.Lp = Lp;
            sa.rows = rows;
            sa.n_slices = (int)std::min(sl.size() - s0, (size_t)kMaxTauPerLaunch + 2);
            sa.conj_sign = 0;
            for (int j = 0; j < sa.n_slices; ++j) sa.G[j] = (const float2*)G_t[sl[s0 + j]];
            sa.out = (char*)B + s0 * bb;
            if (int rc = to_status(timed("fs_split", st, [&] { return launch_fs_split(bf16, sa, st); }),
                                   "split launch"))
                return rc;
        }
        fa.B = B;
        fa.b_stride = bb;
        for (int j = 0; j < 3; ++j) fa.L[j] = geom->L[j];
        fa.Lp = Lp;
        fa.rows = rows;
        fa.N = N;
        fa.n_share = nt;
        fa.n_slots = n_slots;
        fa.colmap = 0;
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const MomGroup& mg = groups[gi];
            const void* tab;
            if (int rc = factor_plan_table(plans[gi], false, st, &tab)) return rc;
            ProjGrid pg;
            memset(&pg, 0, sizeof(pg));
            pg.V3 = V3;
            pg.n_mom = mg.n;
            pg.chunk_planes = cp;
            pg.n_chunks = nch;
            pg.n_colblocks = ncb;
            pg.n_share = nt;
            pg.n_per_share = n_per_share;
            pg.phase = tab;
            pg.partial = part;
            if (int rc = to_status(timed("fs_insertion", st,
                                         [&] {
                                             return fs_launch_noise_parts(bf16, KT, kind, bsplit, cbw, N, n_slots,
                                                                          pg, fa, st);
                                         }),
                                   "projection launch"))
                return rc;
            if (kind == 1) {
                ReduceArgs ra;
                ra.partial = part;
                ra.f64 = 0;
                fill_phase(ra.ph, geom, +1, k, mg);
                ra.out = (double2*)out;
                ra.n_chunks = nch;
                ra.n_colblocks = ncb;
                ra.n_groups = ncb;
                ra.group_cols = kBlockCols;
                ra.n_mom_grp = mg.n;
                ra.n_mom_total = n_mom;
                ra.m_off = mg.off;
                ra.inner = nt;
                ra.outer_stride = n_tau;
                ra.off = j0;
                if (int rc = to_status(timed("reduce", st, [&] { return launch_reduce(ra, st); }), "reduction launch"))
                    return rc;
            } else {
                FsReduceArgs ra;
                ra.partial = (const float2*)part;
                ra.out = (double2*)out;
                fill_phase(ra.ph, geom, +1, k, mg);
                ra.n_chunks = nch;
                ra.n_colblocks = ncb;
                ra.N = N;
                ra.nt = nt;
                ra.j0 = j0;
                ra.n_tau_total = n_tau;
                ra.n_mom_grp = mg.n;
                ra.n_mom_total = n_mom;
                ra.m_off = mg.off;
                if (int rc = to_status(timed("reduce", st, [&] { return launch_fs_reduce(ra, st); }),
                                       "reduction launch"))
                    return rc;
            }
        }
    }
    return C3PT_OK;
}

}  // namespace

// Shared with the batch API (c3pt_batch.hip).
namespace c3pt {
bool api_factor_plan(const int L[3], int sigma, const int* k, int n_mom, FactorPlan* plan) {
    c3pt_geom g;
    memset(&g, 0, sizeof(g));
    for (int j = 0; j < 3; ++j) g.L[j] = L[j];
    return build_factor_plan(&g, sigma, k, MomGroup{0, n_mom}, false, plan);
}
int api_fail(int code, const char* msg) { return fail(code, "%s", msg); }
int api_ok() { return ok(); }
int api_variant(int kind, int mode, int mt) {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_variant[kind][mode][mt_class(mt)];
}
bool api_profiling() {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return g_prof_on;
}
hipError_t api_timed(const char* name, hipStream_t st, const std::function<hipError_t()>& fn) {
    return timed(name, st, fn);
}
}  // namespace c3pt

// c3pt_combine over the insertion timeslices [tau0, tau0 + n_tau) of an
// insertion output holding n_tau_in slices.
// The symmetrized and the two-derivative operators run on the factored
// projection only: every momentum group of the list must factor.
static int check_symmetric(const c3pt_geom* g, const int* k, int n_mom) {
    if (g->proj != C3PT_PROJ_FACTORED)
        return fail(C3PT_EUNSUPPORTED, "n_ops = 9 and 21 need the factored projection (C3PT_PROJ_FACTORED)");
    const bool f64 = g->dtype == C3PT_C128;
    for (const MomGroup& mg : momentum_groups(n_mom, f64)) {
        FactorPlan plan;
        if (!build_factor_plan(g, +1, k, mg, f64, &plan))
            return fail(C3PT_EUNSUPPORTED, "n_ops = 9 or 21: the momentum list does not factor (too many distinct k1)");
    }
    return C3PT_OK;
}

static int combine_impl(const void* spec, int spec_spin, const void* ins, int n_noise, int n_p, int n_q, int n_tau_in,
                 int tau0, int n_tau, int n_ops, int op_begin, int op_end, const double* w, const int* pairs,
                 int n_pairs, void* out, void* stream) {
    if (!spec || !ins || !out) return fail(C3PT_EINVAL, "NULL input or output pointer");
    if (spec_spin != 64 && spec_spin != 1024) return fail(C3PT_EINVAL, "spec_spin = %d (64 or 1024)", spec_spin);
    if (n_noise < 1 || n_p < 1 || n_q < 1 || n_tau < 1 || n_ops < 1)
        return fail(C3PT_EINVAL, "extents must be >= 1");
    if (tau0 < 0 || tau0 + n_tau > n_tau_in)
        return fail(C3PT_EINVAL, "timeslice window [%d, %d) outside the %d insertion slices", tau0, tau0 + n_tau,
                    n_tau_in);
    if (op_begin < 0 || op_end > n_ops || op_begin >= op_end)
        return fail(C3PT_EINVAL, "operator range [%d, %d) invalid for n_ops = %d", op_begin, op_end, n_ops);
    if (!pairs) {
        if (n_pairs != n_p * n_q) return fail(C3PT_EINVAL, "n_pairs must be n_p*n_q when pairs is NULL");
    } else {
        if (n_pairs < 1) return fail(C3PT_EINVAL, "n_pairs = %d < 1", n_pairs);
        for (int j = 0; j < n_pairs; ++j)
            if (pairs[2 * j] < 0 || pairs[2 * j] >= n_p || pairs[2 * j + 1] < 0 || pairs[2 * j + 1] >= n_q)
                return fail(C3PT_EINVAL, "pair %d = (%d, %d) out of range", j, pairs[2 * j], pairs[2 * j + 1]);
    }
    if ((long long)n_pairs * n_tau * (op_end - op_begin) > 0x7fffffffLL)
        return fail(C3PT_EINVAL, "too many (pair, tau, op) tiles");
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> wv(n_noise);
    for (int i = 0; i < n_noise; ++i) wv[i] = w ? w[i] : 1.0 / n_noise;
    const size_t wbytes = (size_t)n_noise * sizeof(double);
    const size_t pbytes = pairs ? (size_t)n_pairs * 2 * sizeof(int) : 0;
    const size_t woff = 0, poff = (wbytes + 255) & ~(size_t)255;
    // Weights and pairs go to the start of this stream's scratch; kernels of
    // earlier calls on the same stream that use it are ordered before the upload.
    void* base;
    if (int rc = scratch_dev(st, poff + pbytes + 256, &base)) return rc;
    std::vector<char> host(poff + pbytes);
    memcpy(host.data() + woff, wv.data(), wbytes);
    if (pairs) memcpy(host.data() + poff, pairs, pbytes);
    if (int rc = upload(st, base, 0, host.data(), host.size())) return rc;
    CombineArgs a;
    a.S = (const double2*)spec;
    a.I = (const double2*)ins;
    a.w = (const double*)base;
    a.pairs = pairs ? (const int*)((char*)base + poff) : nullptr;
    a.out = (double2*)out;
    a.n_noise = n_noise;
    a.n_p = n_p;
    a.n_q = n_q;
    a.n_tau = n_tau;
    a.n_ops = n_ops;
    a.op_begin = op_begin;
    a.n_sel = op_end - op_begin;
    a.spin = spec_spin;
    a.n_pairs = n_pairs;
    a.tau0 = tau0;
    a.n_tau_in = n_tau_in;
    if (int rc = to_status(timed("combine", st, [&] { return launch_combine(a, st); }), "combine launch"))
        return rc;
    return ok();
}

extern "C" {

int c3pt_version(void) { return 100; }

const char* c3pt_strerror(int status) {
    switch (status) {
        case C3PT_OK: return "success";
        case C3PT_EINVAL: return "invalid argument";
        case C3PT_ENOMEM: return "out of device memory";
        case C3PT_EDEVICE: return "device error";
        case C3PT_EUNSUPPORTED: return "unsupported request";
        default: return "unknown status";
    }
}

const char* c3pt_last_error(void) { return g_last_error.c_str(); }

void c3pt_debug_scale_allocations(double scale) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_extent_scale = scale > 0.0 ? scale : 1.0;
}

unsigned long long c3pt_scratch_bytes(void* stream) {
    int dev;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find({dev, (hipStream_t)stream});
    return it == g_scratch.end() ? 0ull : (unsigned long long)it->second.dev_bytes;
}

int c3pt_release_scratch(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(C3PT_EDEVICE, "hipGetDevice failed");
    for (auto& kv : g_phase) {
        hipSetDevice(kv.first.dev);
        hipDeviceSynchronize();
        free_phase_entry(kv.second);
    }
    g_phase.clear();
    for (auto& kv : g_scratch) {
        hipSetDevice(kv.first.first);
        hipStreamSynchronize(kv.first.second);
        if (kv.second.dev) hipFree(kv.second.dev);
        if (kv.second.aux) hipFree(kv.second.aux);
        for (int k = 0; k < kUploadSlots; ++k) {
            if (kv.second.pinned[k]) hipHostFree(kv.second.pinned[k]);
            if (kv.second.ev[k]) hipEventDestroy(kv.second.ev[k]);
        }
    }
    g_scratch.clear();
    hipSetDevice(cur);
    return ok();
}

int c3pt_variant_count(int kind, int mode, int mt_cls) { return variant_count(kind, mode, mt_cls); }

int c3pt_set_variant(int kind, int mode, int mt_cls, int variant) {
    const int n = variant_count(kind, mode, mt_cls);
    if (n == 0) return fail(C3PT_EINVAL, "no kernel for kind %d, mode %d, class %d", kind, mode, mt_cls);
    if (variant < 0 || variant >= n) return fail(C3PT_EINVAL, "variant %d outside [0, %d)", variant, n);
    std::lock_guard<std::mutex> lk(g_mu);
    g_variant[kind][mode][mt_cls] = variant;
    return ok();
}

int c3pt_get_variant(int kind, int mode, int mt_cls) {
    if (variant_count(kind, mode, mt_cls) == 0) return fail(C3PT_EINVAL, "no kernel for this key");
    std::lock_guard<std::mutex> lk(g_mu);
    return g_variant[kind][mode][mt_cls];
}

int c3pt_profile_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return ok();
}

int c3pt_profile_read(c3pt_kernel_stat* stats, int max, int reset) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (ProfRec& r : g_prof_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
            return fail(C3PT_EDEVICE, "timing event failed");
        ProfStat& st = g_prof_stats[r.name];
        st.count++;
        st.total += ms;
        st.mn = std::min(st.mn, (double)ms);
        st.mx = std::max(st.mx, (double)ms);
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    int n = 0;
    for (auto& kv : g_prof_stats) {
        if (stats && n < max) {
            c3pt_kernel_stat& o = stats[n];
            memset(&o, 0, sizeof(o));
            strncpy(o.name, kv.first.c_str(), sizeof(o.name) - 1);
            o.count = kv.second.count;
            o.total_ms = kv.second.total;
            o.min_ms = kv.second.mn;
            o.max_ms = kv.second.mx;
        }
        ++n;
    }
    if (reset) g_prof_stats.clear();
    g_last_error.clear();
    return n;
}

int c3pt_spectator_meson(const c3pt_geom* geom, const void* G_tf, const void* eta, int n_noise,
                         const int* k, int n_mom, void* out) {
    if (int rc = check_geom(geom)) return rc;
    if (int rc = check_momenta(k, n_mom)) return rc;
    if (!G_tf || !eta || !out) return fail(C3PT_EINVAL, "NULL field or output pointer");
    if (n_noise < 1) return fail(C3PT_EINVAL, "n_noise = %d < 1", n_noise);
    if (is_fused(geom)) {
        const int rc = fs_spectator(geom, false, G_tf, nullptr, eta, n_noise, k, n_mom, out);
        return rc ? rc : ok();
    }
    MesonSpecArgs a{{geom->L[0], geom->L[1], geom->L[2]}, G_tf, eta};
    int rc = run_projection("proj_spectator_meson", 0, geom, -1, k, n_mom, n_noise, 1, n_noise, kBlockCols,
                            n_noise, n_noise, 0, 0, out, [&](int mode, const ProjGrid& pg, int mt, int variant, bool fac) {
                                hipStream_t st = (hipStream_t)geom->stream;
                                return fac ? launch_fac_meson(geom->dtype == C3PT_C128, pg.fac_acc, pg, a, st)
                                           : launch_spectator_meson(mode, mt, variant, pg, a, st);
                            });
    return rc ? rc : ok();
}

int c3pt_spectator_baryon(const c3pt_geom* geom, const void* G1_tf, const void* G2_tf,
                          const void* eta, int n_noise, const int* k, int n_mom, void* out) {
    if (int rc = check_geom(geom)) return rc;
    if (int rc = check_momenta(k, n_mom)) return rc;
    if (!G1_tf || !G2_tf || !eta || !out) return fail(C3PT_EINVAL, "NULL field or output pointer");
    if (n_noise < 1) return fail(C3PT_EINVAL, "n_noise = %d < 1", n_noise);
    if (is_fused(geom)) {
        const int rc = fs_spectator(geom, true, G1_tf, G2_tf, eta, n_noise, k, n_mom, out);
        return rc ? rc : ok();
    }
    BaryonSpecArgs a{{geom->L[0], geom->L[1], geom->L[2]}, G1_tf, G2_tf, eta};
    int rc = run_projection("proj_spectator_baryon", 1, geom, -1, k, n_mom, n_noise * 16, 1, n_noise * 16, 3072,
                            n_noise, n_noise, 0, 0, out, [&](int mode, const ProjGrid& pg, int mt, int variant, bool fac) {
                                hipStream_t st = (hipStream_t)geom->stream;
                                return fac ? launch_fac_baryon(geom->dtype == C3PT_C128, pg.fac_acc, pg, a, st)
                                           : launch_spectator_baryon(mode, mt, variant, pg, a, st);
                            });
    return rc ? rc : ok();
}

int c3pt_insertion(const c3pt_geom* geom, const void* const* G_t, const void* const* s_t,
                   int n_noise, const int* taus, int n_tau, const void* const* U_t, int n_ops,
                   const int* k, int n_mom, void* out) {
    if (int rc = check_geom(geom)) return rc;
    if (int rc = check_momenta(k, n_mom)) return rc;
    if (!G_t || !s_t || !out) return fail(C3PT_EINVAL, "NULL pointer table or output");
    if (n_noise < 1) return fail(C3PT_EINVAL, "n_noise = %d < 1", n_noise);
    if (n_tau < 1 || !taus) return fail(C3PT_EINVAL, "empty timeslice list");
    if (n_ops != 1 && n_ops != 5 && n_ops != 9 && n_ops != 21 && n_ops != 37)
        return fail(C3PT_EINVAL, "n_ops = %d (must be 1, 5, 9, 21 or 37)", n_ops);
    if (n_ops > 1 && !U_t) return fail(C3PT_EINVAL, "derivative operators need gauge links");
    const int T = geom->T;
    for (int j = 0; j < n_tau; ++j) {
        const int t = taus[j];
        if (t < 0 || t >= T) return fail(C3PT_EINVAL, "taus[%d] = %d outside [0, %d)", j, t, T);
        if (!G_t[t]) return fail(C3PT_EINVAL, "propagator slice %d missing", t);
        if (!s_t[t]) return fail(C3PT_EINVAL, "stochastic solution slice %d missing", t);
        if (n_ops > 1) {
            const int tn = (t + 1) % T, tp = (t - 1 + T) % T;
            if (!G_t[tn] || !G_t[tp])
                return fail(C3PT_EINVAL, "propagator slices %d and %d needed around %d", tp, tn, t);
            if (!U_t[t] || !U_t[tp]) return fail(C3PT_EINVAL, "link slices %d and %d needed", tp, t);
            if ((n_ops == 9 || n_ops == 37) && (!s_t[tn] || !s_t[tp]))
                return fail(C3PT_EINVAL, "stochastic solution slices %d and %d needed around %d", tp, tn, t);
            if (n_ops >= 21) {
                const int tn2 = (t + 2) % T, tp2 = (t - 2 + 2 * T) % T;
                if (!G_t[tn2] || !G_t[tp2])
                    return fail(C3PT_EINVAL, "propagator slices %d and %d needed around %d", tp2, tn2, t);
                if (!U_t[tn] || !U_t[tp2]) return fail(C3PT_EINVAL, "link slices %d and %d needed", tp2, tn);
                if (n_ops == 37 && (!s_t[tn2] || !s_t[tp2]))
                    return fail(C3PT_EINVAL, "stochastic solution slices %d and %d needed around %d", tp2, tn2, t);
            }
        }
    }
    if (is_fused(geom)) {
        if (n_ops != 1 && n_ops != 5)
            return fail(C3PT_EUNSUPPORTED, "the split-precision fused projection takes n_ops 1 or 5");
        const int rc = fs_insertion(geom, G_t, s_t, n_noise, taus, n_tau, U_t, n_ops, k, n_mom, out);
        return rc ? rc : ok();
    }
    if (n_ops >= 9) {
        if (int rc = check_symmetric(geom, k, n_mom)) return rc;
    }
    // n_ops = 37 runs 53 internal operators: 0..20 as n_ops = 21, then the
    // mixed terms (D_mu s with D_nu G, ops 21 + 4 mu + nu) and the left-left
    // terms (D_nu D_mu s with G, ops 37 + 4 mu + nu); the symmetrized operators
    // are assembled from them at the end
    const int n_int = n_ops == 37 ? 53 : n_ops;
    const bool f64 = geom->dtype == C3PT_C128;
    const size_t elem = f64 ? sizeof(double2) : sizeof(float2);
    const long long V3 = (long long)geom->L[0] * geom->L[1] * geom->L[2];
    hipStream_t dst = (hipStream_t)geom->stream;
    // the stream's second scratch region: the internal operator parts of
    // n_ops = 37, then the derived slices of one launch (the largest launch's)
    const size_t gslice = (size_t)144 * V3 * elem, sslice = (size_t)n_noise * 12 * V3 * elem;
    auto derived_slices = [&](int j0, int nt) {
        std::vector<int> d;
        for (int j = 0; j < nt; ++j)
            for (int dt = -1; dt <= 1; ++dt) {
                const int t = ((taus[j0 + j] + dt) % T + T) % T;
                if (std::find(d.begin(), d.end(), t) == d.end()) d.push_back(t);
            }
        return d;
    };
    const size_t ibytes = n_ops == 37 ? (size_t)n_noise * n_tau * n_int * n_mom * kBlockCols * sizeof(double2) : 0;
    const size_t doff = (ibytes + 255) & ~(size_t)255;
    size_t dmax = 0;
    if (n_ops >= 21)
        for (int j0 = 0; j0 < n_tau; j0 += kMaxTauPerLaunch) {
            const int nt = std::min(kMaxTauPerLaunch, n_tau - j0);
            const size_t nd = derived_slices(j0, nt).size();
            size_t bytes = 4 * nd * gslice;
            if (n_ops == 37) bytes += 4 * nd * sslice + (size_t)16 * nt * sslice;
            dmax = std::max(dmax, bytes);
        }
    void* aux = nullptr;
    if (doff + dmax > 0) {
        if (int rc = scratch_aux(dst, doff + dmax, &aux)) return rc;
    }
    void* outp = out;
    void* iout = n_ops == 37 ? aux : nullptr;
    if (n_ops == 37) outp = iout;
    auto stencil = [&](const void* fp, const void* fm, const void* U, const void* Um, void* o, int n_outer,
                       int n_inner, int rho) {
        DerivStencilArgs da;
        da.fp = fp;
        da.fm = fm;
        da.U = U;
        da.Um = Um;
        da.out = o;
        for (int q = 0; q < 3; ++q) da.L[q] = geom->L[q];
        da.V3 = (int)V3;
        da.n_outer = n_outer;
        da.n_inner = n_inner;
        da.rho = rho;
        return to_status(timed("cov_deriv", dst, [&] { return launch_cov_deriv(f64, da, dst); }),
                         "derivative stencil launch");
    };
    for (int j0 = 0; j0 < n_tau; j0 += kMaxTauPerLaunch) {
        const int nt = std::min(kMaxTauPerLaunch, n_tau - j0);
        InsertionLeftArgs a;
        memset(&a, 0, sizeof(a));
        for (int j = 0; j < 3; ++j) a.L[j] = geom->L[j];
        a.n_tau = nt;
        a.n_ops = n_int;
        a.n_noise = n_noise;
        a.op_lo = 0;
        a.op_cnt = n_int;
        for (int j = 0; j < nt; ++j) {
            const int t = taus[j0 + j];
            const int tn = (t + 1) % T, tp = (t - 1 + T) % T;
            a.G[j] = G_t[t];
            a.s[j] = s_t[t];
            if (n_ops > 1) {
                a.Gn[j] = G_t[tn];
                a.Gp[j] = G_t[tp];
                a.U[j] = U_t[t];
                a.Up[j] = U_t[tp];
            }
            if (n_ops == 9) {
                a.sn[j] = s_t[tn];
                a.sp[j] = s_t[tp];
            }
        }
        // derived fields in stream-ordered memory freed after the projection:
        // D_rho G on every slice next to a timeslice of this launch; with
        // n_ops = 37 also D_mu s there and D_nu D_mu s on the timeslices
        std::vector<int> dsl;
        void* dbuf = nullptr;
        auto dslot = [&](int t) { return (int)(std::find(dsl.begin(), dsl.end(), ((t % T) + T) % T) - dsl.begin()); };
        auto dG = [&](int rho, int t) { return (char*)dbuf + (rho * dsl.size() + dslot(t)) * gslice; };
        auto dS = [&](int mu, int t) {
            return (char*)dbuf + 4 * dsl.size() * gslice + (mu * dsl.size() + dslot(t)) * sslice;
        };
        auto ddS = [&](int mu, int nu, int j) {
            return (char*)dbuf + 4 * dsl.size() * (gslice + sslice) + ((size_t)(4 * mu + nu) * nt + j) * sslice;
        };
        if (n_ops >= 21) {
            dsl = derived_slices(j0, nt);
            dbuf = (char*)aux + doff;
            int rc = 0;
            for (int rho = 0; rho < 4 && !rc; ++rho)
                for (size_t m = 0; m < dsl.size() && !rc; ++m) {
                    const int t = dsl[m], tn = (t + 1) % T, tp = (t - 1 + T) % T;
                    rc = stencil(G_t[rho < 3 ? t : tn], G_t[rho < 3 ? t : tp], U_t[t], U_t[rho < 3 ? t : tp],
                                 dG(rho, t), 4, 12, rho);
                    if (!rc && n_ops == 37)
                        rc = stencil(s_t[rho < 3 ? t : tn], s_t[rho < 3 ? t : tp], U_t[t], U_t[rho < 3 ? t : tp],
                                     dS(rho, t), 4 * n_noise, 1, rho);
                }
            for (int mu = 0; mu < 4 && !rc && n_ops == 37; ++mu)
                for (int nu = 0; nu < 4 && !rc; ++nu)
                    for (int j = 0; j < nt && !rc; ++j) {
                        const int t = taus[j0 + j], tn = (t + 1) % T, tp = (t - 1 + T) % T;
                        rc = stencil(dS(mu, nu < 3 ? t : tn), dS(mu, nu < 3 ? t : tp), U_t[t],
                                     U_t[nu < 3 ? t : tp], ddS(mu, nu, j), 4 * n_noise, 1, nu);
                    }
            if (rc) return rc;
        }
        const int ncb = n_noise * nt * n_int;
        int rc = run_projection("proj_insertion", 2, geom, +1, k, n_mom, ncb, nt, n_noise * n_int, kBlockCols, ncb,
                                nt * n_int, n_tau * n_int, j0 * n_int, outp, [&](int mode, const ProjGrid& pg, int mt, int variant, bool fac) {
                                    hipStream_t st = (hipStream_t)geom->stream;
                                    if (!fac) {
                                        if (n_ops >= 9) return hipErrorNotSupported;
                                        return launch_insertion(mode, mt, variant, pg, a, st);
                                    }
                                    // local and derivative operators in separate launches (each
                                    // kernel keeps only its own path's registers)
                                    InsertionArgs al = a;
                                    al.op_lo = 0;
                                    al.op_cnt = 1;
                                    ProjGrid pl = pg;
                                    pl.n_per_share = n_noise;
                                    hipError_t e = launch_fac_insertion(f64, pg.fac_acc, 1, pl, al, st);
                                    if (e != hipSuccess || n_ops == 1) return e;
                                    InsertionArgs ad = a;
                                    ad.op_lo = 1;
                                    ad.op_cnt = 4;
                                    ProjGrid pd = pg;
                                    pd.n_per_share = n_noise * 4;
                                    e = launch_fac_insertion(f64, pg.fac_acc, 2, pd, ad, st);
                                    if (e != hipSuccess || n_ops == 5) return e;
                                    if (n_ops == 9) {
                                        InsertionLeftArgs ab = a;
                                        ab.op_lo = 5;
                                        ab.op_cnt = 4;
                                        return launch_fac_insertion_left(f64, pg.fac_acc, pd, ab, st);
                                    }
                                    // D_nu of the field D_rho G: the derivative producer on it
                                    for (int rho = 0; rho < 4 && e == hipSuccess; ++rho) {
                                        InsertionArgs ar = a;
                                        ar.op_lo = 5 + 4 * rho;
                                        ar.op_cnt = 4;
                                        for (int j = 0; j < nt; ++j) {
                                            const int t = taus[j0 + j];
                                            ar.G[j] = dG(rho, t);
                                            ar.Gn[j] = dG(rho, t + 1);
                                            ar.Gp[j] = dG(rho, t - 1);
                                        }
                                        e = launch_fac_insertion(f64, pg.fac_acc, 2, pd, ar, st);
                                    }
                                    if (e != hipSuccess || n_ops == 21) return e;
                                    // mixed terms: D_nu G contracted with D_mu s
                                    for (int mu = 0; mu < 4 && e == hipSuccess; ++mu) {
                                        InsertionArgs am = a;
                                        am.op_lo = 21 + 4 * mu;
                                        am.op_cnt = 4;
                                        for (int j = 0; j < nt; ++j) am.s[j] = dS(mu, taus[j0 + j]);
                                        e = launch_fac_insertion(f64, pg.fac_acc, 2, pd, am, st);
                                    }
                                    // left-left terms: G contracted with D_nu D_mu s (local producer;
                                    // its neighbour pointers are G itself)
                                    for (int mn = 0; mn < 16 && e == hipSuccess; ++mn) {
                                        InsertionArgs aw = a;
                                        aw.op_lo = 37 + mn;
                                        aw.op_cnt = 1;
                                        for (int j = 0; j < nt; ++j) {
                                            aw.s[j] = ddS(mn / 4, mn % 4, j);
                                            aw.Gn[j] = aw.Gp[j] = aw.G[j];
                                        }
                                        e = launch_fac_insertion(f64, pg.fac_acc, 1, pl, aw, st);
                                    }
                                    return e;
                                });
        if (rc) return rc;
    }
    if (n_ops == 9) {
        if (int rc = to_status(timed("symmetrize", dst, [&] {
                                   return launch_symmetrize((double2*)out, (long long)n_noise * n_tau, n_mom, dst);
                               }),
                               "symmetrize launch"))
            return rc;
    }
    if (n_ops == 37) {
        if (int rc = to_status(timed("symmetrize", dst, [&] {
                                   return launch_assemble_sym2((const double2*)iout, (double2*)out,
                                                               (long long)n_noise * n_tau, n_mom, dst);
                               }),
                               "assembly launch"))
            return rc;
    }
    return ok();
}

}  // extern "C"

// ---- the insertion entry point that allocates nothing ----------------------
// Its partial sums and the factor plan of each launch live in one fixed
// device array instead of the per-stream scratch and the plan cache.  On the
// host, `scratch` names a host-side stand-in; its device address, one per
// GPU, comes from hipGetSymbolAddress at the first call on that GPU and is the
// only form passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[C3PT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr size_t kNoAllocBytes = (size_t)C3PT_NOALLOC_SCRATCH_BYTES;
constexpr size_t kNoAllocPlanOff = 0;       // FactorPlan of the running launch
constexpr size_t kNoAllocPartOff = 4096;    // split-site partial sums
static_assert(sizeof(FactorPlan) <= kNoAllocPartOff, "the factor plan slot is too small");

std::mutex g_na_mu;
std::map<int, unsigned char*> g_na_ptr;   // device ordinal -> device address of scratch on it

int noalloc_scratch(unsigned char** out) {
    int dev;
    if (int rc = current_device(&dev)) return rc;
    std::lock_guard<std::mutex> lk(g_na_mu);
    auto it = g_na_ptr.find(dev);
    if (it == g_na_ptr.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return fail(C3PT_EDEVICE, "hipGetSymbolAddress of the fixed scratch failed: %s", hipGetErrorString(e));
        }
        it = g_na_ptr.emplace(dev, (unsigned char*)ptr).first;
    }
    *out = it->second;
    return C3PT_OK;
}

// The factor plan travels by value in the kernel arguments and is written
// into the plan slot by one workgroup (no host copy, no allocation).
struct PlanWords {
    int w[sizeof(FactorPlan) / sizeof(int)];
};
__global__ void __launch_bounds__(256) put_plan_kernel(PlanWords pw, int* dst) {
    for (int i = threadIdx.x; i < (int)(sizeof(FactorPlan) / sizeof(int)); i += blockDim.x) dst[i] = pw.w[i];
}

// One launch group of the no-alloc insertion: a momentum group and a block
// of timeslices, with the chunking of its partial sums.
struct NoAllocPiece {
    int mg, j0, nt, chunk_planes, n_chunks;
    FactorPlan plan;
};
}  // namespace

extern "C" {

unsigned long long c3pt_noalloc_scratch_bytes(void) { return (unsigned long long)kNoAllocBytes; }

int c3pt_insertion_noalloc(const c3pt_geom* geom, const void* const* G_t, const void* const* s_t, int n_noise,
                           const int* taus, int n_tau, const void* const* U_t, int n_ops, const int* k, int n_mom,
                           void* out) {
    if (int rc = check_geom(geom)) return rc;
    if (int rc = check_momenta(k, n_mom)) return rc;
    if (geom->proj != C3PT_PROJ_FACTORED)
        return fail(C3PT_EUNSUPPORTED, "c3pt_insertion_noalloc runs the factored projection only (C3PT_PROJ_FACTORED)");
    if (!G_t || !s_t || !out) return fail(C3PT_EINVAL, "NULL pointer table or output");
    if (n_noise < 1) return fail(C3PT_EINVAL, "n_noise = %d < 1", n_noise);
    if (n_tau < 1 || !taus) return fail(C3PT_EINVAL, "empty timeslice list");
    if (n_ops != 1 && n_ops != 5) return fail(C3PT_EINVAL, "n_ops = %d (c3pt_insertion_noalloc: 1 or 5)", n_ops);
    if (n_ops > 1 && !U_t) return fail(C3PT_EINVAL, "derivative operators need gauge links");
    const int T = geom->T;
    for (int j = 0; j < n_tau; ++j) {
        const int t = taus[j];
        if (t < 0 || t >= T) return fail(C3PT_EINVAL, "taus[%d] = %d outside [0, %d)", j, t, T);
        if (!G_t[t]) return fail(C3PT_EINVAL, "propagator slice %d missing", t);
        if (!s_t[t]) return fail(C3PT_EINVAL, "stochastic solution slice %d missing", t);
        if (n_ops > 1) {
            const int tn = (t + 1) % T, tp = (t - 1 + T) % T;
            if (!G_t[tn] || !G_t[tp])
                return fail(C3PT_EINVAL, "propagator slices %d and %d needed around %d", tp, tn, t);
            if (!U_t[t] || !U_t[tp]) return fail(C3PT_EINVAL, "link slices %d and %d needed", tp, t);
        }
    }
    const bool f64 = geom->dtype == C3PT_C128;
    const size_t elem = f64 ? sizeof(double2) : sizeof(float2);
    const auto groups = momentum_groups(n_mom, f64);
    const size_t cap = kNoAllocBytes - kNoAllocPartOff;
    // plan every launch before anything is enqueued
    std::vector<NoAllocPiece> pieces;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        FactorPlan plan;
        if (!build_factor_plan(geom, +1, k, groups[gi], f64, &plan))
            return fail(C3PT_EUNSUPPORTED, "the momentum list does not factor (too many distinct k1 or (k1, k2))");
        const int max_planes =
            f64 ? geom->L[2] : std::max(1, std::min(geom->L[2], kMaxSitesPerChunkF32 / (geom->L[0] * geom->L[1])));
        for (int j0 = 0; j0 < n_tau;) {
            const int nt_max = std::min(kMaxTauPerLaunch, n_tau - j0);
            int nt = 0, cp = 0, nc = 0;
            for (int cand = nt_max; cand >= 1 && nt == 0; --cand) {
                const int ncb = n_noise * cand * n_ops;
                int c, n;
                plan_planes(geom->L, ncb, &c, &n);
                // one timeslice that does not fit: fewer, larger chunks (within the FP32 limit)
                while (cand == 1 && (size_t)n * ncb * groups[gi].n * kBlockCols * elem > cap && c < max_planes) {
                    c = std::min(max_planes, 2 * c);
                    n = (geom->L[2] + c - 1) / c;
                }
                if ((size_t)n * ncb * groups[gi].n * kBlockCols * elem <= cap) {
                    nt = cand;
                    cp = c;
                    nc = n;
                }
            }
            if (nt == 0) {
                int c = max_planes, n = (geom->L[2] + c - 1) / c;
                const size_t need = (size_t)n * n_noise * n_ops * groups[gi].n * kBlockCols * elem;
                return fail(C3PT_EINVAL,
                            "one timeslice needs %zu bytes of partial sums; the fixed scratch of "
                            "c3pt_insertion_noalloc holds %zu",
                            need, cap);
            }
            pieces.push_back(NoAllocPiece{(int)gi, j0, nt, cp, nc, plan});
            j0 += nt;
        }
    }
    for (const NoAllocPiece& pc : pieces)
        if (int rc = check_extent("partial sums",
                                  partial_indexed_bytes(pc.n_chunks, n_noise * pc.nt * n_ops, groups[pc.mg].n, elem),
                                  cap))
            return rc;
    unsigned char* base;
    if (int rc = noalloc_scratch(&base)) return rc;
    int* plan_dev = (int*)(base + kNoAllocPlanOff);
    void* part = base + kNoAllocPartOff;
    hipStream_t st = (hipStream_t)geom->stream;
    const int V3 = geom->L[0] * geom->L[1] * geom->L[2];
    for (const NoAllocPiece& pc : pieces) {
        const MomGroup& mg = groups[pc.mg];
        PlanWords pw;
        memcpy(pw.w, &pc.plan, sizeof(FactorPlan));
        hipLaunchKernelGGL(put_plan_kernel, dim3(1), dim3(256), 0, st, pw, plan_dev);
        if (hipError_t e = hipGetLastError(); e != hipSuccess) return to_status(e, "plan launch");
        const int ncb = n_noise * pc.nt * n_ops;
        ProjGrid pg;
        pg.V3 = V3;
        pg.n_mom = mg.n;
        pg.chunk_sites = 0;
        pg.chunk_planes = pc.chunk_planes;
        pg.fac_acc = 0;
        pg.n_chunks = pc.n_chunks;
        pg.n_colblocks = ncb;
        pg.n_share = pc.nt;
        pg.n_per_share = n_noise * n_ops;
        pg.phase = plan_dev;
        pg.partial = part;
        InsertionArgs a;
        memset(&a, 0, sizeof(a));
        for (int j = 0; j < 3; ++j) a.L[j] = geom->L[j];
        a.n_tau = pc.nt;
        a.n_ops = n_ops;
        a.n_noise = n_noise;
        for (int j = 0; j < pc.nt; ++j) {
            const int t = taus[pc.j0 + j];
            const int tn = (t + 1) % T, tp = (t - 1 + T) % T;
            a.G[j] = G_t[t];
            a.s[j] = s_t[t];
            if (n_ops > 1) {
                a.Gn[j] = G_t[tn];
                a.Gp[j] = G_t[tp];
                a.U[j] = U_t[t];
                a.Up[j] = U_t[tp];
            }
        }
        InsertionArgs al = a;
        al.op_lo = 0;
        al.op_cnt = 1;
        ProjGrid pl = pg;
        pl.n_per_share = n_noise;
        if (int rc = to_status(launch_fac_insertion(f64, false, 1, pl, al, st), "projection launch")) return rc;
        if (n_ops == 5) {
            InsertionArgs ad = a;
            ad.op_lo = 1;
            ad.op_cnt = 4;
            ProjGrid pd = pg;
            pd.n_per_share = n_noise * 4;
            if (int rc = to_status(launch_fac_insertion(f64, false, 2, pd, ad, st), "projection launch")) return rc;
        }
        ReduceArgs ra;
        ra.partial = part;
        ra.f64 = f64 ? 1 : 0;
        fill_phase(ra.ph, geom, +1, k, mg);
        ra.out = (double2*)out;
        ra.n_chunks = pc.n_chunks;
        ra.n_colblocks = ncb;
        ra.n_groups = ncb;
        ra.group_cols = kBlockCols;
        ra.n_mom_grp = mg.n;
        ra.n_mom_total = n_mom;
        ra.m_off = mg.off;
        ra.inner = pc.nt * n_ops;
        ra.outer_stride = n_tau * n_ops;
        ra.off = pc.j0 * n_ops;
        if (int rc = to_status(launch_reduce(ra, st), "reduction launch")) return rc;
    }
    return ok();
}

int c3pt_combine(const void* spec, int spec_spin, const void* ins, int n_noise, int n_p, int n_q,
                 int n_tau, int n_ops, int op_begin, int op_end, const double* w, const int* pairs,
                 int n_pairs, void* out, void* stream) {
    return combine_impl(spec, spec_spin, ins, n_noise, n_p, n_q, n_tau, 0, n_tau, n_ops, op_begin, op_end, w, pairs,
                        n_pairs, out, stream);
}

int c3pt_two_sink_meson(const c3pt_geom* geom, const void* G_fwd, const void* eta_fwd, int t_fwd,
                        const void* G_bwd, const void* eta_bwd, int t_bwd, int t_src, int n_noise,
                        const void* const* G_t, const void* const* s_t, const void* const* U_t, int n_ops,
                        const int* k, int n_mom, const double* w, const int* pairs, int n_pairs, void* spec,
                        void* ins, void* out_fwd, void* out_bwd) {
    // every check of the composed calls first: on error nothing is enqueued
    if (int rc = check_geom(geom)) return rc;
    if (int rc = check_momenta(k, n_mom)) return rc;
    if (!G_fwd || !eta_fwd || !G_bwd || !eta_bwd || !G_t || !s_t || !spec || !ins || !out_fwd || !out_bwd)
        return fail(C3PT_EINVAL, "NULL field, table or output pointer");
    if (n_noise < 1) return fail(C3PT_EINVAL, "n_noise = %d < 1", n_noise);
    if (n_ops != 1 && n_ops != 5 && n_ops != 9) return fail(C3PT_EINVAL, "n_ops = %d (must be 1, 5 or 9)", n_ops);
    if (n_ops > 1 && !U_t) return fail(C3PT_EINVAL, "derivative operators need gauge links");
    const int T = geom->T;
    if (t_fwd < 0 || t_fwd >= T || t_src < 0 || t_src >= T || t_bwd < 0 || t_bwd >= T)
        return fail(C3PT_EINVAL, "timeslices (%d, %d, %d) outside [0, %d)", t_fwd, t_src, t_bwd, T);
    const int d1 = (t_src - t_fwd + T) % T, d2 = (t_bwd - t_src + T) % T;
    if (d1 + d2 >= T) return fail(C3PT_EINVAL, "the two sinks overlap around the periodic time direction");
    const int n_span = d1 + d2 + 1;
    std::vector<int> taus(n_span);
    for (int j = 0; j < n_span; ++j) {
        const int t = (t_fwd + j) % T;
        taus[j] = t;
        if (!G_t[t]) return fail(C3PT_EINVAL, "propagator slice %d missing", t);
        if (!s_t[t]) return fail(C3PT_EINVAL, "stochastic solution slice %d missing", t);
        if (n_ops > 1) {
            const int tn = (t + 1) % T, tp = (t - 1 + T) % T;
            if (!G_t[tn] || !G_t[tp])
                return fail(C3PT_EINVAL, "propagator slices %d and %d needed around %d", tp, tn, t);
            if (!U_t[t] || !U_t[tp]) return fail(C3PT_EINVAL, "link slices %d and %d needed", tp, t);
            if (n_ops == 9 && (!s_t[tn] || !s_t[tp]))
                return fail(C3PT_EINVAL, "stochastic solution slices %d and %d needed around %d", tp, tn, t);
        }
    }
    if (n_ops == 9) {
        if (int rc = check_symmetric(geom, k, n_mom)) return rc;
    }
    if (pairs) {
        if (n_pairs < 1) return fail(C3PT_EINVAL, "n_pairs = %d < 1", n_pairs);
        for (int j = 0; j < n_pairs; ++j)
            if (pairs[2 * j] < 0 || pairs[2 * j] >= n_mom || pairs[2 * j + 1] < 0 || pairs[2 * j + 1] >= n_mom)
                return fail(C3PT_EINVAL, "pair %d = (%d, %d) out of range", j, pairs[2 * j], pairs[2 * j + 1]);
    } else if (n_pairs != n_mom * n_mom) {
        return fail(C3PT_EINVAL, "n_pairs must be n_mom*n_mom when pairs is NULL");
    }
    // spectators at both sinks, one insertion over the whole span, two windowed combines
    char* spec_bwd = (char*)spec + (size_t)n_noise * n_mom * kBlockCols * sizeof(double2);
    if (int rc = c3pt_spectator_meson(geom, G_fwd, eta_fwd, n_noise, k, n_mom, spec)) return rc;
    if (int rc = c3pt_spectator_meson(geom, G_bwd, eta_bwd, n_noise, k, n_mom, spec_bwd)) return rc;
    if (int rc = c3pt_insertion(geom, G_t, s_t, n_noise, taus.data(), n_span, U_t, n_ops, k, n_mom, ins)) return rc;
    if (int rc = combine_impl(spec, 64, ins, n_noise, n_mom, n_mom, n_span, 0, d1 + 1, n_ops, 0, n_ops, w, pairs,
                              n_pairs, out_fwd, geom->stream))
        return rc;
    if (int rc = combine_impl(spec_bwd, 64, ins, n_noise, n_mom, n_mom, n_span, d1, d2 + 1, n_ops, 0, n_ops, w, pairs,
                              n_pairs, out_bwd, geom->stream))
        return rc;
    return ok();
}


int c3pt_gamma_meson(const void* C, int n_blk, const double* g_snk, int n_snk, const double* g_ins, int n_ins,
                     const double* g_src, int n_src, void* out, void* stream) {
    if (!C || !out) return fail(C3PT_EINVAL, "NULL data or output pointer");
    if (n_blk < 1) return fail(C3PT_EINVAL, "n_blk = %d < 1", n_blk);
    const int n[3] = {n_snk, n_ins, n_src};
    const double* m[3] = {g_snk, g_ins, g_src};
    for (int s = 0; s < 3; ++s) {
        if (n[s] < 1 || n[s] > 16) return fail(C3PT_EINVAL, "matrix count %d outside [1, 16]", n[s]);
        if (!m[s] && n[s] != 16) return fail(C3PT_EINVAL, "the default matrix lists hold 16 matrices");
    }
    std::vector<double2> mats(3 * 256, make_double2(0.0, 0.0));
    for (int s = 0; s < 3; ++s) {
        if (m[s])
            memcpy(mats.data() + 256 * s, m[s], (size_t)n[s] * 16 * sizeof(double2));
        else
            c3pt::gamma_default_matrices(s, mats.data() + 256 * s);
    }
    hipStream_t st = (hipStream_t)stream;
    void* base;
    if (int rc = scratch_dev(st, mats.size() * sizeof(double2), &base)) return rc;
    if (int rc = upload(st, base, 0, mats.data(), mats.size() * sizeof(double2))) return rc;
    GammaMesonArgs a;
    a.C = (const double2*)C;
    a.mats = (const double2*)base;
    a.out = (double2*)out;
    a.n_blk = n_blk;
    a.n_snk = n_snk;
    a.n_ins = n_ins;
    a.n_src = n_src;
    if (int rc = to_status(timed("gamma_meson", st, [&] { return launch_gamma_meson(a, st); }), "gamma launch"))
        return rc;
    return ok();
}

int c3pt_gamma_nucleon(const void* C, int n_blk, int channel, const double* A, const double* Abar,
                       const double* P, int n_proj, const double* g_ins, int n_ins, void* out, void* stream) {
    if (!C || !out) return fail(C3PT_EINVAL, "NULL data or output pointer");
    if (n_blk < 1) return fail(C3PT_EINVAL, "n_blk = %d < 1", n_blk);
    if (channel != C3PT_PROTON_D && channel != C3PT_PROTON_U) return fail(C3PT_EINVAL, "unknown channel %d", channel);
    if (n_proj < 1 || n_proj > kMaxNucProj) return fail(C3PT_EINVAL, "n_proj = %d outside [1, 16]", n_proj);
    if (!P && n_proj != 2) return fail(C3PT_EINVAL, "the default projectors are two");
    if (n_ins < 1 || n_ins > 16) return fail(C3PT_EINVAL, "n_ins = %d outside [1, 16]", n_ins);
    if (!g_ins && n_ins != 16) return fail(C3PT_EINVAL, "the default insertion list holds 16 matrices");
    std::vector<int> rows;
    std::vector<double2> w;
    c3pt::nucleon_weights(channel == C3PT_PROTON_D ? 0 : 1, A, Abar, P, n_proj, &rows, &w);
    std::vector<double2> gi(256, make_double2(0.0, 0.0));
    if (g_ins)
        memcpy(gi.data(), g_ins, (size_t)n_ins * 16 * sizeof(double2));
    else
        c3pt::gamma_default_matrices(1, gi.data());
    // device table: Gins, rows, weights (256-byte aligned pieces)
    const size_t gbytes = gi.size() * sizeof(double2);
    const size_t roff = (gbytes + 255) & ~(size_t)255;
    const size_t rbytes = std::max<size_t>(rows.size(), 1) * sizeof(int);
    const size_t woff = (roff + rbytes + 255) & ~(size_t)255;
    const size_t wbytes = w.size() * sizeof(double2);
    std::vector<char> host(woff + wbytes);
    memcpy(host.data(), gi.data(), gbytes);
    if (!rows.empty()) memcpy(host.data() + roff, rows.data(), rows.size() * sizeof(int));
    if (wbytes) memcpy(host.data() + woff, w.data(), wbytes);
    hipStream_t st = (hipStream_t)stream;
    void* base;
    if (int rc = scratch_dev(st, host.size() + 256, &base)) return rc;
    if (int rc = upload(st, base, 0, host.data(), host.size())) return rc;
    GammaNucleonArgs a;
    a.C = (const double2*)C;
    a.gins = (const double2*)base;
    a.rows = (const int*)((char*)base + roff);
    a.w = (const double2*)((char*)base + woff);
    a.out = (double2*)out;
    a.n_blk = n_blk;
    a.n_rows = (int)rows.size();
    a.n_proj = n_proj;
    a.n_ins = n_ins;
    if (int rc = to_status(timed("gamma_nucleon", st, [&] { return launch_gamma_nucleon(a, st); }), "gamma launch"))
        return rc;
    return ok();
}

int c3pt_smear(const c3pt_geom* geom, const void* in, void* out, int n_outer, int n_inner, const void* U,
               double kappa, int n_iter) {
    if (int rc = check_geom(geom)) return rc;
    if (!in || !out || !U) return fail(C3PT_EINVAL, "NULL field or link pointer");
    if (n_outer < 1 || n_inner < 1) return fail(C3PT_EINVAL, "n_outer = %d, n_inner = %d (must be >= 1)", n_outer,
                                                n_inner);
    if (n_iter < 0) return fail(C3PT_EINVAL, "n_iter = %d < 0", n_iter);
    if (!(kappa >= 0.0) || !(kappa < 1e6)) return fail(C3PT_EINVAL, "kappa = %g outside [0, 1e6)", kappa);
    const long long V3 = (long long)geom->L[0] * geom->L[1] * geom->L[2];
    const long long n_val = (long long)n_outer * 3 * n_inner * V3;
    if (n_val > 0xffffffffLL) return fail(C3PT_EINVAL, "field of %lld values exceeds 32-bit indexing", n_val);
    const bool f64 = geom->dtype == C3PT_C128;
    const size_t bytes = (size_t)n_val * (f64 ? sizeof(double2) : sizeof(float2));
    hipStream_t st = (hipStream_t)geom->stream;
    if (n_iter == 0) {
        if (in != out && hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return fail(C3PT_EDEVICE, "field copy failed");
        return ok();
    }
    void* tmp;
    if (int rc = scratch_dev(st, bytes, &tmp)) return rc;
    SmearArgs a;
    for (int j = 0; j < 3; ++j) a.L[j] = geom->L[j];
    a.V3 = (int)V3;
    a.U = U;
    a.n_outer = n_outer;
    a.n_inner = n_inner;
    a.norm = 1.0 / (1.0 + 6.0 * kappa);
    a.kappa_norm = kappa / (1.0 + 6.0 * kappa);
    // step i writes the buffer that is not its input; the last step writes out
    // unless the input is out itself, then the result is copied at the end
    const void* src = in;
    for (int i = 1; i <= n_iter; ++i) {
        void* dst = ((n_iter - i) % 2 == 0) ? out : tmp;
        if (dst == src) dst = (dst == out) ? tmp : out;
        a.in = src;
        a.out = dst;
        if (int rc = to_status(timed("smear", st, [&] { return launch_smear(f64, a, st); }), "smear launch"))
            return rc;
        src = dst;
    }
    if (src != out && hipMemcpyAsync(out, src, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(C3PT_EDEVICE, "field copy failed");
    return ok();
}

}  // extern "C"
