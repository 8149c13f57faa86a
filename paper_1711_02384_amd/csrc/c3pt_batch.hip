// Batches: many spectator / insertion calls over uneven lattices, executed as
// one HIP graph whose projection work runs over lists of (job, column block,
// chunk) items: one workgroup per item for the factored kernels, persistent
// workgroups taking items from a queue for the dense ones.  This is how the
// many source positions of a measurement are handled on one GPU (the paper
// distributes them over MPI ranks, Sec. 2.2-2.3): jobs of different lattice
// sizes share a launch, so the chip stays loaded until the last item.
//
// Schedule (recorded once into a graph at creation):
//   for each group of jobs whose partial sums fit the budget:
//     reset the queue counters (a kernel, not a memset node)
//     one projection launch per producer kind present in the group (factored:
//     and per tile length)
//     batched FP64 reduction of the group's partial sums (source factors applied)
//   combines of (spectator job, insertion job) pairs
#include <string.h>

#include <algorithm>
#include <array>
#include <functional>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/c3pt.h"
#include "c3pt_internal.h"

namespace c3pt {
// from c3pt_api.hip
int api_fail(int code, const char* msg);
int api_ok();
int api_variant(int kind, int mode, int mt);
bool api_profiling();
hipError_t api_timed(const char* name, hipStream_t st, const std::function<hipError_t()>& fn);
}  // namespace c3pt

using namespace c3pt;

struct c3pt_batch {
    // The schedule: every launch of one replay, in order.  Recorded into the
    // graph at creation; run one by one (each timed) while profiling is on.
    struct Op {
        const char* name;
        std::function<hipError_t(hipStream_t)> launch;
    };
    std::vector<Op> ops;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void*> allocations;
    int n_items = 0, n_groups = 0;
    size_t partial_bytes = 0;
    int device = 0;
};

namespace {

struct HostJob {
    BatchJob d;
    int index;
    double cost;
    size_t partial_bytes;
    long long out_elems;
};

int dmalloc(c3pt_batch* b, void** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return api_fail(C3PT_ENOMEM, "batch allocation failed");
    }
    b->allocations.push_back(*p);
    return C3PT_OK;
}

int upload_sync(void* dst, const void* src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return C3PT_OK;
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return api_fail(C3PT_EDEVICE, "batch upload failed");
    return C3PT_OK;
}

void destroy(c3pt_batch* b) {
    if (!b) return;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    for (void* p : b->allocations) hipFree(p);
    delete b;
}

}  // namespace

extern "C" {

int c3pt_batch_create(const c3pt_job* jobs, int n_jobs, const c3pt_combine_job* combines, int n_combines,
                      const int* k, int n_mom, int proj, unsigned long long partial_budget, c3pt_batch** out) {
    if (!out) return api_fail(C3PT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!jobs || n_jobs < 1) return api_fail(C3PT_EINVAL, "empty job list");
    if (n_combines < 0 || (n_combines > 0 && !combines)) return api_fail(C3PT_EINVAL, "bad combine list");
    if (!k || n_mom < 1 || n_mom > kMaxMomGroupF32)
        return api_fail(C3PT_EINVAL, "batches take 1..128 momenta");
    if (proj != C3PT_PROJ_NATIVE && proj != C3PT_PROJ_SPLIT_F16 && proj != C3PT_PROJ_SPLIT_BF16 &&
        proj != C3PT_PROJ_FACTORED)
        return api_fail(C3PT_EINVAL, "unknown projection mode");
    const bool fac = proj == C3PT_PROJ_FACTORED;
    for (int m = 0; m < 3 * n_mom; ++m)
        if (k[m] < -32768 || k[m] > 32767) return api_fail(C3PT_EINVAL, "momentum component outside [-32768, 32767]");
    const int mode = proj == C3PT_PROJ_SPLIT_BF16 ? kModeSplitBF16 : proj == C3PT_PROJ_SPLIT_F16 ? kModeSplitF16 : kModeF32;
    const int mt = (n_mom + 7) / 8;
    const int mtmax = mt <= 4 ? 4 : mt <= 8 ? 8 : mt <= 12 ? 12 : 16;
    if (partial_budget == 0) partial_budget = (unsigned long long)16 << 30;

    // ---- validate and describe the jobs (host side, nothing enqueued yet) ----
    std::vector<HostJob> hj(n_jobs);
    for (int i = 0; i < n_jobs; ++i) {
        const c3pt_job& J = jobs[i];
        if (J.kind < C3PT_JOB_SPECTATOR_MESON || J.kind > C3PT_JOB_INSERTION)
            return api_fail(C3PT_EINVAL, ("job " + std::to_string(i) + ": unknown kind").c_str());
        for (int j = 0; j < 3; ++j)
            if (J.L[j] < 1 || J.L[j] > C3PT_MAX_L)
                return api_fail(C3PT_EINVAL, ("job " + std::to_string(i) + ": bad extent").c_str());
        if (J.T < 1 || J.n_noise < 1 || !J.out)
            return api_fail(C3PT_EINVAL, ("job " + std::to_string(i) + ": bad T, n_noise or out").c_str());
        BatchJob d;
        memset(&d, 0, sizeof(d));
        d.kind = J.kind;
        for (int j = 0; j < 3; ++j) {
            d.L[j] = J.L[j];
            d.r[j] = ((J.r[j] % J.L[j]) + J.L[j]) % J.L[j];
        }
        d.V3 = J.L[0] * J.L[1] * J.L[2];
        d.n_noise = J.n_noise;
        d.out = (double2*)J.out;
        if (J.kind == C3PT_JOB_INSERTION) {
            if (!J.G_t || !J.s_t || !J.taus || J.n_tau < 1 || (J.n_ops != 1 && J.n_ops != 5) ||
                (J.n_ops == 5 && !J.U_t))
                return api_fail(C3PT_EINVAL, ("job " + std::to_string(i) + ": bad insertion arguments").c_str());
            for (int t = 0; t < J.n_tau; ++t) {
                const int tau = J.taus[t];
                if (tau < 0 || tau >= J.T || !J.G_t[tau] || !J.s_t[tau])
                    return api_fail(C3PT_EINVAL, ("job " + std::to_string(i) + ": missing slice").c_str());
                if (J.n_ops == 5) {
                    const int tn = (tau + 1) % J.T, tp = (tau - 1 + J.T) % J.T;
                    if (!J.G_t[tn] || !J.G_t[tp] || !J.U_t[tau] || !J.U_t[tp])
                        return api_fail(C3PT_EINVAL, ("job " + std::to_string(i) + ": missing neighbour").c_str());
                }
            }
            d.sigma = +1;
            d.n_tau = J.n_tau;
            d.n_ops = J.n_ops;
            d.n_colblocks = J.n_noise * J.n_tau * J.n_ops;
            d.group_cols = kBlockCols;
        } else {
            if (!J.G || !J.eta || (J.kind == C3PT_JOB_SPECTATOR_BARYON && !J.G2))
                return api_fail(C3PT_EINVAL, ("job " + std::to_string(i) + ": missing spectator input").c_str());
            d.sigma = -1;
            d.n_tau = 1;
            d.n_ops = 1;
            d.G = J.G;
            d.G2 = J.G2;
            d.eta = J.eta;
            d.n_colblocks = J.kind == C3PT_JOB_SPECTATOR_MESON ? J.n_noise : 16 * J.n_noise;
            d.group_cols = J.kind == C3PT_JOB_SPECTATOR_MESON ? kBlockCols : 3072;
        }
        if (fac) {
            // chunks of x3 planes (about 2048 or 4096 sites, the kind's tuned variant)
            d.chunk_sites = batch_fac_chunk_planes(d.L, api_variant(d.kind, kModeBatchFacVariants, mt));
            d.n_chunks = (d.L[2] + d.chunk_sites - 1) / d.chunk_sites;
        } else {
            d.n_chunks = (d.V3 + kMaxSitesPerChunkF32 - 1) / kMaxSitesPerChunkF32;
            const int tiles = (d.V3 + kSiteTile - 1) / kSiteTile;
            d.chunk_sites = (tiles + d.n_chunks - 1) / d.n_chunks * kSiteTile;
            d.n_chunks = (d.V3 + d.chunk_sites - 1) / d.chunk_sites;
        }
        d.n_mom = n_mom;
        d.out_inner = d.n_colblocks / (d.group_cols / kBlockCols);   // output groups: identity map
        d.out_stride = d.out_inner;
        d.out_off = 0;
        hj[i].d = d;
        hj[i].index = i;
        hj[i].cost = (double)d.V3 * d.n_colblocks;
        hj[i].partial_bytes = (size_t)d.n_chunks * d.n_colblocks * n_mom * kBlockCols * sizeof(float2);
        hj[i].out_elems = (long long)d.n_colblocks / (d.group_cols / kBlockCols) * n_mom * d.group_cols;
        if (hj[i].partial_bytes > partial_budget)
            return api_fail(C3PT_EINVAL, ("job " + std::to_string(i) + ": partial sums exceed the budget").c_str());
    }
    for (int c = 0; c < n_combines; ++c) {
        const c3pt_combine_job& C = combines[c];
        if (C.spec_job < 0 || C.spec_job >= n_jobs || C.ins_job < 0 || C.ins_job >= n_jobs ||
            jobs[C.spec_job].kind == C3PT_JOB_INSERTION || jobs[C.ins_job].kind != C3PT_JOB_INSERTION ||
            jobs[C.spec_job].n_noise != jobs[C.ins_job].n_noise || !C.out ||
            C.op_begin < 0 || C.op_end > jobs[C.ins_job].n_ops || C.op_begin >= C.op_end ||
            (C.pairs && C.n_pairs < 1))
            return api_fail(C3PT_EINVAL, ("combine " + std::to_string(c) + ": bad arguments").c_str());
        if (C.pairs)
            for (int j = 0; j < 2 * C.n_pairs; ++j)
                if (C.pairs[j] < 0 || C.pairs[j] >= n_mom)
                    return api_fail(C3PT_EINVAL, ("combine " + std::to_string(c) + ": pair out of range").c_str());
    }

    c3pt_batch* b = new c3pt_batch();
    hipGetDevice(&b->device);
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return api_fail(C3PT_EDEVICE, "stream creation failed");
    }
    auto bail = [&](int rc) {
        hipStreamSynchronize(st);
        hipStreamDestroy(st);
        destroy(b);
        return rc;
    };

    // ---- phase tables (owned by the batch, one per (extents, sign)) and
    //      insertion pointer tables ----
    int* kdev;
    if (int rc = dmalloc(b, (void**)&kdev, (size_t)n_mom * 3 * sizeof(int))) return bail(rc);
    if (int rc = upload_sync(kdev, k, (size_t)n_mom * 3 * sizeof(int), st)) return bail(rc);
    std::map<std::array<int, 4>, const void*> tables;
    for (HostJob& h : hj) {
        h.d.k = kdev;
        BatchJob& d = h.d;
        const c3pt_job& J = jobs[h.index];
        const std::array<int, 4> key = {d.L[0], d.L[1], d.L[2], d.sigma};
        auto it = tables.find(key);
        if (it == tables.end() && fac) {
            FactorPlan plan;
            if (!api_factor_plan(d.L, d.sigma, k, n_mom, &plan))
                return bail(api_fail(C3PT_EUNSUPPORTED,
                                     "the momentum list has too many distinct k1 or (k1, k2) for the factored "
                                     "projection"));
            void* dp;
            if (int rc = dmalloc(b, &dp, sizeof(FactorPlan))) return bail(rc);
            if (int rc = upload_sync(dp, &plan, sizeof(FactorPlan), st)) return bail(rc);
            it = tables.emplace(key, dp).first;
        } else if (it == tables.end()) {
            PhaseSpec ph;
            memset(&ph, 0, sizeof(ph));
            for (int j = 0; j < 3; ++j) ph.L[j] = d.L[j];
            ph.sigma = d.sigma;
            ph.n_mom = n_mom;
            for (int m = 0; m < n_mom; ++m)
                for (int j = 0; j < 3; ++j) ph.k[j][m] = (uint8_t)(((k[3 * m + j] % d.L[j]) + d.L[j]) % d.L[j]);
            void* tab;
            if (int rc = dmalloc(b, &tab, phase_table_bytes(mode, d.V3, mtmax))) return bail(rc);
            if (launch_phase_table(mode, ph, d.V3, mtmax, tab, st) != hipSuccess)
                return bail(api_fail(C3PT_EDEVICE, "building a phase table failed"));
            it = tables.emplace(key, tab).first;
        }
        d.phase = it->second;
        if (J.kind == C3PT_JOB_INSERTION) {
            std::vector<const void*> tp((size_t)J.n_tau * 6, nullptr);
            for (int t = 0; t < J.n_tau; ++t) {
                const int tau = J.taus[t];
                const int tn = (tau + 1) % J.T, tpv = (tau - 1 + J.T) % J.T;
                tp[6 * t + 0] = J.G_t[tau];
                tp[6 * t + 3] = J.s_t[tau];
                if (J.n_ops == 5) {
                    tp[6 * t + 1] = J.G_t[tn];
                    tp[6 * t + 2] = J.G_t[tpv];
                    tp[6 * t + 4] = J.U_t[tau];
                    tp[6 * t + 5] = J.U_t[tpv];
                }
            }
            void* dev;
            if (int rc = dmalloc(b, &dev, tp.size() * sizeof(void*))) return bail(rc);
            if (int rc = upload_sync(dev, tp.data(), tp.size() * sizeof(void*), st)) return bail(rc);
            d.tau_ptrs = (const void* const*)dev;
        }
    }

    // ---- groups under the partial-sum budget, largest jobs first ----
    std::vector<int> order(n_jobs);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return hj[a].cost > hj[c].cost; });
    std::vector<std::vector<int>> groups;
    size_t acc = 0, max_group = 0;
    for (int i : order) {
        if (groups.empty() || acc + hj[i].partial_bytes > partial_budget) {
            groups.emplace_back();
            acc = 0;
        }
        groups.back().push_back(i);
        acc += hj[i].partial_bytes;
        max_group = std::max(max_group, acc);
    }
    void* partial;
    if (int rc = dmalloc(b, &partial, max_group)) return bail(rc);
    b->partial_bytes = max_group;
    b->n_groups = (int)groups.size();

    // device job table in group order; partial regions per group
    std::vector<BatchJob> djobs;
    std::vector<int> job_pos(n_jobs);
    for (auto& grp : groups) {
        size_t off = 0;
        for (int i : grp) {
            hj[i].d.partial = (char*)partial + off;
            off += hj[i].partial_bytes;
            job_pos[i] = (int)djobs.size();
            djobs.push_back(hj[i].d);
        }
    }
    void* djobs_dev;
    if (int rc = dmalloc(b, &djobs_dev, djobs.size() * sizeof(BatchJob))) return bail(rc);
    if (int rc = upload_sync(djobs_dev, djobs.data(), djobs.size() * sizeof(BatchJob), st)) return bail(rc);
    const BatchJob* JD = (const BatchJob*)djobs_dev;

    // queues: per group and kind, items (job, column block, chunk)
    struct Queue {
        int kind;
        int4* items;
        int n;
        int* counter;
        int variant, n_wg;
    };
    int n_cu = 256;
    hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, b->device);
    std::vector<std::vector<Queue>> queues(groups.size());
    std::vector<std::pair<long long*, long long>> out_offsets(groups.size());
    // queue kinds: 0 meson spectator, 1 baryon spectator, 2 insertion (factored:
    // local operator only), 3 factored insertion derivative operators; factored
    // queues split further into jobs on 16- and on 32-site tiles (slot
    // 2 * kind + t32) when the kind's variant asks for 32-site tiles
    constexpr int kQueueKinds = 4;
    constexpr int kQueueSlots = 2 * kQueueKinds;
    int* counters;
    if (int rc = dmalloc(b, (void**)&counters, groups.size() * kQueueSlots * sizeof(int))) return bail(rc);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        for (int qs = 0; qs < kQueueSlots; ++qs) {
            const int kind = qs / 2, t32 = qs % 2;
            if (kind == 3 && !fac) continue;
            if (t32 && !fac) continue;
            // factored variant of this queue: the producer kind's tuned choice,
            // with 32-site tiles for the jobs whose rows split into them
            const int fv = fac ? api_variant(std::min(kind, 2), kModeBatchFacVariants, mt) : 0;
            const bool want32 = fac && (fv & kBatchFacKT32) && batch_fac_allows32(kind);
            if (t32 && !want32) continue;
            // Issue order: largest job first; within a job, items that read the
            // same input slice and site chunk are adjacent, so they run together
            // and share its cache lines.
            std::vector<int4> items;
            for (int i : groups[gi]) {
                const BatchJob& d = hj[i].d;
                if (d.kind != std::min(kind, 2)) continue;
                if (kind == 3 && d.n_ops == 1) continue;
                if (fac && (want32 && d.L[0] % 32 == 0) != (t32 == 1)) continue;
                const int n_share = d.kind == 2 ? d.n_tau : 1;
                const int n_within = d.n_colblocks / n_share;
                const int n_item_chunks = d.n_chunks;
                for (int sh = 0; sh < n_share; ++sh)
                    for (int ch = 0; ch < n_item_chunks; ++ch)
                        for (int w = 0; w < n_within; ++w) {
                            const int op = d.kind == 2 ? w % d.n_ops : 0;
                            if (fac && d.kind == 2 && (op == 0) != (kind == 2)) continue;
                            const int cb = d.kind == 2 ? ((w / d.n_ops) * d.n_tau + sh) * d.n_ops + op : w;
                            items.push_back(make_int4(job_pos[i], cb, ch, 0));
                        }
            }
            if (items.empty()) continue;
            void* dev;
            if (int rc = dmalloc(b, &dev, items.size() * sizeof(int4))) return bail(rc);
            if (int rc = upload_sync(dev, items.data(), items.size() * sizeof(int4), st)) return bail(rc);
            // dense persistent grid: as many workgroups as fit on the chip at once
            // (the factored launch takes one workgroup per item)
            const int variant = fac ? (t32 ? kBatchFacKT32 : 0) : api_variant(kind, mode, mt);
            hipError_t e = hipSuccess;
            int per_cu;
            if (fac)
                per_cu = kind == 0   ? batch_fac_meson(variant, nullptr, st, &e)
                         : kind == 1 ? batch_fac_baryon(variant, nullptr, st, &e)
                                     : batch_fac_insertion(variant, kind == 2 ? 1 : 2, nullptr, st, &e);
            else
                per_cu = kind == 0   ? batch_meson(mode, mt, variant, nullptr, 0, st, &e)
                         : kind == 1 ? batch_baryon(mode, mt, variant, nullptr, 0, st, &e)
                                     : batch_insertion(mode, mt, variant, nullptr, 0, st, &e);
            if (e != hipSuccess || per_cu < 1) return bail(api_fail(C3PT_EUNSUPPORTED, "no kernel for this batch"));
            const int n_wg = std::max(1, (int)std::min<long long>((long long)items.size(), (long long)per_cu * n_cu));
            queues[gi].push_back(
                Queue{kind, (int4*)dev, (int)items.size(), counters + kQueueSlots * gi + qs, variant, n_wg});
            b->n_items += (int)items.size();
        }
        std::vector<long long> offs(1, 0);
        for (int i : groups[gi]) offs.push_back(offs.back() + hj[i].out_elems);
        void* dev;
        if (int rc = dmalloc(b, &dev, offs.size() * sizeof(long long))) return bail(rc);
        if (int rc = upload_sync(dev, offs.data(), offs.size() * sizeof(long long), st)) return bail(rc);
        out_offsets[gi] = {(long long*)dev, offs.back()};
    }

    // combine parameters
    std::vector<CombineArgs> cargs;
    for (int c = 0; c < n_combines; ++c) {
        const c3pt_combine_job& C = combines[c];
        const c3pt_job& JS = jobs[C.spec_job];
        const c3pt_job& JI = jobs[C.ins_job];
        const int N = JS.n_noise;
        std::vector<double> w(N);
        for (int i = 0; i < N; ++i) w[i] = C.w ? C.w[i] : 1.0 / N;
        void* wdev;
        if (int rc = dmalloc(b, &wdev, N * sizeof(double))) return bail(rc);
        if (int rc = upload_sync(wdev, w.data(), N * sizeof(double), st)) return bail(rc);
        void* pdev = nullptr;
        if (C.pairs) {
            if (int rc = dmalloc(b, &pdev, (size_t)C.n_pairs * 2 * sizeof(int))) return bail(rc);
            if (int rc = upload_sync(pdev, C.pairs, (size_t)C.n_pairs * 2 * sizeof(int), st)) return bail(rc);
        }
        CombineArgs a;
        a.S = (const double2*)JS.out;
        a.I = (const double2*)JI.out;
        a.w = (const double*)wdev;
        a.pairs = (const int*)pdev;
        a.out = (double2*)C.out;
        a.n_noise = N;
        a.n_p = n_mom;
        a.n_q = n_mom;
        a.n_tau = JI.n_tau;
        a.n_ops = JI.n_ops;
        a.op_begin = C.op_begin;
        a.n_sel = C.op_end - C.op_begin;
        a.spin = JS.kind == C3PT_JOB_SPECTATOR_MESON ? 64 : 1024;
        a.n_pairs = C.pairs ? C.n_pairs : n_mom * n_mom;
        cargs.push_back(a);
    }

    // ---- the schedule ----
    BatchReduceArgs rbase;
    memset(&rbase, 0, sizeof(rbase));
    int job_base = 0;
    static const char* kProjName[4] = {"batch_proj_spectator_meson", "batch_proj_spectator_baryon",
                                       "batch_proj_insertion", "batch_proj_insertion_deriv"};
    static const char* kFacName[4] = {"batch_fac_spectator_meson", "batch_fac_spectator_baryon",
                                      "batch_fac_insertion", "batch_fac_insertion_deriv"};
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        int* cnt = counters + kQueueSlots * gi;
        b->ops.push_back({"batch_reset", [cnt](hipStream_t s) { return launch_reset(cnt, kQueueSlots, s); }});
        for (const Queue& q : queues[gi]) {
            BatchGrid bg;
            bg.jobs = JD;
            bg.items = q.items;
            bg.n_items = q.n;
            bg.counter = q.counter;
            const int kind = q.kind, variant = q.variant, n_wg = q.n_wg;
            b->ops.push_back({fac ? kFacName[kind] : kProjName[kind], [=](hipStream_t s) {
                                  hipError_t e = hipSuccess;
                                  if (fac) {
                                      if (kind == 0) batch_fac_meson(variant, &bg, s, &e);
                                      else if (kind == 1) batch_fac_baryon(variant, &bg, s, &e);
                                      else batch_fac_insertion(variant, kind == 2 ? 1 : 2, &bg, s, &e);
                                  } else if (kind == 0) {
                                      batch_meson(mode, mt, variant, &bg, n_wg, s, &e);
                                  } else if (kind == 1) {
                                      batch_baryon(mode, mt, variant, &bg, n_wg, s, &e);
                                  } else {
                                      batch_insertion(mode, mt, variant, &bg, n_wg, s, &e);
                                  }
                                  return e;
                              }});
        }
        BatchReduceArgs ra = rbase;
        ra.jobs = JD + job_base;
        ra.out_offset = out_offsets[gi].first;
        ra.n_jobs = (int)groups[gi].size();
        const long long total = out_offsets[gi].second;
        b->ops.push_back({"batch_reduce", [ra, total](hipStream_t s) { return launch_batch_reduce(ra, total, s); }});
        job_base += (int)groups[gi].size();
    }
    for (const CombineArgs& a : cargs)
        b->ops.push_back({"combine", [a](hipStream_t s) { return launch_combine(a, s); }});

    // ---- record it into a graph ----
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bail(api_fail(C3PT_EDEVICE, "graph capture failed to start"));
    hipError_t cap = hipSuccess;
    for (const auto& op : b->ops) {
        cap = op.launch(st);
        if (cap != hipSuccess) break;
    }
    hipGraph_t graph = nullptr;
    hipError_t endc = hipStreamEndCapture(st, &graph);
    if (cap != hipSuccess || endc != hipSuccess || !graph) {
        if (graph) hipGraphDestroy(graph);
        return bail(api_fail(C3PT_EDEVICE, "recording the batch graph failed"));
    }
    b->graph = graph;
    if (hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0) != hipSuccess)
        return bail(api_fail(C3PT_EDEVICE, "graph instantiation failed"));
    hipStreamSynchronize(st);
    hipStreamDestroy(st);
    *out = b;
    return api_ok();
}

int c3pt_batch_run(c3pt_batch* b, void* stream) {
    if (!b || !b->exec) return api_fail(C3PT_EINVAL, "batch is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (api_profiling()) {
        for (const auto& op : b->ops)
            if (api_timed(op.name, st, [&] { return op.launch(st); }) != hipSuccess)
                return api_fail(C3PT_EDEVICE, "batch launch failed");
        return api_ok();
    }
    if (hipGraphLaunch(b->exec, st) != hipSuccess) return api_fail(C3PT_EDEVICE, "graph launch failed");
    return api_ok();
}

int c3pt_batch_info(const c3pt_batch* b, int* n_items, int* n_groups, unsigned long long* partial_bytes) {
    if (!b) return api_fail(C3PT_EINVAL, "batch is NULL");
    if (n_items) *n_items = b->n_items;
    if (n_groups) *n_groups = b->n_groups;
    if (partial_bytes) *partial_bytes = b->partial_bytes;
    return C3PT_OK;
}

int c3pt_batch_destroy(c3pt_batch* b) {
    if (!b) return C3PT_OK;
    hipDeviceSynchronize();
    destroy(b);
    return C3PT_OK;
}

}  // extern "C"
