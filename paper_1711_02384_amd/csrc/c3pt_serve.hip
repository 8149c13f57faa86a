// Serving engine: continuous batching of contraction requests on one GPU.
//
// A request is one measurement of Eq. (8) on one lattice and source: the
// spectator part (meson, or the two nucleon spectators) at t_f, the insertion
// part at every tau from t_src to t_f, and the noise-weighted combines.  The
// paper runs such measurements as MPI jobs over many nodes (Sec. 2.2-2.3);
// here many of them share one GPU.
//
//  * Admission by memory: each request's outputs (and its small parameter
//    tables, factor plans, dense phase tables) are sub-allocated first-fit
//    from an arena of caller-provided device memory; requests are admitted
//    while a slot (max_active) and arena space are free, the one with the
//    least work first (with a bound on how often the first in line is passed).
//  * Packets: an admitted request is cut into packets -- a block of noise
//    vectors of a spectator, a block of timeslices (or of timeslices x noise
//    vectors) of an insertion -- whose FP32 partial sums fit a fixed share of
//    the step workspace.
//  * Steps: every step takes packets from the active requests with the least
//    remaining work first (one left out for four steps goes first), each as
//    many as fit, until the workspace (or, while no request waits for
//    admission, the step work cap) is full, runs them through one launch per producer kind
//    (dense: and momentum-tile class; factored: and tile length), reduces
//    the partial sums in FP64 into the requests' outputs, and enqueues the
//    combines of every request whose last packet ran in the step, followed by
//    an event that marks the request complete.  Requests arriving while
//    others run join at the next step: their work shares the same launches.
//
// A request's results do not depend on the other requests: every output
// element is summed over the same fixed site chunks and reduced in the same
// order whatever the packet or step it ran in.
#include <string.h>

#include <algorithm>
#include <array>
#include <deque>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "../../include/c3pt.h"
#include "c3pt_internal.h"

namespace c3pt {
int api_fail(int code, const char* msg);
int api_ok();
int api_variant(int kind, int mode, int mt);
bool api_profiling();
hipError_t api_timed(const char* name, hipStream_t st, const std::function<hipError_t()>& fn);
}  // namespace c3pt

using namespace c3pt;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
  public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t m = 0;
        for (auto& f : free_) m = std::max(m, f.second);
        return m;
    }

  private:
    std::map<size_t, size_t> free_;
};

struct Packet {
    int kind;     // 0 meson spectator, 1 baryon spectator, 2 insertion
    int part;     // output index (nucleon: spectator (u,u) / (u,d); insertion u / d)
    int n0, nn;   // noise vectors [n0, n0 + nn)
    int t0, nt;   // insertion timeslices [t0, t0 + nt) of the request's list
};

enum ReqState { kQueued, kActive, kDone, kFailed };

struct Request {
    long long id;
    int kind;          // C3PT_REQ_MESON / C3PT_REQ_NUCLEON
    int L[3], T, r[3], V3;
    int t_f, n_noise, n_ops, n_mom, n_pairs;
    std::vector<int> taus, k, pairs;
    std::vector<const void*> G, G2, s, U;
    const void* eta;
    int n_chunks, chunk_sites;
    // arena
    size_t off = 0, bytes = 0;
    size_t o_spec[2], o_ins[2], o_comb[2], o_k, o_pairs, o_w;
    size_t o_plan[2] = {0, 0};   // factored: FactorPlan for sigma = -1 (spectators), +1 (insertions)
    std::vector<int> tab_key[2];  // dense: phase tables held while active (sigma = -1, +1)
    size_t spec_elems, ins_elems, comb_elems;
    int n_parts;
    char* pinned = nullptr;   // host copy of k | pairs | w, uploaded asynchronously at admission
    size_t pinned_bytes = 0;
    // progress
    std::deque<Packet> todo;
    bool combines_enqueued = false;
    hipEvent_t done = nullptr;
    ReqState state = kQueued;
    int error = 0;                // status of a request that failed at admission, and its message
    std::string error_msg;
    double work = 0;              // all packets: column blocks x sites
    int bypassed = 0;             // admissions that passed it while it was first in line
    int idle_steps = 0;           // steps since it last had a packet in one
};

// A dense phase table in the arena, shared by the requests that use it.
struct PhaseEntry {
    size_t off = 0, bytes = 0;
    int refs = 0;                 // active requests holding it
    long long last_use = 0;
};

}  // namespace

struct c3pt_server {
    int device = 0;
    hipStream_t st = nullptr;
    int proj = 0, mode = kModeF32;
    bool fac = false;          // factored projection
    int max_active = 1;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    Arena alloc;
    size_t step_bytes = 0, packet_cap = 0;
    double step_work = 0;      // cap on a step's work (column blocks x sites); 0: none
    void* partial = nullptr;
    // step parameters: one device block, two pinned staging blocks
    size_t params_cap = 0;
    char* dparams = nullptr;
    char* staging[2] = {nullptr, nullptr};
    hipEvent_t staged[2] = {nullptr, nullptr};
    bool staged_used[2] = {false, false};
    int step_no = 0;
    int* counters = nullptr;   // device [kMaxLaunches]
    std::map<std::vector<int>, PhaseEntry> phase;   // dense: (L, sigma, mode, mtmax, k...) -> table in the arena
    long long clock = 0;
    std::deque<Request*> queue;
    std::vector<Request*> active;
    std::map<long long, Request*> all;
    long long next_id = 1;
    int n_cu = 256;
};

namespace {

constexpr int kMaxLaunches = 32;
constexpr int kMaxStepJobs = 4096;
constexpr size_t kMaxStepItems = (size_t)1 << 20;
constexpr int kMaxStepTau = 1 << 16;
constexpr int kServeMaxChunks = 16;   // factored: x3-plane chunks per request at most

int spin_of(const Request& q) { return q.kind == C3PT_REQ_MESON ? 64 : 1024; }

size_t packet_partial(const Request& q, const Packet& p) {
    const size_t per_cb = (size_t)q.n_chunks * q.n_mom * kBlockCols * sizeof(float2);
    if (p.kind == 2) return per_cb * p.nn * p.nt * q.n_ops;
    return per_cb * p.nn * (p.kind == 1 ? 16 : 1);
}

// Largest packet of a request: a quarter of the step workspace, and at most
// half the item capacity of a step.
size_t request_cap(const Request& q, size_t packet_cap) {
    return std::min(packet_cap, kMaxStepItems / 2 * (size_t)q.n_mom * kBlockCols * sizeof(float2));
}

// Packets of a request, each within the packet cap (the caller checks that
// one noise vector of one timeslice fits) and, when work_cap > 0, within
// work_cap column blocks x sites where a packet of one noise vector (of one
// timeslice) allows it.
void make_packets(Request& q, size_t packet_cap, double work_cap) {
    const size_t cap = request_cap(q, packet_cap);
    const size_t per_cb = (size_t)q.n_chunks * q.n_mom * kBlockCols * sizeof(float2);
    const int n_tau = (int)q.taus.size();
    const int spec_kind = q.kind == C3PT_REQ_MESON ? 0 : 1;
    const int spec_cb = spec_kind == 1 ? 16 : 1;
    auto by_work = [&](double per_unit) {
        return work_cap > 0 ? std::max(1.0, std::floor(work_cap / per_unit)) : 1e9;
    };
    const int nn_spec = std::max<int>(
        1, (int)std::min<double>({(double)q.n_noise, (double)(cap / (per_cb * spec_cb)), by_work((double)spec_cb * q.V3)}));
    for (int part = 0; part < q.n_parts; ++part)
        for (int n0 = 0; n0 < q.n_noise; n0 += nn_spec)
            q.todo.push_back(Packet{spec_kind, part, n0, std::min(nn_spec, q.n_noise - n0), 0, 0});
    const size_t per_tau = per_cb * q.n_noise * q.n_ops;
    const double work_tau = (double)q.n_noise * q.n_ops * q.V3;
    for (int part = 0; part < q.n_parts; ++part) {
        if (per_tau <= cap && by_work(work_tau) >= 1.0 && (work_cap <= 0 || work_tau <= work_cap)) {
            const int nt = std::max<int>(1, (int)std::min<double>({(double)n_tau, (double)(cap / per_tau), by_work(work_tau)}));
            for (int t0 = 0; t0 < n_tau; t0 += nt)
                q.todo.push_back(Packet{2, part, 0, q.n_noise, t0, std::min(nt, n_tau - t0)});
        } else {
            const int nn = std::max<int>(
                1, (int)std::min<double>((double)(cap / (per_cb * q.n_ops)), by_work((double)q.n_ops * q.V3)));
            for (int t0 = 0; t0 < n_tau; ++t0)
                for (int n0 = 0; n0 < q.n_noise; n0 += nn)
                    q.todo.push_back(Packet{2, part, n0, std::min(nn, q.n_noise - n0), t0, 1});
        }
    }
}

int mtmax_of(int n_mom) {
    const int mt = (n_mom + 7) / 8;
    return mt <= 4 ? 4 : mt <= 8 ? 8 : mt <= 12 ? 12 : 16;
}

// Work of a packet for scheduling: column blocks x sites.
double packet_work(const Request& q, const Packet& p) {
    const double cbs = p.kind == 2 ? (double)p.nn * p.nt * q.n_ops : (double)p.nn * (p.kind == 1 ? 16 : 1);
    return cbs * q.V3;
}

std::vector<int> phase_key(const c3pt_server* sv, const Request& q, int sigma) {
    std::vector<int> key = {q.L[0], q.L[1], q.L[2], sigma, sv->mode, mtmax_of(q.n_mom)};
    key.insert(key.end(), q.k.begin(), q.k.end());
    return key;
}

size_t phase_bytes(const c3pt_server* sv, const Request& q) {
    return align_up(phase_table_bytes(sv->mode, q.V3, mtmax_of(q.n_mom)));
}

// Arena allocation that evicts cached phase tables no active request holds
// (least recently used first) until the block fits; false if it cannot fit
// with every such table gone.
bool arena_alloc(c3pt_server* sv, size_t bytes, size_t* off) {
    while (!sv->alloc.alloc(bytes, off)) {
        auto victim = sv->phase.end();
        for (auto e = sv->phase.begin(); e != sv->phase.end(); ++e)
            if (e->second.refs == 0 && (victim == sv->phase.end() || e->second.last_use < victim->second.last_use))
                victim = e;
        if (victim == sv->phase.end()) return false;
        sv->alloc.release(victim->second.off, victim->second.bytes);
        sv->phase.erase(victim);
    }
    return true;
}

// Dense modes: hold the phase table for (extents, sign, momentum list),
// building it in the arena at first use (on the server stream, before the
// request's packets).  Tables no active request holds stay cached and are
// evicted, least recently used first, when the arena needs their space.
// Returns C3PT_OK, 1 when the arena has no room now, or a negative status.
int hold_phase(c3pt_server* sv, Request& q, int sigma) {
    std::vector<int> key = phase_key(sv, q, sigma);
    auto it = sv->phase.find(key);
    if (it == sv->phase.end()) {
        const size_t bytes = phase_bytes(sv, q);
        size_t off;
        if (!arena_alloc(sv, bytes, &off)) return 1;
        PhaseSpec ph;
        memset(&ph, 0, sizeof(ph));
        for (int j = 0; j < 3; ++j) ph.L[j] = q.L[j];
        ph.sigma = sigma;
        ph.n_mom = q.n_mom;
        for (int m = 0; m < q.n_mom; ++m)
            for (int j = 0; j < 3; ++j) ph.k[j][m] = (uint8_t)(((q.k[3 * m + j] % q.L[j]) + q.L[j]) % q.L[j]);
        if (launch_phase_table(sv->mode, ph, q.V3, mtmax_of(q.n_mom), sv->arena + off, sv->st) != hipSuccess) {
            sv->alloc.release(off, bytes);
            return api_fail(C3PT_EDEVICE, "building a phase table failed");
        }
        PhaseEntry e;
        e.off = off;
        e.bytes = bytes;
        it = sv->phase.emplace(key, e).first;
    }
    it->second.refs += 1;
    it->second.last_use = ++sv->clock;
    q.tab_key[sigma > 0 ? 1 : 0] = key;
    return C3PT_OK;
}

void drop_phases(c3pt_server* sv, Request& q) {
    for (auto& key : q.tab_key) {
        if (key.empty()) continue;
        auto it = sv->phase.find(key);
        if (it != sv->phase.end() && it->second.refs > 0) it->second.refs -= 1;
        key.clear();
    }
}

// Device address of the request's phase data for sign sigma: its own factor
// plan (factored) or the held table (dense).
const void* phase_of(const c3pt_server* sv, const Request& q, int sigma) {
    if (sv->fac) return sv->arena + q.off + q.o_plan[sigma > 0 ? 1 : 0];
    return sv->arena + sv->phase.at(q.tab_key[sigma > 0 ? 1 : 0]).off;
}

// Arena layout of a request's outputs and parameter tables (factored: and its
// two factor plans, uploaded with the parameters).
size_t layout(Request& q, bool fac) {
    const int n_tau = (int)q.taus.size();
    const int spin = spin_of(q);
    q.spec_elems = (size_t)q.n_noise * q.n_mom * spin * 3;
    q.ins_elems = (size_t)q.n_noise * n_tau * q.n_ops * q.n_mom * kBlockCols;
    q.comb_elems = (size_t)q.n_pairs * n_tau * q.n_ops * spin * 64;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes);
        return at;
    };
    for (int p = 0; p < q.n_parts; ++p) q.o_spec[p] = take(q.spec_elems * 16);
    for (int p = 0; p < q.n_parts; ++p) q.o_ins[p] = take(q.ins_elems * 16);
    for (int p = 0; p < q.n_parts; ++p) q.o_comb[p] = take(q.comb_elems * 16);
    q.o_k = take(q.k.size() * sizeof(int));
    q.o_pairs = take(q.pairs.size() * sizeof(int));
    q.o_w = take((size_t)q.n_noise * sizeof(double));
    if (fac) {
        q.o_plan[0] = take(sizeof(FactorPlan));
        q.o_plan[1] = take(sizeof(FactorPlan));
    }
    return o;
}

void destroy_request(Request* q) {
    if (q->done) hipEventDestroy(q->done);
    if (q->pinned) hipHostFree(q->pinned);
    delete q;
}

// True when some admitted request (running, or done and not yet released)
// holds arena space that will be returned.
bool arena_held(const c3pt_server* sv) {
    for (const auto& kv : sv->all)
        if (kv.second->state == kActive || kv.second->state == kDone) return true;
    return false;
}

// A request that cannot be admitted for a reason of its own leaves the queue
// as failed; poll and result report its status.
void fail_queued(c3pt_server* sv, Request* q, int rc) {
    q->state = kFailed;
    q->error = rc;
    q->error_msg = c3pt_last_error();
    sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), q));
}

// Admission while a slot is free: the queued request with the least work
// first, except that the one first in line is taken in turn once later ones
// have passed it 2 * max_active times.  Outputs (and dense phase tables)
// must fit the arena; when the chosen request does not fit now, admission
// stops until space is released.
int admit(c3pt_server* sv) {
    while (!sv->queue.empty() && (int)sv->active.size() < sv->max_active) {
        Request* head = sv->queue.front();
        Request* q = head;
        if (head->bypassed < 2 * sv->max_active)
            for (Request* c : sv->queue)
                if (c->work < q->work) q = c;
        size_t off;
        if (!arena_alloc(sv, q->bytes, &off)) {
            if (!arena_held(sv)) {
                // nothing will release space: the request can never fit
                fail_queued(sv, q, api_fail(C3PT_ENOMEM, "the request's outputs do not fit the arena"));
                continue;
            }
            break;
        }
        q->off = off;
        char* base = sv->arena + off;
        if (!sv->fac) {
            int rc = hold_phase(sv, *q, -1);
            if (rc == C3PT_OK) rc = hold_phase(sv, *q, +1);
            if (rc != C3PT_OK) {
                drop_phases(sv, *q);
                sv->alloc.release(off, q->bytes);
                if (rc < 0) {
                    fail_queued(sv, q, rc);
                    continue;
                }
                if (!arena_held(sv)) {
                    // nothing will release space: the request can never fit
                    fail_queued(sv, q, api_fail(C3PT_ENOMEM, "outputs and phase tables exceed the arena"));
                    continue;
                }
                break;
            }
        }
        // parameter tables (and factor plans) of the request, stream-ordered before its packets
        if (hipMemcpyAsync(base + q->o_k, q->pinned, q->pinned_bytes, hipMemcpyHostToDevice, sv->st) != hipSuccess) {
            drop_phases(sv, *q);
            sv->alloc.release(off, q->bytes);
            return api_fail(C3PT_EDEVICE, "uploading request parameters failed");
        }
        make_packets(*q, sv->packet_cap, sv->step_work / 4);
        q->state = kActive;
        if (q != head) head->bypassed += 1;
        sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), q));
        sv->active.push_back(q);
    }
    return C3PT_OK;
}

// Device job of one packet; tau pointer rows are appended to `taus`.
BatchJob packet_job(c3pt_server* sv, const Request& q, const Packet& p, std::vector<const void*>& taus,
                    size_t tau_dev_off) {
    BatchJob d;
    memset(&d, 0, sizeof(d));
    d.kind = p.kind;
    d.V3 = q.V3;
    for (int j = 0; j < 3; ++j) {
        d.L[j] = q.L[j];
        d.r[j] = q.r[j];
    }
    d.n_noise = p.nn;
    d.n_mom = q.n_mom;
    d.k = (const int*)(sv->arena + q.off + q.o_k);
    d.n_chunks = q.n_chunks;
    d.chunk_sites = q.chunk_sites;
    const size_t noise_bytes = (size_t)12 * q.V3 * sizeof(float2);
    const void* tab = nullptr;
    if (p.kind == 2) {
        d.sigma = +1;
        d.n_tau = p.nt;
        d.n_ops = q.n_ops;
        d.n_colblocks = p.nn * p.nt * q.n_ops;
        d.group_cols = kBlockCols;
        const int n_tau = (int)q.taus.size();
        d.out_inner = p.nt * q.n_ops;
        d.out_stride = n_tau * q.n_ops;
        d.out_off = (p.n0 * n_tau + p.t0) * q.n_ops;
        d.out = (double2*)(sv->arena + q.off + q.o_ins[p.part]);
        const std::vector<const void*>& Gv = p.part == 0 ? q.G : q.G2;
        d.tau_ptrs = (const void* const*)(sv->dparams + tau_dev_off + taus.size() * sizeof(void*));
        for (int tl = 0; tl < p.nt; ++tl) {
            const int tau = q.taus[p.t0 + tl];
            const int tn = (tau + 1) % q.T, tp = (tau - 1 + q.T) % q.T;
            taus.push_back(Gv[tau]);
            taus.push_back(q.n_ops == 5 ? Gv[tn] : nullptr);
            taus.push_back(q.n_ops == 5 ? Gv[tp] : nullptr);
            taus.push_back((const char*)q.s[tau] + (size_t)p.n0 * noise_bytes);
            taus.push_back(q.n_ops == 5 ? q.U[tau] : nullptr);
            taus.push_back(q.n_ops == 5 ? q.U[tp] : nullptr);
        }
    } else {
        d.sigma = -1;
        d.n_tau = 1;
        d.n_ops = 1;
        d.G = q.G[q.t_f];
        d.G2 = p.kind == 1 ? (p.part == 0 ? q.G[q.t_f] : q.G2[q.t_f]) : nullptr;
        d.eta = (const char*)q.eta + (size_t)p.n0 * noise_bytes;
        d.n_colblocks = p.nn * (p.kind == 1 ? 16 : 1);
        d.group_cols = p.kind == 1 ? 3072 : kBlockCols;
        d.out_inner = p.nn;
        d.out_stride = 0;
        d.out_off = p.n0;
        d.out = (double2*)(sv->arena + q.off + q.o_spec[p.part]);
    }
    tab = phase_of(sv, q, d.sigma);   // held since admission
    d.phase = tab;
    return d;
}

// One step: choose packets, upload their parameters, enqueue the work.
int step(c3pt_server* sv, int* n_done_enqueued) {
    *n_done_enqueued = 0;
    if (int rc = admit(sv)) return rc;
    if (sv->active.empty()) return C3PT_OK;

    // ---- choose packets under the workspace budget ----
    // Requests with the least remaining work first, each taking as many of
    // its packets as fit, so short requests finish in few steps; a request
    // that has had no packet for four steps goes first.
    struct Chosen {
        Request* q;
        Packet p;
        size_t bytes;
    };
    std::vector<Chosen> chosen;
    size_t used = 0, items = 0, tau_rows = 0;
    double work = 0;
    // The work cap holds while no request waits for admission: it bounds how
    // long a new arrival waits for the steps in flight.  With requests
    // waiting, steps fill the workspace (throughput first).
    const bool capped = sv->step_work > 0 && sv->queue.empty();
    std::vector<std::pair<double, Request*>> order;
    for (Request* q : sv->active) {
        if (q->todo.empty()) continue;
        double rem = 0;
        for (const Packet& p : q->todo) rem += packet_work(*q, p);
        order.push_back({q->idle_steps >= 4 ? -1.0 / (1 + q->idle_steps) : rem, q});
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<double, Request*>& a, const std::pair<double, Request*>& b) {
                         return a.first < b.first;
                     });
    for (auto& oq : order) {
        Request* q = oq.second;
        bool took = false;
        while (!q->todo.empty()) {
            const Packet& p = q->todo.front();
            const size_t b = packet_partial(*q, p);
            const size_t it = b / ((size_t)q->n_mom * kBlockCols * sizeof(float2));
            const size_t tr = p.kind == 2 ? (size_t)p.nt : 0;
            const double wk = packet_work(*q, p);
            if (!chosen.empty() && (used + b > sv->step_bytes || items + it > kMaxStepItems ||
                                    tau_rows + tr > (size_t)kMaxStepTau || chosen.size() >= (size_t)kMaxStepJobs ||
                                    (capped && work + wk > sv->step_work)))
                break;
            chosen.push_back({q, p, b});
            used += b;
            work += wk;
            items += it;
            tau_rows += tr;
            q->todo.pop_front();
            took = true;
        }
        q->idle_steps = took ? 0 : q->idle_steps + 1;
    }

    // ---- parameter block: jobs | items | tau rows | output offsets ----
    size_t n_tau_rows = 0;
    for (auto& c : chosen)
        if (c.p.kind == 2) n_tau_rows += (size_t)c.p.nt * 6;
    const size_t o_jobs = 0;
    const size_t o_items = align_up(o_jobs + chosen.size() * sizeof(BatchJob));
    const size_t o_taus = align_up(o_items + items * sizeof(int4));
    const size_t o_offs = align_up(o_taus + n_tau_rows * sizeof(void*));
    const size_t total = align_up(o_offs + (chosen.size() + 1) * sizeof(long long));
    if (total > sv->params_cap) return api_fail(C3PT_EUNSUPPORTED, "step parameters exceed their buffer");
    const int slot = sv->step_no & 1;
    if (sv->staged_used[slot] && hipEventSynchronize(sv->staged[slot]) != hipSuccess)
        return api_fail(C3PT_EDEVICE, "waiting for the staging buffer failed");
    char* h = sv->staging[slot];
    BatchJob* hj = (BatchJob*)(h + o_jobs);
    int4* hi = (int4*)(h + o_items);
    long long* ho = (long long*)(h + o_offs);
    std::vector<const void*> taus;
    taus.reserve(n_tau_rows);
    // Launch groups.  Dense: (producer kind, momentum-tile class).  Factored:
    // (queue kind, 32-site tiles) with queue kinds 0 meson, 1 baryon,
    // 2 insertion local operator, 3 insertion derivative operators.
    std::map<std::pair<int, int>, std::vector<int4>> lists;
    std::map<std::pair<int, int>, int> list_mt;
    size_t part_off = 0;
    for (size_t ci = 0; ci < chosen.size(); ++ci) {
        Chosen& c = chosen[ci];
        const int ji = (int)ci;
        BatchJob d = packet_job(sv, *c.q, c.p, taus, o_taus);
        d.partial = (char*)sv->partial + part_off;
        part_off += c.bytes;
        hj[ji] = d;
        const int mt = (c.q->n_mom + 7) / 8;
        const int n_share = d.kind == 2 ? d.n_tau : 1;
        const int n_within = d.n_colblocks / n_share;
        const int n_item_chunks = d.n_chunks;
        for (int sh = 0; sh < n_share; ++sh)
            for (int ch = 0; ch < n_item_chunks; ++ch)
                for (int w = 0; w < n_within; ++w) {
                    const int op = d.kind == 2 ? w % d.n_ops : 0;
                    const int cb = d.kind == 2 ? ((w / d.n_ops) * d.n_tau + sh) * d.n_ops + op : w;
                    std::pair<int, int> key;
                    if (sv->fac) {
                        const int qk = d.kind < 2 ? d.kind : (op == 0 ? 2 : 3);
                        const int fv = api_variant(d.kind, kModeBatchFacVariants, mt);
                        const bool t32 = (fv & kBatchFacKT32) && batch_fac_allows32(qk) && d.L[0] % 32 == 0;
                        key = {qk, t32 ? 1 : 0};
                    } else {
                        key = {d.kind, mt_class(mt)};
                    }
                    lists[key].push_back(make_int4(ji, cb, ch, 0));
                    int& lm = list_mt[key];
                    lm = std::max(lm, mt);
                }
    }
    if (lists.size() > (size_t)kMaxLaunches) return api_fail(C3PT_EUNSUPPORTED, "too many launch groups");
    size_t n_items = 0;
    struct Launch {
        int kind, mt;
        size_t item0, n;
        int variant;
    };
    std::vector<Launch> launches;
    for (auto& kv : lists) {
        const size_t item0 = n_items;
        for (const int4& it4 : kv.second) hi[n_items++] = it4;
        const int kind = kv.first.first;
        const int mt = list_mt[kv.first];
        const int variant =
            sv->fac ? (kv.first.second ? kBatchFacKT32 : 0) : api_variant(kind, sv->mode, mt);
        launches.push_back({kind, mt, item0, n_items - item0, variant});
    }
    std::vector<int> job_order(chosen.size());
    for (size_t ci = 0; ci < chosen.size(); ++ci) job_order[ci] = (int)ci;
    memcpy(h + o_taus, taus.data(), taus.size() * sizeof(void*));
    ho[0] = 0;
    for (size_t j = 0; j < job_order.size(); ++j) {
        const BatchJob& d = hj[j];
        ho[j + 1] = ho[j] + (long long)d.n_colblocks * d.n_mom * kBlockCols;
    }

    // ---- enqueue ----
    hipStream_t st = sv->st;
    if (hipMemcpyAsync(sv->dparams, h, total, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(sv->staged[slot], st) != hipSuccess)
        return api_fail(C3PT_EDEVICE, "uploading step parameters failed");
    sv->staged_used[slot] = true;
    ++sv->step_no;
    const BatchJob* JD = (const BatchJob*)(sv->dparams + o_jobs);
    const int4* ID = (const int4*)(sv->dparams + o_items);
    auto run = [&](const char* name, const std::function<hipError_t()>& fn) {
        return api_timed(name, st, fn) == hipSuccess;
    };
    bool okk = run("serve_reset", [&] { return launch_reset(sv->counters, (int)launches.size(), st); });
    static const char* kName[3] = {"serve_proj_spectator_meson", "serve_proj_spectator_baryon",
                                   "serve_proj_insertion"};
    static const char* kFacName[4] = {"serve_fac_spectator_meson", "serve_fac_spectator_baryon",
                                      "serve_fac_insertion", "serve_fac_insertion_deriv"};
    for (size_t li = 0; li < launches.size() && okk; ++li) {
        const Launch& L = launches[li];
        BatchGrid bg;
        bg.jobs = JD;
        bg.items = ID + L.item0;
        bg.n_items = (int)L.n;
        bg.counter = sv->counters + li;
        hipError_t e = hipSuccess;
        int per_cu;
        if (sv->fac)
            per_cu = L.kind == 0   ? batch_fac_meson(L.variant, nullptr, st, &e)
                     : L.kind == 1 ? batch_fac_baryon(L.variant, nullptr, st, &e)
                                   : batch_fac_insertion(L.variant, L.kind == 2 ? 1 : 2, nullptr, st, &e);
        else
            per_cu = L.kind == 0   ? batch_meson(sv->mode, L.mt, L.variant, nullptr, 0, st, &e)
                     : L.kind == 1 ? batch_baryon(sv->mode, L.mt, L.variant, nullptr, 0, st, &e)
                                   : batch_insertion(sv->mode, L.mt, L.variant, nullptr, 0, st, &e);
        const int n_wg = (int)std::max<long long>(1, std::min<long long>((long long)L.n, (long long)per_cu * sv->n_cu));
        okk = run(sv->fac ? kFacName[L.kind] : kName[L.kind], [&] {
            hipError_t e2 = hipSuccess;
            if (sv->fac) {
                if (L.kind == 0) batch_fac_meson(L.variant, &bg, st, &e2);
                else if (L.kind == 1) batch_fac_baryon(L.variant, &bg, st, &e2);
                else batch_fac_insertion(L.variant, L.kind == 2 ? 1 : 2, &bg, st, &e2);
            } else if (L.kind == 0) {
                batch_meson(sv->mode, L.mt, L.variant, &bg, n_wg, st, &e2);
            } else if (L.kind == 1) {
                batch_baryon(sv->mode, L.mt, L.variant, &bg, n_wg, st, &e2);
            } else {
                batch_insertion(sv->mode, L.mt, L.variant, &bg, n_wg, st, &e2);
            }
            return e2;
        });
    }
    if (okk) {
        BatchReduceArgs ra;
        ra.jobs = JD;
        ra.out_offset = (const long long*)(sv->dparams + o_offs);
        ra.n_jobs = (int)job_order.size();
        const long long tot = ho[job_order.size()];
        okk = run("serve_reduce", [&] { return launch_batch_reduce(ra, tot, st); });
    }
    // combines and completion of every request whose last packet ran
    for (Request* q : sv->active) {
        if (!okk) break;
        if (!q->todo.empty() || q->combines_enqueued) continue;
        bool in_step = false;
        for (auto& c : chosen) in_step |= c.q == q;
        if (!in_step) continue;
        char* base = sv->arena + q->off;
        for (int part = 0; part < q->n_parts && okk; ++part) {
            CombineArgs a;
            // meson: S x I; nucleon (proton isovector): (u,u) x I_d and (u,d) x I_u
            const int ip = q->n_parts == 2 ? 1 - part : 0;
            a.S = (const double2*)(base + q->o_spec[part]);
            a.I = (const double2*)(base + q->o_ins[ip]);
            a.w = (const double*)(base + q->o_w);
            a.pairs = (const int*)(base + q->o_pairs);
            a.out = (double2*)(base + q->o_comb[part]);
            a.n_noise = q->n_noise;
            a.n_p = q->n_mom;
            a.n_q = q->n_mom;
            a.n_tau = (int)q->taus.size();
            a.n_ops = q->n_ops;
            a.op_begin = 0;
            a.n_sel = q->n_ops;
            a.spin = spin_of(*q);
            a.n_pairs = q->n_pairs;
            okk = run("combine", [&] { return launch_combine(a, st); });
        }
        if (okk) {
            okk = hipEventRecord(q->done, st) == hipSuccess;
            q->combines_enqueued = true;
            ++*n_done_enqueued;
        }
    }
    if (!okk) return api_fail(C3PT_EDEVICE, "a serving launch failed");
    // requests whose combines are enqueued leave the active set (they keep
    // their arena space until released)
    std::vector<Request*> still;
    for (Request* q : sv->active) {
        if (q->combines_enqueued) {
            q->state = kDone;
            drop_phases(sv, *q);   // its launches are enqueued; the tables stay cached
        } else {
            still.push_back(q);
        }
    }
    sv->active.swap(still);
    return C3PT_OK;
}

void free_server(c3pt_server* sv) {
    if (!sv) return;
    for (auto& kv : sv->all) destroy_request(kv.second);
    for (int i = 0; i < 2; ++i) {
        if (sv->staging[i]) hipHostFree(sv->staging[i]);
        if (sv->staged[i]) hipEventDestroy(sv->staged[i]);
    }
    if (sv->dparams) hipFree(sv->dparams);
    if (sv->partial) hipFree(sv->partial);
    if (sv->counters) hipFree(sv->counters);
    delete sv;
}

}  // namespace

extern "C" {

int c3pt_server_create(int proj, void* arena, unsigned long long arena_bytes, unsigned long long step_bytes,
                       int max_active, void* stream, c3pt_server** out) {
    if (!out) return api_fail(C3PT_EINVAL, "out is NULL");
    *out = nullptr;
    if (proj != C3PT_PROJ_NATIVE && proj != C3PT_PROJ_SPLIT_F16 && proj != C3PT_PROJ_SPLIT_BF16 &&
        proj != C3PT_PROJ_FACTORED)
        return api_fail(C3PT_EINVAL, "unknown projection mode");
    if (!arena || arena_bytes < kAlign || ((uintptr_t)arena % kAlign) != 0)
        return api_fail(C3PT_EINVAL, "the arena must be device memory of at least 256 bytes, 256-byte aligned");
    if (step_bytes < ((size_t)1 << 20)) return api_fail(C3PT_EINVAL, "step workspace below 1 MiB");
    if (max_active < 1) return api_fail(C3PT_EINVAL, "max_active < 1");
    c3pt_server* sv = new c3pt_server();
    hipGetDevice(&sv->device);
    hipDeviceGetAttribute(&sv->n_cu, hipDeviceAttributeMultiprocessorCount, sv->device);
    sv->st = (hipStream_t)stream;
    sv->proj = proj;
    sv->mode = proj == C3PT_PROJ_SPLIT_BF16 ? kModeSplitBF16 : proj == C3PT_PROJ_SPLIT_F16 ? kModeSplitF16 : kModeF32;
    sv->fac = proj == C3PT_PROJ_FACTORED;
    sv->max_active = max_active;
    sv->arena = (char*)arena;
    sv->arena_bytes = arena_bytes;
    sv->alloc.init(arena_bytes);
    sv->step_bytes = step_bytes;
    sv->packet_cap = step_bytes / 4;
    sv->params_cap = align_up((size_t)kMaxStepJobs * sizeof(BatchJob)) + align_up(kMaxStepItems * sizeof(int4)) +
                     align_up((size_t)kMaxStepTau * 6 * sizeof(void*)) +
                     align_up(((size_t)kMaxStepJobs + 1) * sizeof(long long));
    bool okk = hipMalloc(&sv->partial, step_bytes) == hipSuccess &&
               hipMalloc((void**)&sv->dparams, sv->params_cap) == hipSuccess &&
               hipMalloc((void**)&sv->counters, kMaxLaunches * sizeof(int)) == hipSuccess;
    for (int i = 0; i < 2 && okk; ++i)
        okk = hipHostMalloc((void**)&sv->staging[i], sv->params_cap, hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&sv->staged[i], hipEventDisableTiming) == hipSuccess;
    if (!okk) {
        (void)hipGetLastError();
        free_server(sv);
        return api_fail(C3PT_ENOMEM, "server workspace allocation failed");
    }
    *out = sv;
    return api_ok();
}

int c3pt_server_submit(c3pt_server* sv, const c3pt_request* R, long long* id) {
    if (!sv || !R || !id) return api_fail(C3PT_EINVAL, "NULL argument");
    *id = 0;
    if (R->kind != C3PT_REQ_MESON && R->kind != C3PT_REQ_NUCLEON) return api_fail(C3PT_EINVAL, "unknown request kind");
    for (int j = 0; j < 3; ++j)
        if (R->L[j] < 1 || R->L[j] > C3PT_MAX_L) return api_fail(C3PT_EINVAL, "bad extent");
    if (R->T < 1 || R->t_src < 0 || R->t_src >= R->T || R->t_f < 0 || R->t_f >= R->T)
        return api_fail(C3PT_EINVAL, "bad T, t_src or t_f");
    if (R->n_noise < 1 || (R->n_ops != 1 && R->n_ops != 5)) return api_fail(C3PT_EINVAL, "bad n_noise or n_ops");
    if (!R->k || R->n_mom < 1 || R->n_mom > kMaxMomGroupF32) return api_fail(C3PT_EINVAL, "requests take 1..128 momenta");
    if (!R->G_t || !R->s_t || !R->eta || (R->kind == C3PT_REQ_NUCLEON && !R->G2_t) || (R->n_ops == 5 && !R->U_t))
        return api_fail(C3PT_EINVAL, "missing input table");
    if (R->pairs && R->n_pairs < 1) return api_fail(C3PT_EINVAL, "n_pairs < 1");
    Request* q = new Request();
    q->kind = R->kind;
    q->T = R->T;
    for (int j = 0; j < 3; ++j) {
        q->L[j] = R->L[j];
        q->r[j] = ((R->r[j] % R->L[j]) + R->L[j]) % R->L[j];
    }
    q->V3 = q->L[0] * q->L[1] * q->L[2];
    q->t_f = R->t_f;
    q->n_noise = R->n_noise;
    q->n_ops = R->n_ops;
    q->n_mom = R->n_mom;
    q->n_parts = R->kind == C3PT_REQ_NUCLEON ? 2 : 1;
    for (int t = R->t_src;; t = (t + 1) % R->T) {
        q->taus.push_back(t);
        if (t == R->t_f) break;
    }
    q->k.assign(R->k, R->k + 3 * R->n_mom);
    if (R->pairs) {
        q->n_pairs = R->n_pairs;
        q->pairs.assign(R->pairs, R->pairs + 2 * R->n_pairs);
    } else {
        q->n_pairs = R->n_mom * R->n_mom;
        for (int p = 0; p < R->n_mom; ++p)
            for (int qq = 0; qq < R->n_mom; ++qq) {
                q->pairs.push_back(p);
                q->pairs.push_back(qq);
            }
    }
    auto reject = [&](const char* msg) {
        delete q;
        return api_fail(C3PT_EINVAL, msg);
    };
    for (int m = 0; m < 3 * R->n_mom; ++m)
        if (R->k[m] < -(1 << 20) || R->k[m] > (1 << 20)) return reject("momentum component out of range");
    for (int v : q->pairs)
        if (v < 0 || v >= R->n_mom) return reject("pair index out of range");
    q->G.assign(R->G_t, R->G_t + R->T);
    if (R->G2_t) q->G2.assign(R->G2_t, R->G2_t + R->T);
    q->s.assign(R->s_t, R->s_t + R->T);
    if (R->n_ops == 5) q->U.assign(R->U_t, R->U_t + R->T);
    q->eta = R->eta;
    // required slices
    if (!q->G[q->t_f] || (q->n_parts == 2 && !q->G2[q->t_f])) return reject("missing propagator slice at t_f");
    for (int tau : q->taus) {
        const int tn = (tau + 1) % q->T, tp = (tau - 1 + q->T) % q->T;
        if (!q->G[tau] || !q->s[tau]) return reject("missing slice on the insertion range");
        if (q->n_parts == 2 && !q->G2[tau]) return reject("missing d-propagator slice");
        if (q->n_ops == 5 && (!q->G[tn] || !q->G[tp] || !q->U[tau] || !q->U[tp] ||
                              (q->n_parts == 2 && (!q->G2[tn] || !q->G2[tp]))))
            return reject("missing neighbour slice for the derivative operators");
    }
    FactorPlan plans[2];
    if (sv->fac) {
        if (!api_factor_plan(q->L, -1, q->k.data(), q->n_mom, &plans[0]) ||
            !api_factor_plan(q->L, +1, q->k.data(), q->n_mom, &plans[1]))
            return reject("the momentum list does not factor (too many distinct k1 or (k1, k2))");
        // chunks of about 2048 or 4096 sites: the insertion's tuned variant (its
        // work dominates a request) sets them for every part of the request
        // and at most kServeMaxChunks chunks, so that large lattices keep their
        // partial sums (and packets) small
        q->chunk_sites = std::max(batch_fac_chunk_planes(q->L, api_variant(2, kModeBatchFacVariants, (q->n_mom + 7) / 8)),
                                  (q->L[2] + kServeMaxChunks - 1) / kServeMaxChunks);
        q->n_chunks = (q->L[2] + q->chunk_sites - 1) / q->chunk_sites;
    } else {
        q->n_chunks = (q->V3 + kMaxSitesPerChunkF32 - 1) / kMaxSitesPerChunkF32;
        const int tiles = (q->V3 + kSiteTile - 1) / kSiteTile;
        q->chunk_sites = (tiles + q->n_chunks - 1) / q->n_chunks * kSiteTile;
        q->n_chunks = (q->V3 + q->chunk_sites - 1) / q->chunk_sites;
    }
    q->bytes = layout(*q, sv->fac);
    if (q->bytes + (sv->fac ? 0 : 2 * phase_bytes(sv, *q)) > sv->arena_bytes)
        return reject("the request's outputs (and phase tables) exceed the arena");
    const size_t per_cb = (size_t)q->n_chunks * q->n_mom * kBlockCols * sizeof(float2);
    const size_t cap = request_cap(*q, sv->packet_cap);
    if (per_cb * q->n_ops > cap || per_cb * (q->kind == C3PT_REQ_NUCLEON ? 16 : 1) > cap)
        return reject("one noise vector of this request exceeds the step workspace");
    if (q->taus.size() * 6 > (size_t)kMaxStepTau) return reject("too many timeslices");
    if (hipEventCreateWithFlags(&q->done, hipEventDisableTiming) != hipSuccess) {
        destroy_request(q);
        return api_fail(C3PT_EDEVICE, "event creation failed");
    }
    q->pinned_bytes = sv->fac ? q->o_plan[1] + sizeof(FactorPlan) - q->o_k
                              : q->o_w - q->o_k + (size_t)q->n_noise * sizeof(double);
    if (hipHostMalloc((void**)&q->pinned, q->pinned_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        q->pinned = nullptr;
        destroy_request(q);
        return api_fail(C3PT_ENOMEM, "pinned parameter buffer allocation failed");
    }
    memcpy(q->pinned, q->k.data(), q->k.size() * sizeof(int));
    memcpy(q->pinned + (q->o_pairs - q->o_k), q->pairs.data(), q->pairs.size() * sizeof(int));
    double* w = (double*)(q->pinned + (q->o_w - q->o_k));
    for (int i = 0; i < q->n_noise; ++i) w[i] = 1.0 / q->n_noise;
    if (sv->fac)
        for (int sg = 0; sg < 2; ++sg) memcpy(q->pinned + (q->o_plan[sg] - q->o_k), &plans[sg], sizeof(FactorPlan));
    make_packets(*q, sv->packet_cap, 0);
    for (const Packet& pk : q->todo) q->work += packet_work(*q, pk);
    q->todo.clear();
    q->id = sv->next_id++;
    sv->all[q->id] = q;
    sv->queue.push_back(q);
    *id = q->id;
    return api_ok();
}

int c3pt_server_set_step_work(c3pt_server* sv, double max_work) {
    if (!sv) return api_fail(C3PT_EINVAL, "server is NULL");
    if (!(max_work >= 0)) return api_fail(C3PT_EINVAL, "max_work must be >= 0");
    sv->step_work = max_work;
    return api_ok();
}

int c3pt_server_step(c3pt_server* sv, int* n_active, int* n_queued) {
    if (!sv) return api_fail(C3PT_EINVAL, "server is NULL");
    int done = 0;
    if (int rc = step(sv, &done)) return rc;
    if (n_active) *n_active = (int)sv->active.size();
    if (n_queued) *n_queued = (int)sv->queue.size();
    return api_ok();
}

int c3pt_server_poll(c3pt_server* sv, long long id) {
    if (!sv) return api_fail(C3PT_EINVAL, "server is NULL");
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return api_fail(C3PT_EINVAL, "unknown request id");
    Request* q = it->second;
    if (q->state == kFailed) return api_fail(q->error, q->error_msg.c_str());
    if (q->state != kDone) return 0;
    const hipError_t e = hipEventQuery(q->done);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return api_fail(C3PT_EDEVICE, "event query failed");
}

int c3pt_server_result(c3pt_server* sv, long long id, c3pt_result* res) {
    if (!sv || !res) return api_fail(C3PT_EINVAL, "NULL argument");
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return api_fail(C3PT_EINVAL, "unknown request id");
    Request* q = it->second;
    if (q->state == kQueued) return api_fail(C3PT_EINVAL, "request not admitted yet");
    if (q->state == kFailed) return api_fail(q->error, q->error_msg.c_str());
    memset(res, 0, sizeof(*res));
    char* base = sv->arena + q->off;
    for (int p = 0; p < q->n_parts; ++p) {
        res->spec[p] = base + q->o_spec[p];
        res->ins[p] = base + q->o_ins[p];
        res->comb[p] = base + q->o_comb[p];
    }
    res->n_parts = q->n_parts;
    res->n_tau = (int)q->taus.size();
    res->n_pairs = q->n_pairs;
    return api_ok();
}

int c3pt_server_release(c3pt_server* sv, long long id) {
    if (!sv) return api_fail(C3PT_EINVAL, "server is NULL");
    auto it = sv->all.find(id);
    if (it == sv->all.end()) return api_fail(C3PT_EINVAL, "unknown request id");
    Request* q = it->second;
    if (q->state == kActive) return api_fail(C3PT_EINVAL, "request still running");
    if (q->state == kDone) {
        if (hipEventSynchronize(q->done) != hipSuccess) return api_fail(C3PT_EDEVICE, "event sync failed");
        sv->alloc.release(q->off, q->bytes);
    } else if (q->state == kQueued) {
        sv->queue.erase(std::find(sv->queue.begin(), sv->queue.end(), q));
    }
    sv->all.erase(it);
    destroy_request(q);
    return api_ok();
}

int c3pt_server_info(const c3pt_server* sv, int* n_active, int* n_queued, unsigned long long* arena_free_largest) {
    if (!sv) return api_fail(C3PT_EINVAL, "server is NULL");
    if (n_active) *n_active = (int)sv->active.size();
    if (n_queued) *n_queued = (int)sv->queue.size();
    if (arena_free_largest) *arena_free_largest = sv->alloc.largest();
    return api_ok();
}

int c3pt_server_destroy(c3pt_server* sv) {
    if (!sv) return C3PT_OK;
    if (sv->st) hipStreamSynchronize(sv->st);
    else hipDeviceSynchronize();
    free_server(sv);
    return C3PT_OK;
}

}  // extern "C"
