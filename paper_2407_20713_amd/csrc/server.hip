// server.hip -- continuous batching of calibration requests (sabr_server_*).
//
// A worker thread admits queued requests into free slots of a device-resident
// slot table when their device footprint fits the memory budget (first fit in
// one arena), then replays one captured HIP graph per quantum: normalise the
// grids of new slots, advance every formula slot by Q temperature levels and
// every Monte Carlo slot by one iteration, and copy the slot states back.
// Finished slots release their memory and report their latency (completion
// minus submission, host steady clock).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../include/sabr.h"
#include "sabr_server_dev.h"

using namespace sabr;
using Clock = std::chrono::steady_clock;

namespace sabrhost {
int fail(sabr_ctx *c, int code, const char *fmt, ...);
int device_of(const sabr_ctx *c);
int base_npar(int model);
int n_steps(double T, int spy);
int check_request(sabr_ctx *c, const sabr_request &q);
}  // namespace sabrhost
using namespace sabrhost;

namespace {

struct Owned {   // deep copy of a submitted request
    uint64_t ticket = 0;
    Clock::time_point t_submit;
    std::vector<double> T, fwd, disc, K, target, lb, ub, x0;
    std::vector<int32_t> offs;
    sabr_request req;
    int kind = 0;
    size_t bytes = 0;
};

struct SlotHost {
    bool busy = false;
    uint64_t ticket = 0;
    Clock::time_point t_submit;
    size_t off = 0, bytes = 0;
    int n_par = 0;
    bool cancel = false;
};

struct Done {
    uint64_t ticket;
    sabr_result res;
    double latency_s;
};

// First-fit allocator over [0, size) with coalescing.
struct Arena {
    size_t size = 0;
    std::vector<std::pair<size_t, size_t>> free_;   // (offset, length), sorted
    void init(size_t n) {
        size = n;
        free_.assign(1, {0, n});
    }
    bool alloc(size_t n, size_t &off) {
        n = (n + 255) / 256 * 256;
        for (size_t i = 0; i < free_.size(); ++i)
            if (free_[i].second >= n) {
                off = free_[i].first;
                free_[i].first += n;
                free_[i].second -= n;
                if (free_[i].second == 0) free_.erase(free_.begin() + (long)i);
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n) {
        n = (n + 255) / 256 * 256;
        auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (size_t)0));
        it = free_.insert(it, {off, n});
        size_t i = (size_t)(it - free_.begin());
        if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
            free_[i].second += free_[i + 1].second;
            free_.erase(free_.begin() + (long)i + 1);
        }
        if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
            free_[i - 1].second += free_[i].second;
            free_.erase(free_.begin() + (long)i);
        }
    }
    size_t in_use() const {
        size_t f = 0;
        for (auto &b : free_) f += b.second;
        return size - f;
    }
};

// Layout of one request inside its arena block (offsets in bytes).
struct Layout {
    size_t total = 0;
    size_t take(size_t n) {
        const size_t o = total;
        total += (n + 255) / 256 * 256;
        return o;
    }
};

int slot_kind(const sabr_request &q) {
    if (q.obj.kind == SABR_OBJ_MC) return KIND_MC;
    return q.problem.model == SABR_STATIC ? KIND_STATIC : KIND_DYN_I;
}

}  // namespace

struct sabr_server {
    sabr_ctx *ctx = nullptr;
    int device = 0;
    int n_slots = 0, n_mc = 0, Q = 1;
    hipStream_t stream = nullptr;      // uploads, formula slots, status
    hipStream_t stream_mc = nullptr;   // Monte Carlo slots (overlap the formula slots)
    hipEvent_t ev_up = nullptr, ev_mc = nullptr;
    unsigned char *arena_dev = nullptr;
    Arena arena;
    SlotDev *d_slots = nullptr;
    SlotStatus *d_status = nullptr, *h_status = nullptr;
    unsigned char *stage = nullptr;   // pinned upload staging
    size_t stage_bytes = 0, stage_used = 0;
    std::vector<SlotHost> slots;
    hipGraph_t graph = nullptr, graph_mc = nullptr, graph_st = nullptr;
    hipGraphExec_t gexec = nullptr, gexec_mc = nullptr, gexec_st = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Owned *> queue;
    std::deque<Done> done;
    std::set<uint64_t> cancelled;
    std::thread worker;
    std::atomic<bool> stop{false};
    uint64_t next_ticket = 1;
    int32_t device_error = 0;
    std::string err;
    // statistics
    int64_t quanta = 0, admitted = 0, completed = 0;
    size_t peak_bytes = 0;
    int peak_active = 0;
};

namespace {

size_t footprint(const sabr_request &q, Layout *lay = nullptr, size_t *offs_out = nullptr) {
    Layout L;
    const int n_pts = q.market.offs[q.market.n_mat];
    const int n_mat = q.market.n_mat;
    const int NP = q.problem.n_par;
    const int P = q.sa.n_chains;
    const int levels = (q.sa.n_iters + q.sa.chain_len - 1) / q.sa.chain_len;
    size_t o[40];
    int k = 0;
    for (int i = 0; i < 9; ++i) o[k++] = L.take(sizeof(double) * n_pts);   // K lfk lkf P1 Z Q1 Q2 target sw
    o[k++] = L.take(sizeof(int32_t) * n_pts);                              // row
    for (int i = 0; i < 5; ++i) o[k++] = L.take(sizeof(double) * n_mat);   // T fwd lnf F1 disc
    o[k++] = L.take(sizeof(int32_t) * (n_mat + 1));                        // offs
    o[k++] = L.take(sizeof(double) * levels);                              // sched g
    o[k++] = L.take(sizeof(double) * levels);                              // sched h
    o[k++] = L.take(sizeof(double) * P * NP);                              // cx
    o[k++] = L.take(sizeof(double) * P);                                   // cf
    o[k++] = L.take(sizeof(double) * P * NP);                              // bx
    o[k++] = L.take(sizeof(double) * P);                                   // bf
    o[k++] = L.take(sizeof(unsigned long long) * P);                       // nacc
    if (q.obj.kind == SABR_OBJ_MC) {
        o[k++] = L.take(sizeof(McSaState));                                // mcst
        o[k++] = L.take(sizeof(double) * P * NP);                          // Y
        o[k++] = L.take(sizeof(double) * P);                               // fy
        o[k++] = L.take(sizeof(float) * (size_t)n_pts * kMcPBlocks * 64);  // part
        o[k++] = L.take(sizeof(int32_t) * n_mat);                          // msteps
        o[k++] = L.take(sizeof(int32_t) * n_pts);                          // obsrow
        o[k++] = L.take(sizeof(double) * (size_t)n_pts * 64);              // e2
    }
    if (lay) *lay = L;
    if (offs_out) std::memcpy(offs_out, o, sizeof(size_t) * k);
    return L.total;
}

int stage_copy(sabr_server *s, void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return SABR_OK;
    const size_t need = (bytes + 255) / 256 * 256;
    if (s->stage_used + need > s->stage_bytes) {
        if (hipStreamSynchronize(s->stream) != hipSuccess) return SABR_E_DEVICE;
        s->stage_used = 0;
        if (need > s->stage_bytes) {
            if (s->stage) hipHostFree(s->stage);
            s->stage = nullptr;
            s->stage_bytes = 0;
            void *h = nullptr;
            const size_t want = std::max<size_t>(need, 8 << 20);
            if (hipHostMalloc(&h, want, hipHostMallocDefault) != hipSuccess) return SABR_E_NOMEM;
            s->stage = (unsigned char *)h;
            s->stage_bytes = want;
        }
    }
    unsigned char *h = s->stage + s->stage_used;
    std::memcpy(h, src, bytes);
    s->stage_used += need;
    return hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, s->stream) == hipSuccess ? SABR_OK : SABR_E_DEVICE;
}

// Temperature levels a formula slot advances per quantum.  A quantum lasts as
// long as its slowest slot, so each slot takes as many levels as keep its work
// within four full quanta of the largest static slot (41 strikes, two lanes
// per chain), at least one and at most Q.  (Eight gives the largest dynamic
// grids more levels per quantum but makes every quantum, and so the static
// requests and the Monte Carlo iterations that start once per quantum,
// slower: a longer serving tail.)  Work per iteration and lane, in
// point evaluations: static ceil(n_pts / 2) + 8 (proposal, random words,
// Metropolis test), dynamic n_pts + 15 n_mat (the row blocks) + 10.  A
// request's result does not depend on how its levels are cut into quanta.
int slot_quantum_levels(int Q, int kind, int n_pts, int n_mat) {
    if (kind == KIND_MC) return Q;
    const double ref = 4.0 * Q * (21 + 8);
    const double c = kind == KIND_STATIC ? (n_pts + 1) / 2 + 8 : n_pts + 15.0 * n_mat + 10;
    const int q = (int)(ref / c);
    return q < 1 ? 1 : (q > Q ? Q : q);
}

// Build the device slot of request `o` in slot `si` (arena block at `base`).
int upload_slot(sabr_server *s, int si, const Owned &o, size_t base) {
    const sabr_request &q = o.req;
    const sabr_market &m = q.market;
    const sabr_problem &p = q.problem;
    const int n_pts = m.offs[m.n_mat], n_mat = m.n_mat, NP = p.n_par, P = q.sa.n_chains;
    const int levels = (q.sa.n_iters + q.sa.chain_len - 1) / q.sa.chain_len;
    size_t off[40];
    footprint(q, nullptr, off);
    unsigned char *b = s->arena_dev + base;
    SlotDev d;
    std::memset(&d, 0, sizeof d);
    int k = 0;
    d.K = (const double *)(b + off[k++]);
    d.lfk = (double *)(b + off[k++]);
    d.lkf = (double *)(b + off[k++]);
    d.P1 = (double *)(b + off[k++]);
    d.Z = (double *)(b + off[k++]);
    d.Q1 = (double *)(b + off[k++]);
    d.Q2 = (double *)(b + off[k++]);
    d.target = (double *)(b + off[k++]);
    d.sw = (double *)(b + off[k++]);
    d.row = (int32_t *)(b + off[k++]);
    d.T = (double *)(b + off[k++]);
    d.fwd = (double *)(b + off[k++]);
    d.lnf = (double *)(b + off[k++]);
    d.F1 = (double *)(b + off[k++]);
    d.disc = (double *)(b + off[k++]);
    d.offs = (int32_t *)(b + off[k++]);
    d.sched_g = (const double *)(b + off[k++]);
    d.sched_h = (const double *)(b + off[k++]);
    d.cx = (double *)(b + off[k++]);
    d.cf = (double *)(b + off[k++]);
    d.bx = (double *)(b + off[k++]);
    d.bf = (double *)(b + off[k++]);
    d.nacc = (unsigned long long *)(b + off[k++]);
    d.kind = slot_kind(q);
    d.state = SLOT_NEW;
    d.level = 0;
    d.q_levels = slot_quantum_levels(s->Q, d.kind, n_pts, n_mat);
    d.iter = -1;
    // descriptor
    ReqDesc &rq = d.rq;
    rq.model = p.model;
    rq.formula = p.model == SABR_STATIC ? q.obj.formula : 0;
    rq.weighting = q.obj.weighting;
    rq.beta_free = 0;
    rq.n_par = NP;
    rq.n_mat = n_mat;
    rq.n_pts = n_pts;
    rq.n_chains = P;
    rq.n_iters = q.sa.n_iters;
    rq.chain_len = q.sa.chain_len;
    rq.n_levels = levels;
    rq.n_wg = 1;
    rq.polish = q.sa.polish;
    rq.rsplit = 1;
    rq.key0 = (uint32_t)(q.sa.seed & 0xffffffffu);
    rq.key1 = (uint32_t)(q.sa.seed >> 32);
    rq.beta = p.beta;
    rq.T0 = q.sa.T0;
    double tmax = 0;
    for (int i = 0; i < n_mat; ++i) tmax = std::max(tmax, m.T[i]);
    rq.t_max = tmax;
    for (int j = 0; j < NP; ++j) {
        rq.lb[j] = p.lb[j];
        rq.ub[j] = p.ub[j];
        rq.x0[j] = p.x0 ? p.x0[j] : 0.5 * (p.lb[j] + p.ub[j]);
    }
    // schedule (same arithmetic as the batch path)
    std::vector<double> sg(levels), sh(levels);
    const double cL = std::pow(q.sa.cooling, (double)q.sa.chain_len);
    double g = 1.0;
    for (int l = 0; l < levels; ++l) {
        sg[l] = g;
        sh[l] = std::fmax(q.sa.step0 * std::sqrt(g), q.sa.step_min);
        g = g * cL;
    }
    std::vector<double> disc(n_mat);
    for (int i = 0; i < n_mat; ++i) disc[i] = m.disc ? m.disc[i] : 1.0;
    int rc;
    if ((rc = stage_copy(s, (void *)d.K, m.K, sizeof(double) * n_pts)) ||
        (rc = stage_copy(s, d.target, m.target, sizeof(double) * n_pts)) ||
        (rc = stage_copy(s, d.T, m.T, sizeof(double) * n_mat)) ||
        (rc = stage_copy(s, d.fwd, m.fwd, sizeof(double) * n_mat)) ||
        (rc = stage_copy(s, d.disc, disc.data(), sizeof(double) * n_mat)) ||
        (rc = stage_copy(s, d.offs, m.offs, sizeof(int32_t) * (n_mat + 1))) ||
        (rc = stage_copy(s, (void *)d.sched_g, sg.data(), sizeof(double) * levels)) ||
        (rc = stage_copy(s, (void *)d.sched_h, sh.data(), sizeof(double) * levels)))
        return rc;
    if (d.kind == KIND_MC) {
        d.mcst = (McSaState *)(b + off[k++]);
        d.Y = (double *)(b + off[k++]);
        d.fy = (double *)(b + off[k++]);
        d.part = (float *)(b + off[k++]);
        d.msteps = (int32_t *)(b + off[k++]);
        d.obsrow = (int32_t *)(b + off[k++]);
        d.e2 = (double *)(b + off[k++]);
        std::vector<int32_t> ms(n_mat), orow(n_pts);
        std::vector<double> sw(n_pts);
        int m_max = 0;
        for (int i = 0; i < n_mat; ++i) {
            ms[i] = n_steps(m.T[i], q.mc.steps_per_year);
            m_max = std::max(m_max, ms[i]);
            for (int j = m.offs[i]; j < m.offs[i + 1]; ++j) {
                orow[j] = i;
                sw[j] = q.obj.weighting == SABR_W_RELATIVE ? 1.0 / m.target[j] : 1.0;
            }
        }
        McCrnDesc &c = d.crn;
        c.n_mat = n_mat;
        c.n_obs = n_pts;
        c.m_max = m_max;
        c.n_pblocks = kMcPBlocks;
        c.n_chains = P;
        c.n_paths = q.mc.n_paths;
        c.paths_per_block = (q.mc.n_paths + kMcPBlocks - 1) / kMcPBlocks;
        c.np_stride = NP;
        c.beta_free = 0;
        c.dt = 1.0 / (double)q.mc.steps_per_year;
        c.f0 = m.fwd[0];
        c.beta = p.beta;
        c.key0 = (uint32_t)(q.mc.seed & 0xffffffffu);
        c.key1 = (uint32_t)(q.mc.seed >> 32);
        c.model = p.model;
        c.t_max = tmax;
        McSaDesc &a = d.sa;
        a.model = p.model;
        a.n_par = NP;
        a.n_chains = P;
        a.n_iters = q.sa.n_iters;
        a.chain_len = q.sa.chain_len;
        a.key0 = rq.key0;
        a.key1 = rq.key1;
        a.T0 = q.sa.T0;
        a.t_max = tmax;
        for (int j = 0; j < NP; ++j) {
            a.lb[j] = rq.lb[j];
            a.ub[j] = rq.ub[j];
            a.x0[j] = rq.x0[j];
        }
        if ((rc = stage_copy(s, d.msteps, ms.data(), sizeof(int32_t) * n_mat)) ||
            (rc = stage_copy(s, d.obsrow, orow.data(), sizeof(int32_t) * n_pts)) ||
            (rc = stage_copy(s, d.sw, sw.data(), sizeof(double) * n_pts)) ||
            (rc = stage_copy(s, d.Y, rq.x0, sizeof(double) * NP)))
            return rc;
        d.state = SLOT_READY;   // nothing to normalise for the path objective
    }
    return stage_copy(s, &s->d_slots[si], &d, sizeof d);
}

// Mark a slot free on the device (before the next quantum).
int clear_slot(sabr_server *s, int si) {
    SlotDev d;
    std::memset(&d, 0, sizeof d);
    d.state = SLOT_FREE;
    return stage_copy(s, &s->d_slots[si], &d, sizeof d);
}

// Capture the work queued on `st` by `body` as an executable graph.
template <typename F>
int capture_one(hipStream_t st, hipGraph_t *g, hipGraphExec_t *ge, F body) {
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return SABR_E_DEVICE;
    const bool ok = body();
    hipGraph_t gr = nullptr;
    const bool ended = hipStreamEndCapture(st, &gr) == hipSuccess;
    if (!ok || !ended) {
        hipGetLastError();
        if (gr) hipGraphDestroy(gr);
        return SABR_E_DEVICE;
    }
    *g = gr;
    return hipGraphInstantiate(ge, gr, nullptr, nullptr, 0) == hipSuccess ? SABR_OK : SABR_E_DEVICE;
}

// The work is three graphs.  The formula graph (main stream) normalises the
// grids of new formula slots and advances every formula slot by Q
// temperature levels in one launch of sa_slot_kernel; the formula status
// graph copies those slots' states back.  The Monte Carlo graph (second
// stream) runs one iteration of every Monte Carlo slot (paths, prices,
// objectives, accept/propose) and copies their states back;
// it runs beside the formula quanta and is relaunched when it has finished.
int capture_graph(sabr_server *s) {
    int nmc = s->n_mc, nf = s->n_slots - s->n_mc;
    int Q = s->Q;
    SlotDev *ds = s->d_slots;
    int rc = capture_one(s->stream, &s->graph, &s->gexec, [&] {
        void *a0[] = {&ds, &nmc};
        bool ok = hipLaunchKernel(slot_prepare_kernel_ptr(), dim3(nf), dim3(256), a0, 0, s->stream) == hipSuccess;
        void *a1[] = {&ds, &nmc, &Q};
        ok = ok && hipLaunchKernel(sa_slot_kernel_ptr(), dim3(nf), dim3(kSlotThreads), a1, sa_slot_smem_bytes(),
                                   s->stream) == hipSuccess;
        ok = ok && hipLaunchKernel(slot_polish_kernel_ptr(), dim3(nf), dim3(64), a0, slot_polish_smem_bytes(),
                                   s->stream) == hipSuccess;
        return ok;
    });
    if (rc) return rc;
    rc = capture_one(s->stream, &s->graph_st, &s->gexec_st, [&] {
        SlotStatus *dst = s->d_status;
        void *a4[] = {&ds, &nmc, &nf, &dst};
        bool ok = hipLaunchKernel(slot_status_kernel_ptr(), dim3((nf + 63) / 64), dim3(64), a4, 0, s->stream) ==
                  hipSuccess;
        ok = ok && hipMemcpyAsync(s->h_status + nmc, s->d_status + nmc, sizeof(SlotStatus) * nf,
                                  hipMemcpyDeviceToHost, s->stream) == hipSuccess;
        return ok;
    });
    if (rc) return rc;
    return capture_one(s->stream_mc, &s->graph_mc, &s->gexec_mc, [&] {
        // a linear graph: its kernels stay on the Monte Carlo stream's own
        // hardware queue (the parallel branches of a graph run on further
        // queues, one of which the formula stream can share, and a formula
        // quantum then waits behind a Monte Carlo kernel)
        void *a2[] = {&ds};
        bool ok = hipLaunchKernel(mc_slot_crn_kernel_ptr(), dim3(nmc * kMcPBlocks), dim3(64), a2,
                                  mc_crn_smem_bytes(kSlotMaxMcObs, true), s->stream_mc) == hipSuccess;
        void *a3[] = {&ds};
        ok = ok && hipLaunchKernel(mc_slot_prices_kernel_ptr(), dim3(nmc, kMcPriceGroups), dim3(256), a3, 0,
                                   s->stream_mc) == hipSuccess;
        ok = ok && hipLaunchKernel(mc_slot_objective_kernel_ptr(), dim3(nmc), dim3(64), a3, 0, s->stream_mc) ==
                   hipSuccess;
        ok = ok && hipLaunchKernel(mc_slot_step_kernel_ptr(), dim3(nmc), dim3(256), a3, 0, s->stream_mc) == hipSuccess;
        int zero = 0;
        SlotStatus *dst = s->d_status;
        void *a4[] = {&ds, &zero, &nmc, &dst};
        ok = ok && hipLaunchKernel(slot_status_kernel_ptr(), dim3((nmc + 63) / 64), dim3(64), a4, 0, s->stream_mc) ==
                   hipSuccess;
        ok = ok && hipMemcpyAsync(s->h_status, s->d_status, sizeof(SlotStatus) * nmc, hipMemcpyDeviceToHost,
                                  s->stream_mc) == hipSuccess;
        return ok;
    });
}

// Results of the finished or cancelled slots of [lo, hi) (caller holds the lock).
void collect(sabr_server *s, int lo, int hi) {
    const auto now = Clock::now();
    for (int i = lo; i < hi; ++i) {
        SlotHost &h = s->slots[i];
        if (!h.busy) continue;
        const SlotStatus &st = s->h_status[i];
        if (st.state != SLOT_DONE && !h.cancel) continue;
        Done d;
        d.ticket = h.ticket;
        std::memset(&d.res, 0, sizeof d.res);
        if (h.cancel) {
            d.res.status = SABR_E_CANCELLED;
            s->cancelled.erase(h.ticket);
        } else {
            for (int k = 0; k < h.n_par; ++k) d.res.x[k] = st.x[k];
            d.res.f = st.f;
            d.res.f_before_polish = st.f_pre;
            d.res.n_accept = (int64_t)st.n_accept;
            d.res.n_evals = (int64_t)st.n_evals;
            d.res.status = SABR_OK;
        }
        d.latency_s = std::chrono::duration<double>(now - h.t_submit).count();
        s->done.push_back(d);
        s->arena.release(h.off, h.bytes);
        h.busy = false;
        clear_slot(s, i);
        ++s->completed;
    }
}

void device_failed(sabr_server *s, const char *what) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->device_error = 1;
    s->err = what;
    s->cv_done.notify_all();
}

void worker_loop(sabr_server *s) {
    hipSetDevice(s->device);
    bool mc_busy = false;   // the Monte Carlo graph is in flight: its slots are not touched
    while (!s->stop.load()) {
        int active_f = 0, active_mc = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            // cancellations of queued requests
            for (auto it = s->queue.begin(); it != s->queue.end();) {
                if (s->cancelled.count((*it)->ticket)) {
                    Done d{(*it)->ticket, {}, 0.0};
                    d.res.status = SABR_E_CANCELLED;
                    s->done.push_back(d);
                    s->cancelled.erase((*it)->ticket);
                    delete *it;
                    it = s->queue.erase(it);
                } else {
                    ++it;
                }
            }
            // admission: first come first served within each kind; a request
            // needs a free slot of its kind and room in the arena (if the arena
            // is full, nothing behind it is admitted); Monte Carlo slots are
            // filled only while their graph is idle
            bool blocked[2] = {false, mc_busy};
            for (auto it = s->queue.begin(); it != s->queue.end();) {
                Owned *o = *it;
                const int kc = o->kind == KIND_MC ? 1 : 0;
                if (blocked[kc]) {
                    ++it;
                    continue;
                }
                int si = -1;
                const int lo = kc ? 0 : s->n_mc, hi = kc ? s->n_mc : s->n_slots;
                for (int i = lo; i < hi; ++i)
                    if (!s->slots[i].busy) {
                        si = i;
                        break;
                    }
                if (si < 0) {
                    blocked[kc] = true;
                    ++it;
                    continue;
                }
                size_t offb = 0;
                if (!s->arena.alloc(o->bytes, offb)) break;
                if (upload_slot(s, si, *o, offb) != SABR_OK) {
                    s->device_error = 1;
                    s->arena.release(offb, o->bytes);
                    break;
                }
                SlotHost &h = s->slots[si];
                h.busy = true;
                h.ticket = o->ticket;
                h.t_submit = o->t_submit;
                h.off = offb;
                h.bytes = o->bytes;
                h.n_par = o->req.problem.n_par;
                h.cancel = false;
                it = s->queue.erase(it);
                delete o;
                ++s->admitted;
            }
            for (auto &h : s->slots)
                if (h.busy && s->cancelled.count(h.ticket)) h.cancel = true;
            for (int i = 0; i < s->n_slots; ++i)
                if (s->slots[i].busy) (i < s->n_mc ? active_mc : active_f) += 1;
            s->peak_bytes = std::max(s->peak_bytes, s->arena.in_use());
            s->peak_active = std::max(s->peak_active, active_f + active_mc);
            if (active_f == 0 && active_mc == 0 && !mc_busy) {
                s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
        }
        // a new Monte Carlo iteration once the previous one has finished (it
        // waits for this round's uploads, which are on the main stream)
        if (!mc_busy && active_mc > 0) {
            if (hipEventRecord(s->ev_up, s->stream) != hipSuccess ||
                hipStreamWaitEvent(s->stream_mc, s->ev_up, 0) != hipSuccess ||
                hipGraphLaunch(s->gexec_mc, s->stream_mc) != hipSuccess ||
                hipEventRecord(s->ev_mc, s->stream_mc) != hipSuccess)
                return device_failed(s, "Monte Carlo graph launch failed");
            mc_busy = true;
        }
        if (active_f > 0) {
            if (hipGraphLaunch(s->gexec, s->stream) != hipSuccess ||
                hipGraphLaunch(s->gexec_st, s->stream) != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess)
                return device_failed(s, "formula graph replay failed");
        } else if (mc_busy) {
            if (hipEventSynchronize(s->ev_mc) != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess)
                return device_failed(s, "Monte Carlo graph failed");
        }
        bool mc_done = false;
        if (mc_busy) {
            const hipError_t q = hipEventQuery(s->ev_mc);
            if (q == hipSuccess)
                mc_done = true;
            else if (q != hipErrorNotReady)
                return device_failed(s, "Monte Carlo graph failed");
            else
                hipGetLastError();
        }
        s->stage_used = 0;   // the main stream has drained: staging is free again
        std::lock_guard<std::mutex> lk(s->mu);
        ++s->quanta;
        if (active_f > 0) collect(s, s->n_mc, s->n_slots);
        if (mc_done) {
            collect(s, 0, s->n_mc);
            mc_busy = false;
        }
        s->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

int sabr_server_create(sabr_ctx *ctx, int32_t max_slots, size_t hbm_budget_bytes, int32_t quantum_levels,
                       sabr_server **out) {
    if (!ctx || !out) return SABR_E_INVAL;
    *out = nullptr;
    if (max_slots < 2 || max_slots > 4096 || quantum_levels < 1)
        return fail(ctx, SABR_E_INVAL, "max_slots must be in [2, 4096] and quantum_levels >= 1");
    sabr_server *s = new (std::nothrow) sabr_server();
    if (!s) return SABR_E_NOMEM;
    s->ctx = ctx;
    s->device = device_of(ctx);
    hipSetDevice(s->device);
    s->n_slots = max_slots;
    s->n_mc = std::max(1, max_slots / 8);
    s->Q = quantum_levels;
    const size_t budget = hbm_budget_bytes ? hbm_budget_bytes : ((size_t)1 << 30);
    s->arena.init(budget);
    bool ok = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&s->stream_mc, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&s->ev_up, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&s->ev_mc, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->arena_dev, budget) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->d_slots, sizeof(SlotDev) * max_slots) == hipSuccess;
    ok = ok && hipMalloc((void **)&s->d_status, sizeof(SlotStatus) * max_slots) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&s->h_status, sizeof(SlotStatus) * max_slots, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        hipGetLastError();
        sabr_server_destroy(s);
        return fail(ctx, SABR_E_NOMEM, "server allocation failed");
    }
    s->slots.resize(max_slots);
    // every slot starts free: write the free table with a plain copy (no memset node in the graph)
    std::vector<SlotDev> z(max_slots);
    std::memset(z.data(), 0, sizeof(SlotDev) * max_slots);
    ok = hipMemcpy(s->d_slots, z.data(), sizeof(SlotDev) * max_slots, hipMemcpyHostToDevice) == hipSuccess;
    const size_t sm = sa_slot_smem_bytes();
    ok = ok && hipFuncSetAttribute(sa_slot_kernel_ptr(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm) == hipSuccess;
    ok = ok && hipFuncSetAttribute(slot_polish_kernel_ptr(), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)slot_polish_smem_bytes()) == hipSuccess;
    const size_t msm = mc_crn_smem_bytes(kSlotMaxMcObs, true);
    ok = ok && hipFuncSetAttribute(mc_slot_crn_kernel_ptr(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)msm) == hipSuccess;
    if (!ok || capture_graph(s) != SABR_OK) {
        hipGetLastError();
        sabr_server_destroy(s);
        return fail(ctx, SABR_E_DEVICE, "server graph capture failed");
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return SABR_OK;
}

int sabr_server_submit(sabr_server *s, const sabr_market *market, const sabr_problem *problem,
                       const sabr_objspec *obj, const sabr_sa *sa, const sabr_mc *mc, uint64_t *ticket) {
    if (!s || !market || !problem || !obj || !sa || !ticket) return SABR_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->device_error) return fail(s->ctx, SABR_E_DEVICE, "server stopped after a device error");
    if (obj->kind == SABR_OBJ_MC && !mc) return fail(s->ctx, SABR_E_INVAL, "the Monte Carlo objective needs mc settings");
    sabr_request q;
    std::memset(&q, 0, sizeof q);
    q.market = *market;
    q.problem = *problem;
    q.obj = *obj;
    q.sa = *sa;
    if (mc) q.mc = *mc;
    int rc = check_request(s->ctx, q);
    if (rc) return rc;
    const int kind = slot_kind(q);
    const int n_pts = q.market.offs[q.market.n_mat];
    if (q.obj.precision != SABR_FP32 || q.problem.beta_free || q.problem.model == SABR_DYN_II ||
        (q.problem.model == SABR_STATIC && q.obj.kind == SABR_OBJ_FORMULA && q.obj.formula != SABR_F_HAGAN) ||
        (kind == KIND_MC && q.problem.model != SABR_STATIC))
        return fail(s->ctx, SABR_E_INVAL,
                    "the server runs FP32 static Hagan, dynamic case I and static Monte Carlo requests with a fixed "
                    "beta; use sabr_calibrate for the others");
    const int cap = kind == KIND_STATIC ? kSlotThreads / 2 : (kind == KIND_DYN_I ? kSlotThreads : 64);
    if (q.sa.n_chains > cap) return fail(s->ctx, SABR_E_INVAL, "at most %d chains per request of this kind", cap);
    if (n_pts > kSlotMaxPts || q.market.n_mat > kSlotMaxMat || (kind == KIND_MC && n_pts > kSlotMaxMcObs))
        return fail(s->ctx, SABR_E_INVAL, "grid too large for a serving slot");
    if (kind == KIND_MC && q.mc.scheme != SABR_MC_PLAIN)
        return fail(s->ctx, SABR_E_INVAL, "the serving loop takes the plain path scheme only");
    // each lane of a path block adds its block's payoffs in float: at most
    // 256 per block (the bound of the float partial sums), kMcPBlocks blocks
    if (kind == KIND_MC && q.mc.n_paths > (int64_t)256 * kMcPBlocks)
        return fail(s->ctx, SABR_E_INVAL, "a served Monte Carlo request takes at most %d paths", 256 * kMcPBlocks);
    Owned *o = new Owned();
    o->kind = kind;
    const sabr_market &m = q.market;
    o->T.assign(m.T, m.T + m.n_mat);
    o->fwd.assign(m.fwd, m.fwd + m.n_mat);
    if (m.disc) o->disc.assign(m.disc, m.disc + m.n_mat);
    o->offs.assign(m.offs, m.offs + m.n_mat + 1);
    o->K.assign(m.K, m.K + n_pts);
    o->target.assign(m.target, m.target + n_pts);
    const int NP = q.problem.n_par;
    o->lb.assign(q.problem.lb, q.problem.lb + NP);
    o->ub.assign(q.problem.ub, q.problem.ub + NP);
    if (q.problem.x0) o->x0.assign(q.problem.x0, q.problem.x0 + NP);
    o->req = q;
    o->req.market.T = o->T.data();
    o->req.market.fwd = o->fwd.data();
    o->req.market.disc = m.disc ? o->disc.data() : nullptr;
    o->req.market.offs = o->offs.data();
    o->req.market.K = o->K.data();
    o->req.market.target = o->target.data();
    o->req.problem.lb = o->lb.data();
    o->req.problem.ub = o->ub.data();
    o->req.problem.x0 = q.problem.x0 ? o->x0.data() : nullptr;
    o->bytes = footprint(o->req);
    if (o->bytes > s->arena.size) {
        delete o;
        return fail(s->ctx, SABR_E_BUDGET, "request needs more device memory than the server budget");
    }
    o->ticket = s->next_ticket++;
    o->t_submit = Clock::now();
    *ticket = o->ticket;
    s->queue.push_back(o);
    s->cv_work.notify_one();
    return SABR_OK;
}

int sabr_server_poll(sabr_server *s, int32_t max, int32_t timeout_us, uint64_t *tickets, sabr_result *res,
                     double *latency_s, int32_t *n_done) {
    if (!s || !n_done || max < 0 || (max > 0 && (!tickets || !res))) return SABR_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_us > 0 && !s->device_error)
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !s->done.empty() || s->device_error; });
    int n = 0;
    while (n < max && !s->done.empty()) {
        tickets[n] = s->done.front().ticket;
        res[n] = s->done.front().res;
        if (latency_s) latency_s[n] = s->done.front().latency_s;
        s->done.pop_front();
        ++n;
    }
    *n_done = n;
    if (s->device_error) return fail(s->ctx, SABR_E_DEVICE, "server stopped after a device error");
    return (n == 0 && timeout_us > 0) ? SABR_E_TIMEOUT : SABR_OK;
}

int sabr_server_cancel(sabr_server *s, uint64_t ticket) {
    if (!s) return SABR_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->cancelled.insert(ticket);
    s->cv_work.notify_one();
    return SABR_OK;
}

int sabr_server_stats(sabr_server *s, int64_t *quanta, int64_t *admitted, int64_t *completed, int64_t *queued,
                      int32_t *active, size_t *bytes_in_use, size_t *peak_bytes, int32_t *peak_active) {
    if (!s) return SABR_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    int a = 0;
    for (auto &h : s->slots) a += h.busy ? 1 : 0;
    if (quanta) *quanta = s->quanta;
    if (admitted) *admitted = s->admitted;
    if (completed) *completed = s->completed;
    if (queued) *queued = (int64_t)s->queue.size();
    if (active) *active = a;
    if (bytes_in_use) *bytes_in_use = s->arena.in_use();
    if (peak_bytes) *peak_bytes = s->peak_bytes;
    if (peak_active) *peak_active = s->peak_active;
    return SABR_OK;
}

int sabr_server_destroy(sabr_server *s) {
    if (!s) return SABR_E_INVAL;
    s->stop.store(true);
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    hipSetDevice(s->device);
    if (s->stream) hipStreamSynchronize(s->stream);
    if (s->stream_mc) hipStreamSynchronize(s->stream_mc);
    for (hipGraphExec_t ge : {s->gexec, s->gexec_mc, s->gexec_st})
        if (ge) hipGraphExecDestroy(ge);
    for (hipGraph_t g : {s->graph, s->graph_mc, s->graph_st})
        if (g) hipGraphDestroy(g);
    if (s->ev_up) hipEventDestroy(s->ev_up);
    if (s->ev_mc) hipEventDestroy(s->ev_mc);
    if (s->arena_dev) hipFree(s->arena_dev);
    if (s->d_slots) hipFree(s->d_slots);
    if (s->d_status) hipFree(s->d_status);
    if (s->h_status) hipHostFree(s->h_status);
    if (s->stage) hipHostFree(s->stage);
    if (s->stream) hipStreamDestroy(s->stream);
    if (s->stream_mc) hipStreamDestroy(s->stream_mc);
    for (auto *o : s->queue) delete o;
    delete s;
    return SABR_OK;
}

}  // extern "C"
