// runtime.hip -- host side of libsabr_hip.so: the C ABI of include/sabr.h.
//
// Validates requests, lays the market grids out in device memory (CSR),
// launches the kernels on the context's stream and copies results back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sabr.h"
#include "sabr_kernels.h"

using namespace sabr;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = false;   // allocated by the library (else a region of the caller's workspace)
};

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace

struct sabr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0;
    size_t held = 0;
    std::string err;
    std::vector<DevBuf> bufs;   // reusable device buffers, by slot
    int n_cu = 0;
    size_t max_smem = 0;
    // timing of the dominant kernel
    bool timing = false;
    double kernel_ms = 0.0;
    int64_t launches = 0;
    std::string kernel_name;
    std::vector<EventPair> pending;
    std::vector<EventPair> pool;
    int force_lpc = 0;      // SABR_LANES_PER_CHAIN overrides the choice (1, 2, 4, 8 or 16)
    int force_rsplit = 0;   // SABR_ROW_SPLIT overrides the row split of a lane group (1 .. 16)
    int spin_limit = 1 << 22;   // SABR_EXCHANGE_SPINS: polls of a level-end slot before a wait fails
    int crn_variant = 0;    // SABR_CRN_VARIANT: Monte Carlo objective kernel layout (0 = production)
    // caller's device workspace (sabr_ctx_set_workspace): buffers are carved from it
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0, ws_used = 0;
    // pinned staging for host-to-device copies: valid until the next sync
    unsigned char *stage = nullptr;
    size_t stage_bytes = 0, stage_used = 0;
};

// ---------------------------------------------------------------------------
// Device memory of sabr_mc_price_noalloc: a file-scope array that each device
// holds from the loading of the library until the process ends.  In host
// code its name is only a stand-in: the address of each device's copy comes
// from hipGetSymbolAddress, taken once per device when the first context on
// that device is created, and only that address is handed to kernels and
// copies.  Layout of one call (256-byte aligned pieces): the workgroup
// partial sums and sums of squares (2048 x n_obs doubles each), price and
// standard error, strikes, discount factors, maturities, row offsets,
// maturity steps and option rows.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)17 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch[kMaxDevices];      // device address of each device's copy
static hipError_t g_scratch_err[kMaxDevices];

// With `device` current: look up its copy of the scratch array once.
static void scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        hipGetLastError();
        g_scratch_err[device] = e;
        return;
    }
    g_scratch[device] = static_cast<unsigned char *>(ptr);
}

namespace {

}  // namespace
namespace sabrhost {
int fail(sabr_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
}
namespace {
using namespace sabrhost;

#define HIPCHK(ctx, expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, SABR_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                                \
    } while (0)

// Slots of the context's reusable device buffers.
enum Slot {
    S_K, S_FWDP, S_BETAP, S_FORMP, S_WGHTP, S_TARGET, S_LFK, S_LKF, S_P1, S_Z, S_Q1, S_Q2, S_SW, S_ROW,
    S_T, S_FWD, S_BETAM, S_LNF, S_F1, S_OFFS, S_REQ, S_WGREQ, S_SCHED_G, S_SCHED_H, S_CAND,
    S_BEST, S_ACC, S_ERR, S_EVALS, S_POLREQ, S_X, S_F, S_MODEL, S_MSTEPS, S_MOFFS, S_DISC, S_OBSROW,
    S_PART, S_PARTQ, S_E2, S_PRICE, S_SE, S_Y, S_CX, S_CF, S_BX, S_BF, S_FY, S_MCSTATE, S_RESET, S_NSLOTS
};

// Start of an API call that computes: with a caller workspace, the buffers
// are carved again from its beginning (the previous call has synchronised).
void begin_call(sabr_ctx *c) {
    if (!c->ws) return;
    for (auto &b : c->bufs) b = DevBuf{};
    c->ws_used = 0;
}

int get_buf(sabr_ctx *c, int slot, size_t bytes, void **out) {
    if (bytes == 0) bytes = 16;
    if ((int)c->bufs.size() < S_NSLOTS) c->bufs.resize(S_NSLOTS);
    DevBuf &b = c->bufs[slot];
    if (c->ws) {
        // carve from the caller's workspace; a slot keeps its region for the call
        if (b.bytes < bytes) {
            const size_t off = (c->ws_used + 255) / 256 * 256;
            if (off + bytes > c->ws_bytes)
                return fail(c, SABR_E_BUDGET, "workspace of %zu bytes is too small (needs more than %zu)", c->ws_bytes,
                            off + bytes);
            b.p = c->ws + off;
            b.bytes = bytes;
            b.owned = false;
            c->ws_used = off + bytes;
        }
        *out = b.p;
        return SABR_OK;
    }
    if (b.bytes < bytes) {
        size_t want = std::max(bytes, b.bytes * 3 / 2);
        if (c->budget && c->held - b.bytes + want > c->budget) {
            want = bytes;
            if (c->held - b.bytes + want > c->budget)
                return fail(c, SABR_E_BUDGET, "device memory budget exceeded (%zu + %zu > %zu bytes)",
                            c->held - b.bytes, want, c->budget);
        }
        if (b.p) {
            hipStreamSynchronize(c->stream);
            hipFree(b.p);
            c->held -= b.bytes;
            b.p = nullptr;
            b.bytes = 0;
        }
        void *p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) {
            hipGetLastError();
            return fail(c, SABR_E_NOMEM, "hipMalloc of %zu bytes failed", want);
        }
        b.p = p;
        b.bytes = want;
        b.owned = true;
        c->held += want;
    }
    *out = b.p;
    return SABR_OK;
}

// Asynchronous host-to-device copy through the context's pinned staging
// buffer, so that the caller's host memory may be released at once.
int copy_h2d(sabr_ctx *c, void *dst, const void *src, size_t bytes) {
    if (bytes == 0) return SABR_OK;
    const size_t need = (bytes + 255) / 256 * 256;
    if (c->stage_used + need > c->stage_bytes) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->stage_used = 0;
        if (need > c->stage_bytes) {
            if (c->stage) hipHostFree(c->stage);
            c->stage = nullptr;
            c->stage_bytes = 0;
            const size_t want = std::max<size_t>(need, 1 << 20);
            void *h = nullptr;
            if (hipHostMalloc(&h, want, hipHostMallocDefault) != hipSuccess) {
                hipGetLastError();
                return fail(c, SABR_E_NOMEM, "hipHostMalloc of %zu bytes failed", want);
            }
            c->stage = static_cast<unsigned char *>(h);
            c->stage_bytes = want;
        }
    }
    unsigned char *h = c->stage + c->stage_used;
    std::memcpy(h, src, bytes);
    c->stage_used += need;
    HIPCHK(c, hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, c->stream));
    return SABR_OK;
}

template <typename T>
int upload(sabr_ctx *c, int slot, const std::vector<T> &v, T **out) {
    void *p;
    int rc = get_buf(c, slot, v.size() * sizeof(T), &p);
    if (rc) return rc;
    if ((rc = copy_h2d(c, p, v.data(), v.size() * sizeof(T)))) return rc;
    *out = static_cast<T *>(p);
    return SABR_OK;
}

EventPair take_events(sabr_ctx *c) {
    EventPair e;
    if (!c->pool.empty()) {
        e = c->pool.back();
        c->pool.pop_back();
    } else {
        hipEventCreate(&e.a);
        hipEventCreate(&e.b);
    }
    return e;
}

// Launch `fn` bracketed by timing events when timing is on.
int launch(sabr_ctx *c, bool dominant, const char *name, const void *fn, dim3 grid, dim3 block,
           void **args, size_t smem, bool cooperative = false) {
    EventPair ev;
    const bool t = c->timing && dominant;
    if (t) {
        ev = take_events(c);
        HIPCHK(c, hipEventRecord(ev.a, c->stream));
    }
    hipError_t e = cooperative ? hipLaunchCooperativeKernel(fn, grid, block, args, (unsigned)smem, c->stream)
                               : hipLaunchKernel(fn, grid, block, args, smem, c->stream);
    if (e != hipSuccess) {
        hipGetLastError();
        return fail(c, SABR_E_DEVICE, "launch of %s failed: %s", name, hipGetErrorString(e));
    }
    if (t) {
        HIPCHK(c, hipEventRecord(ev.b, c->stream));
        c->pending.push_back(ev);
        c->kernel_name = name;
    }
    return SABR_OK;
}

int sync_and_account(sabr_ctx *c) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->stage_used = 0;
    for (auto &ev : c->pending) {
        float ms = 0.0f;
        hipEventElapsedTime(&ms, ev.a, ev.b);
        c->kernel_ms += ms;
        c->launches += 1;
        c->pool.push_back(ev);
    }
    c->pending.clear();
    return SABR_OK;
}

int set_smem(sabr_ctx *c, const void *fn, size_t smem) {
    if (smem > c->max_smem)
        return fail(c, SABR_E_INVAL, "market grid needs %zu bytes of LDS, the device has %zu", smem,
                    c->max_smem);
    if (smem > 65536) HIPCHK(c, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
    return SABR_OK;
}

}  // namespace

namespace sabrhost {
int fail(sabr_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}
int device_of(const sabr_ctx *c) { return c->device; }
int base_npar(int model) { return model == SABR_STATIC ? 3 : (model == SABR_DYN_I ? 5 : (model == SABR_DYN_II ? 9 : -1)); }

int n_steps(double T, int spy) {
    const int m = (int)std::floor(T * (double)spy + 1e-9);
    return m < 1 ? 1 : m;
}

static bool finite(double v) { return std::isfinite(v); }

// --- validation ---------------------------------------------------------------
int check_market(sabr_ctx *c, const sabr_market *m, bool need_target, bool mc, int weighting) {
    if (!m) return fail(c, SABR_E_INVAL, "market is NULL");
    if (m->n_mat < 1) return fail(c, SABR_E_INVAL, "n_mat must be >= 1");
    if (!m->T || !m->fwd || !m->offs || !m->K) return fail(c, SABR_E_INVAL, "market arrays must not be NULL");
    if (m->offs[0] != 0) return fail(c, SABR_E_INVAL, "offs[0] must be 0");
    for (int i = 0; i < m->n_mat; ++i) {
        if (m->offs[i + 1] <= m->offs[i]) return fail(c, SABR_E_INVAL, "offs must be strictly increasing");
        if (!(m->T[i] > 0) || !finite(m->T[i])) return fail(c, SABR_E_INVAL, "T[%d] must be > 0", i);
        if (!(m->fwd[i] > 0) || !finite(m->fwd[i])) return fail(c, SABR_E_INVAL, "fwd[%d] must be > 0", i);
        if (m->disc && (!(m->disc[i] > 0) || !finite(m->disc[i])))
            return fail(c, SABR_E_INVAL, "disc[%d] must be > 0", i);
    }
    const int n = m->offs[m->n_mat];
    for (int j = 0; j < n; ++j) {
        if (!finite(m->K[j]) || (mc ? m->K[j] < 0 : !(m->K[j] > 0)))
            return fail(c, SABR_E_INVAL, "K[%d] out of range", j);
        if (m->target) {
            if (!finite(m->target[j])) return fail(c, SABR_E_INVAL, "target[%d] not finite", j);
            if (weighting == SABR_W_RELATIVE && !(m->target[j] > 0))
                return fail(c, SABR_E_INVAL, "target[%d] must be > 0 under relative weighting", j);
        }
    }
    if (need_target && !m->target) return fail(c, SABR_E_INVAL, "market target is NULL");
    if (mc)
        for (int i = 1; i < m->n_mat; ++i)
            if (m->fwd[i] != m->fwd[0])
                return fail(c, SABR_E_INVAL, "Monte Carlo needs one forward for all maturities");
    return SABR_OK;
}

int check_problem(sabr_ctx *c, const sabr_problem *p, bool need_box) {
    if (!p) return fail(c, SABR_E_INVAL, "problem is NULL");
    const int np = base_npar(p->model);
    if (np < 0) return fail(c, SABR_E_INVAL, "unknown model %d", p->model);
    if (p->n_par != np + (p->beta_free ? 1 : 0))
        return fail(c, SABR_E_INVAL, "n_par %d does not match model %d (beta_free %d)", p->n_par, p->model,
                    p->beta_free);
    if (!p->beta_free && !(p->beta >= 0.0 && p->beta <= 1.0)) return fail(c, SABR_E_INVAL, "beta must be in [0,1]");
    if (need_box) {
        if (!p->lb || !p->ub) return fail(c, SABR_E_INVAL, "lb/ub must not be NULL");
        for (int k = 0; k < p->n_par; ++k) {
            if (!finite(p->lb[k]) || !finite(p->ub[k]) || p->lb[k] > p->ub[k])
                return fail(c, SABR_E_INVAL, "box coordinate %d invalid", k);
            if (p->x0 && !(p->x0[k] >= p->lb[k] && p->x0[k] <= p->ub[k]))
                return fail(c, SABR_E_INVAL, "x0[%d] outside the box", k);
        }
        if (!(p->lb[0] > 0)) return fail(c, SABR_E_INVAL, "alpha lower bound must be > 0");
        if (p->lb[1] < -1.0 || p->ub[1] > 1.0) return fail(c, SABR_E_INVAL, "rho bounds must lie in [-1, 1]");
        if (p->lb[2] < 0.0) return fail(c, SABR_E_INVAL, "nu lower bound must be >= 0");
        if (p->beta_free && (p->lb[p->n_par - 1] < 0.0 || p->ub[p->n_par - 1] > 1.0))
            return fail(c, SABR_E_INVAL, "beta bounds must lie in [0, 1]");
    }
    return SABR_OK;
}

int check_obj(sabr_ctx *c, const sabr_objspec *o, int model) {
    if (!o) return fail(c, SABR_E_INVAL, "objspec is NULL");
    if (o->kind != SABR_OBJ_FORMULA && o->kind != SABR_OBJ_MC) return fail(c, SABR_E_INVAL, "bad objective kind");
    if (o->formula < 0 || o->formula > 2) return fail(c, SABR_E_INVAL, "bad formula");
    if (o->weighting != SABR_W_ABSOLUTE && o->weighting != SABR_W_RELATIVE) return fail(c, SABR_E_INVAL, "bad weighting");
    if (o->precision != SABR_FP64 && o->precision != SABR_FP32) return fail(c, SABR_E_INVAL, "bad precision");
    (void)model;
    return SABR_OK;
}

int check_mc(sabr_ctx *c, const sabr_mc *m) {
    if (!m) return fail(c, SABR_E_INVAL, "mc settings are NULL");
    if (m->n_paths < 1 || m->n_paths > (int64_t)0xffffffffLL) return fail(c, SABR_E_INVAL, "n_paths must be in [1, 2^32)");
    if (m->steps_per_year < 1) return fail(c, SABR_E_INVAL, "steps_per_year must be >= 1");
    if (m->scheme != SABR_MC_PLAIN && m->scheme != SABR_MC_ANTITHETIC)
        return fail(c, SABR_E_INVAL, "unknown path scheme %d", m->scheme);
    if (m->scheme == SABR_MC_ANTITHETIC && m->n_paths % 2 != 0)
        return fail(c, SABR_E_INVAL, "antithetic paths come in pairs: n_paths must be even");
    return SABR_OK;
}

int check_sa(sabr_ctx *c, const sabr_sa *s) {
    if (s->n_chains < 1 || s->n_iters < 1 || s->chain_len < 1) return fail(c, SABR_E_INVAL, "annealing sizes must be >= 1");
    if (!(s->cooling > 0.0 && s->cooling <= 1.0)) return fail(c, SABR_E_INVAL, "cooling must be in (0, 1]");
    if (!(s->step0 > 0.0) || !(s->step_min >= 0.0)) return fail(c, SABR_E_INVAL, "step sizes invalid");
    return SABR_OK;
}

// Validation of one calibration request (shared by sabr_calibrate and the server).
int check_request(sabr_ctx *c, const sabr_request &q) {
    int rc;
    const bool mc = q.obj.kind == SABR_OBJ_MC;
    if ((rc = check_obj(c, &q.obj, q.problem.model)) || (rc = check_problem(c, &q.problem, true)) ||
        (rc = check_market(c, &q.market, true, mc, q.obj.weighting)) || (rc = check_sa(c, &q.sa)) ||
        (mc && (rc = check_mc(c, &q.mc))))
        return rc;
    return SABR_OK;
}

}  // namespace sabrhost

namespace {
using namespace sabrhost;

bool case2_ok_host(const double *x, double tmax) {
    auto range = [&](double c0, double c1, double k, double d, double &lo, double &hi) {
        const double v0 = c0 + d, v1 = (c0 + c1 * tmax) * std::exp(-k * tmax) + d;
        lo = std::min(v0, v1);
        hi = std::max(v0, v1);
        if (k != 0.0 && c1 != 0.0) {   // interior extremum, either sign of k
            const double ts = 1.0 / k - c0 / c1;
            if (ts > 0.0 && ts < tmax) {
                const double v = (c0 + c1 * ts) * std::exp(-k * ts) + d;
                lo = std::min(lo, v);
                hi = std::max(hi, v);
            }
        }
    };
    double rlo, rhi, nlo, nhi;
    range(x[1], x[7], x[3], x[5], rlo, rhi);
    range(x[2], x[8], x[4], x[6], nlo, nhi);
    return rlo >= -1.0 && rhi <= 1.0 && nlo > 0.0;
}

// --- grid packing ---------------------------------------------------------------
struct Packed {
    std::vector<double> K, fwdp, betap, target, T, fwd, betam;
    std::vector<int32_t> formp, wghtp, row, offs;
};

// Append one grid; returns the point and maturity offsets.
void pack_grid(Packed &pk, const sabr_market &m, const sabr_problem &p, const sabr_objspec &o, int &pt_off,
               int &mat_off) {
    pt_off = (int)pk.K.size();
    mat_off = (int)pk.T.size();
    const double beta = p.beta_free ? 1.0 : p.beta;
    for (int i = 0; i < m.n_mat; ++i) {
        pk.T.push_back(m.T[i]);
        pk.fwd.push_back(m.fwd[i]);
        pk.betam.push_back(beta);
        pk.offs.push_back(pt_off + m.offs[i]);
        for (int j = m.offs[i]; j < m.offs[i + 1]; ++j) {
            pk.K.push_back(m.K[j]);
            pk.fwdp.push_back(m.fwd[i]);
            pk.betap.push_back(beta);
            pk.formp.push_back(o.formula);
            pk.wghtp.push_back(o.weighting);
            pk.target.push_back(m.target ? m.target[j] : 0.0);
            pk.row.push_back(mat_off + i);
        }
    }
}

struct DevGrid {
    PointsD P;
    MatsD Mt;
};

// Device memory of one launch: the context's reusable buffers, or (for a
// prepared batch) allocations the batch owns until it is destroyed.
struct Alloc {
    sabr_ctx *c;
    std::vector<void *> *owned = nullptr;
    int get(int slot, size_t bytes, void **p) {
        if (!owned) return get_buf(c, slot, bytes, p);
        if (bytes == 0) bytes = 16;
        void *q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) {
            hipGetLastError();
            return fail(c, SABR_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
        }
        owned->push_back(q);
        *p = q;
        return SABR_OK;
    }
    template <typename T>
    int put(int slot, const std::vector<T> &v, T **out) {
        void *p;
        int rc = get(slot, v.size() * sizeof(T), &p);
        if (rc) return rc;
        if ((rc = copy_h2d(c, p, v.data(), v.size() * sizeof(T)))) return rc;
        *out = static_cast<T *>(p);
        return SABR_OK;
    }
};

// Packed raw grids in device memory, and the buffers their normalisation fills.
struct RawGrid {
    double *K, *fwdp, *betap, *target, *T, *fwd, *betam;
    int32_t *formp, *wghtp, *row, *offs;
    double *lfk, *lkf, *P1, *Z, *Q1, *Q2, *sw, *lnf, *F1;
    int np, nm;
};

// Copy packed grids to the device and reserve the normalised arrays.
int upload_raw(sabr_ctx *c, Packed &pk, RawGrid &g, Alloc &al) {
    pk.offs.push_back((int32_t)pk.K.size());   // closing offset of the last grid
    int rc;
    if ((rc = al.put(S_K, pk.K, &g.K)) || (rc = al.put(S_FWDP, pk.fwdp, &g.fwdp)) ||
        (rc = al.put(S_BETAP, pk.betap, &g.betap)) || (rc = al.put(S_TARGET, pk.target, &g.target)) ||
        (rc = al.put(S_T, pk.T, &g.T)) || (rc = al.put(S_FWD, pk.fwd, &g.fwd)) ||
        (rc = al.put(S_BETAM, pk.betam, &g.betam)) || (rc = al.put(S_FORMP, pk.formp, &g.formp)) ||
        (rc = al.put(S_WGHTP, pk.wghtp, &g.wghtp)) || (rc = al.put(S_ROW, pk.row, &g.row)) ||
        (rc = al.put(S_OFFS, pk.offs, &g.offs)))
        return rc;
    g.np = (int)pk.K.size();
    g.nm = (int)pk.T.size();
    const size_t np = (size_t)g.np, nm = (size_t)g.nm;
    void *b[9];
    if ((rc = al.get(S_LFK, np * 8, &b[0])) || (rc = al.get(S_LKF, np * 8, &b[1])) ||
        (rc = al.get(S_P1, np * 8, &b[2])) || (rc = al.get(S_Z, np * 8, &b[3])) ||
        (rc = al.get(S_Q1, np * 8, &b[4])) || (rc = al.get(S_Q2, np * 8, &b[5])) ||
        (rc = al.get(S_SW, np * 8, &b[6])) || (rc = al.get(S_LNF, nm * 8, &b[7])) ||
        (rc = al.get(S_F1, nm * 8, &b[8])))
        return rc;
    double **d[9] = {&g.lfk, &g.lkf, &g.P1, &g.Z, &g.Q1, &g.Q2, &g.sw, &g.lnf, &g.F1};
    for (int i = 0; i < 9; ++i) *d[i] = (double *)b[i];
    return SABR_OK;
}

// Grid normalisation (row a1 of the path): per point and per maturity.
int launch_normalise(sabr_ctx *c, const RawGrid &g, DevGrid &dg) {
    int rc;
    int n = g.np;
    void *a1[] = {&n, (void *)&g.K, (void *)&g.fwdp, (void *)&g.betap, (void *)&g.formp, (void *)&g.wghtp,
                  (void *)&g.target, (void *)&g.lfk, (void *)&g.lkf, (void *)&g.P1, (void *)&g.Z,
                  (void *)&g.Q1, (void *)&g.Q2, (void *)&g.sw};
    if ((rc = launch(c, false, "prepare_points", prepare_points_kernel_ptr(), dim3((n + 255) / 256), dim3(256), a1, 0)))
        return rc;
    int nmi = g.nm;
    void *a2[] = {&nmi, (void *)&g.fwd, (void *)&g.betam, (void *)&g.lnf, (void *)&g.F1};
    if ((rc = launch(c, false, "prepare_mats", prepare_mats_kernel_ptr(), dim3((nmi + 255) / 256), dim3(256), a2, 0)))
        return rc;
    dg.P = PointsD{g.lfk, g.lkf, g.P1, g.Z, g.Q1, g.Q2, g.target, g.sw, g.row};
    dg.Mt = MatsD{g.T, g.lnf, g.F1, g.offs};
    return SABR_OK;
}

// Upload packed grids and run the normalisation kernels.
int upload_grids(sabr_ctx *c, Packed &pk, DevGrid &g) {
    Alloc al{c};
    RawGrid raw;
    int rc;
    if ((rc = upload_raw(c, pk, raw, al))) return rc;
    return launch_normalise(c, raw, g);
}

void fill_desc(ReqDesc &d, const sabr_market &m, const sabr_problem &p, const sabr_objspec &o, int pt_off,
               int mat_off) {
    std::memset(&d, 0, sizeof d);
    d.model = p.model;
    d.formula = p.model == SABR_STATIC ? o.formula : F_HAGAN;
    d.weighting = o.weighting;
    d.beta_free = p.beta_free ? 1 : 0;
    d.n_par = p.n_par;
    d.n_mat = m.n_mat;
    d.n_pts = m.offs[m.n_mat];
    d.pt_off = pt_off;
    d.mat_off = mat_off;
    d.beta = p.beta;
    double tmax = 0;
    for (int i = 0; i < m.n_mat; ++i) tmax = std::max(tmax, m.T[i]);
    d.t_max = tmax;
    for (int k = 0; k < p.n_par && p.lb; ++k) {
        d.lb[k] = p.lb[k];
        d.ub[k] = p.ub[k];
        d.x0[k] = p.x0 ? p.x0[k] : 0.5 * (p.lb[k] + p.ub[k]);
    }
}

bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    std::memset(&a, 0, sizeof a);
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// --- formula calibration ------------------------------------------------------------
struct Group {
    int model, formula, fp32, bfree, lpc;
    std::vector<int> reqs;
};

// Lanes per chain, a property of the request alone (so that its result never
// depends on the other requests of a batch): requests of 1024 chains or more
// split each chain's work over two lanes, which doubles the waves of the
// few-but-large requests that would otherwise leave SIMDs half idle.  Float
// dynamic requests of 256 chains or more (many maturity rows, each with its
// own integrals, so little work is repeated across the lanes of a group)
// widen the group up to 16 lanes while the request stays within two waves
// per SIMD of the whole chip (131072 lanes) and the group within twice its
// rows.
int lanes_per_chain(const sabr_ctx *c, const sabr_request &q) {
    const bool wide = wide_lanes_supported(q.problem.model, q.obj.precision == SABR_FP32);
    if (c->force_lpc) return c->force_lpc > 2 && !wide ? 2 : c->force_lpc;
    if (wide && q.sa.n_chains >= 256) {
        int lpc = 1;
        while (lpc < 16 && (int64_t)q.sa.n_chains * lpc * 2 <= 131072 && lpc * 2 <= 2 * q.market.n_mat) lpc *= 2;
        return lpc;
    }
    return q.sa.n_chains >= 1024 ? 2 : 1;
}

// How the lanes of a group share the maturity rows.  0: whole rounds of one
// row per lane, then the remaining rows over the smallest power of two of
// lanes that holds them, the other lanes splitting their strikes.  A fixed
// split r (SABR_ROW_SPLIT) gives lane s the rows s % r (mod r) and the
// strikes of each such row to the LPC / r lanes that share it.  The static
// z-form formulas split strikes only.
int row_split(const sabr_ctx *c, const sabr_request &q, int lpc) {
    if (lpc == 1 || q.problem.model == SABR_STATIC) return 1;
    if (c->force_rsplit) return std::min(c->force_rsplit, lpc);
    return 0;
}

// A request spread over several workgroups needs them all resident at once
// (level-end exchange); a group too large for that is split into groups of
// fewer requests that run as consecutive launches (each request's result is
// unchanged).
void split_group(sabr_ctx *c, const sabr_request *reqs, const Group &grp, std::vector<Group> &out) {
    const int nr = (int)grp.reqs.size();
    const int chains_per_wg = kWG / grp.lpc;
    if (nr > 1) {
        const bool fp32 = grp.fp32 != 0;
        size_t smem = 0;
        int64_t total = 0;
        bool multi = false;
        for (int r : grp.reqs) {
            const sabr_request &q = reqs[r];
            smem = std::max(smem, grid_smem_bytes(fp32, q.market.offs[q.market.n_mat], q.market.n_mat));
            const int64_t nwg = (q.sa.n_chains + chains_per_wg - 1) / chains_per_wg;
            total += nwg;
            multi |= nwg > 1;
        }
        smem += sa_smem_fixed_bytes();
        const void *fn = sa_kernel_ptr(grp.model, grp.formula, fp32, grp.bfree != 0, grp.lpc);
        int per_cu = 0;
        if (multi && fn && smem <= c->max_smem) {
            if (smem > 65536) hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kWG, smem) != hipSuccess) per_cu = 0;
            hipGetLastError();
            if (per_cu > 0 && total > (int64_t)per_cu * c->n_cu) {
                Group a = grp, b = grp;
                a.reqs.assign(grp.reqs.begin(), grp.reqs.begin() + nr / 2);
                b.reqs.assign(grp.reqs.begin() + nr / 2, grp.reqs.end());
                split_group(c, reqs, a, out);
                split_group(c, reqs, b, out);
                return;
            }
        }
    }
    out.push_back(grp);
}

// Host side of one annealing launch: packed grids, descriptors, schedules,
// workgroup map, kernels and their LDS sizes.
struct GroupPlan {
    Group grp;
    Packed pk;
    std::vector<ReqDesc> desc;
    std::vector<double> sg, sh;
    std::vector<int32_t> wg_req, pol;
    int cand_slots = 0;
    size_t smem = 0, psm = 0;
    bool multi_wg = false;
    const void *fn = nullptr, *pf = nullptr;
};

// Device side of one annealing launch.
struct GroupDev {
    RawGrid raw;
    ReqDesc *dreq = nullptr;
    int32_t *dwg = nullptr, *dpol = nullptr;
    double *dsg = nullptr, *dsh = nullptr;
    void *cand = nullptr, *best = nullptr, *acc = nullptr, *err = nullptr, *evals = nullptr;
};

int plan_group(sabr_ctx *c, const sabr_request *reqs, const Group &grp, GroupPlan &pl) {
    const int nr = (int)grp.reqs.size();
    const int lpc = grp.lpc;
    const int chains_per_wg = kWG / lpc;
    pl.grp = grp;
    pl.desc.resize(nr);
    for (int r = 0; r < nr; ++r) {
        const sabr_request &q = reqs[grp.reqs[r]];
        int pt_off, mat_off;
        pack_grid(pl.pk, q.market, q.problem, q.obj, pt_off, mat_off);
        ReqDesc &d = pl.desc[r];
        fill_desc(d, q.market, q.problem, q.obj, pt_off, mat_off);
        d.n_chains = q.sa.n_chains;
        d.n_iters = q.sa.n_iters;
        d.chain_len = q.sa.chain_len;
        d.n_levels = (q.sa.n_iters + q.sa.chain_len - 1) / q.sa.chain_len;
        d.sched_off = (int)pl.sg.size();
        d.polish = q.sa.polish;
        d.rsplit = row_split(c, q, lpc);
        d.spin_limit = c->spin_limit;
        d.key0 = (uint32_t)(q.sa.seed & 0xffffffffu);
        d.key1 = (uint32_t)(q.sa.seed >> 32);
        d.T0 = q.sa.T0;
        const double cL = std::pow(q.sa.cooling, (double)q.sa.chain_len);
        double g = 1.0;
        for (int k = 0; k < d.n_levels; ++k) {
            pl.sg.push_back(g);
            pl.sh.push_back(std::fmax(q.sa.step0 * std::sqrt(g), q.sa.step_min));
            g = g * cL;
        }
        d.n_wg = (q.sa.n_chains + chains_per_wg - 1) / chains_per_wg;
        if (d.n_wg > kMaxReaders * kWG)
            return fail(c, SABR_E_BUDGET, "request %d spans %d annealing workgroups (at most %d)", r, d.n_wg,
                        kMaxReaders * kWG);
        d.wg_first = (int)pl.wg_req.size();
        for (int w = 0; w < d.n_wg; ++w) pl.wg_req.push_back(r);
        d.cand_off = pl.cand_slots;
        // two halves of candidates, then for each round parity the result
        // slots of the reader workgroups (one per kWG candidates, wide requests)
        pl.cand_slots += 2 * d.n_wg + 2 * ((d.n_wg + kWG - 1) / kWG);
        if (d.polish) pl.pol.push_back(r);
        pl.multi_wg |= d.n_wg > 1;
    }
    const bool fp32 = grp.fp32 != 0;
    // the polish stages the double grid: refuse a grid it cannot hold before annealing
    for (int r = 0; r < nr; ++r) {
        const size_t psm = grid_smem_bytes(false, pl.desc[r].n_pts, pl.desc[r].n_mat) + sizeof(int32_t) * pl.desc[r].n_pts;
        if (pl.desc[r].polish && psm > c->max_smem)
            return fail(c, SABR_E_INVAL, "the polish needs %zu bytes of LDS for this grid, the device has %zu", psm,
                        c->max_smem);
        if (pl.desc[r].polish) pl.psm = std::max(pl.psm, psm);
    }
    for (int r = 0; r < nr; ++r) pl.smem = std::max(pl.smem, grid_smem_bytes(fp32, pl.desc[r].n_pts, pl.desc[r].n_mat));
    pl.smem += sa_smem_fixed_bytes();
    pl.fn = sa_kernel_ptr(grp.model, grp.formula, fp32, grp.bfree != 0, lpc);
    if (!pl.fn) return fail(c, SABR_E_INVAL, "no kernel for model %d formula %d", grp.model, grp.formula);
    int rc;
    if ((rc = set_smem(c, pl.fn, pl.smem))) return rc;
    if (pl.multi_wg) {
        int per_cu = 0;
        HIPCHK(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pl.fn, kWG, pl.smem));
        if ((int64_t)per_cu * c->n_cu < (int64_t)pl.wg_req.size())
            return fail(c, SABR_E_BUDGET,
                        "%d annealing workgroups cannot be resident at once (%d per CU x %d CUs); split the batch",
                        (int)pl.wg_req.size(), per_cu, c->n_cu);
    }
    if (!pl.pol.empty()) {
        pl.pf = polish_kernel_ptr(grp.model, grp.formula, grp.bfree != 0);
        if ((rc = set_smem(c, pl.pf, pl.psm))) return rc;
    }
    return SABR_OK;
}

int upload_group(sabr_ctx *c, GroupPlan &pl, GroupDev &gd, Alloc &al) {
    const int nr = (int)pl.desc.size();
    int rc;
    if ((rc = upload_raw(c, pl.pk, gd.raw, al))) return rc;
    if ((rc = al.put(S_REQ, pl.desc, &gd.dreq)) || (rc = al.put(S_WGREQ, pl.wg_req, &gd.dwg)) ||
        (rc = al.put(S_SCHED_G, pl.sg, &gd.dsg)) || (rc = al.put(S_SCHED_H, pl.sh, &gd.dsh)))
        return rc;
    if (!pl.pol.empty() && (rc = al.put(S_POLREQ, pl.pol, &gd.dpol))) return rc;
    if ((rc = al.get(S_CAND, sizeof(Cand) * std::max(pl.cand_slots, 1), &gd.cand)) ||
        (rc = al.get(S_BEST, sizeof(ChainOut) * nr, &gd.best)) ||
        (rc = al.get(S_ACC, sizeof(unsigned long long) * nr, &gd.acc)) ||
        (rc = al.get(S_ERR, sizeof(int32_t), &gd.err)) ||
        (rc = al.get(S_EVALS, sizeof(unsigned long long) * nr, &gd.evals)))
        return rc;
    return SABR_OK;
}

// Grid normalisation, annealing, polish and results of one planned launch;
// out is indexed like the requests the group was planned from.
int exec_group(sabr_ctx *c, const GroupPlan &pl, GroupDev &gd, sabr_result *out) {
    const int nr = (int)pl.desc.size();
    int rc;
    DevGrid g;
    if ((rc = launch_normalise(c, gd.raw, g))) return rc;
    HIPCHK(c, hipMemsetAsync(gd.cand, 0, sizeof(Cand) * std::max(pl.cand_slots, 1), c->stream));   // exchange tags
    HIPCHK(c, hipMemsetAsync(gd.acc, 0, sizeof(unsigned long long) * nr, c->stream));
    HIPCHK(c, hipMemsetAsync(gd.err, 0, sizeof(int32_t), c->stream));
    HIPCHK(c, hipMemsetAsync(gd.evals, 0, sizeof(unsigned long long) * nr, c->stream));
    PointsD P = g.P;
    MatsD Mt = g.Mt;
    void *args[] = {&gd.dreq, &gd.dwg, &P, &Mt, &gd.dsg, &gd.dsh, &gd.cand, &gd.best, &gd.acc, &gd.err};
    if ((rc = launch(c, true, "sa_kernel", pl.fn, dim3((unsigned)pl.wg_req.size()), dim3(kWG), args, pl.smem,
                     pl.multi_wg)))
        return rc;
    std::vector<ChainOut> hpre(nr);
    HIPCHK(c, hipMemcpyAsync(hpre.data(), gd.best, sizeof(ChainOut) * nr, hipMemcpyDeviceToHost, c->stream));
    if (!pl.pol.empty()) {
        void *pargs[] = {&gd.dreq, &gd.dpol, &P, &Mt, &gd.best, &gd.evals};
        if ((rc = launch(c, false, "polish_kernel", pl.pf, dim3((unsigned)pl.pol.size()), dim3(64), pargs, pl.psm)))
            return rc;
    }
    std::vector<ChainOut> hb(nr);
    std::vector<unsigned long long> ha(nr), he(nr);
    int32_t herr = 0;
    HIPCHK(c, hipMemcpyAsync(hb.data(), gd.best, sizeof(ChainOut) * nr, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(ha.data(), gd.acc, sizeof(unsigned long long) * nr, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(he.data(), gd.evals, sizeof(unsigned long long) * nr, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&herr, gd.err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    if ((rc = sync_and_account(c))) return rc;
    if (herr) return fail(c, SABR_E_TIMEOUT, "a workgroup of the annealing kernel exceeded its wait bound");
    for (int r = 0; r < nr; ++r) {
        sabr_result &o = out[pl.grp.reqs[r]];
        std::memset(&o, 0, sizeof o);
        for (int k = 0; k < pl.desc[r].n_par; ++k) o.x[k] = hb[r].bx[k];
        o.f = hb[r].bf;
        o.f_before_polish = hpre[r].bf;
        o.n_accept = (int64_t)ha[r];
        o.n_evals = 1 + (int64_t)pl.desc[r].n_chains * pl.desc[r].n_iters + (int64_t)he[r];
        o.status = SABR_OK;
    }
    return SABR_OK;
}

int run_formula_group(sabr_ctx *c, const sabr_request *reqs, const Group &grp, sabr_result *out) {
    std::vector<Group> parts;
    split_group(c, reqs, grp, parts);
    for (const Group &g : parts) {
        GroupPlan pl;
        GroupDev gd;
        Alloc al{c};
        int rc;
        if ((rc = plan_group(c, reqs, g, pl)) || (rc = upload_group(c, pl, gd, al)) || (rc = exec_group(c, pl, gd, out)))
            return rc;
    }
    return SABR_OK;
}

// --- Monte Carlo objective ----------------------------------------------------------
struct McGrid {
    int n_mat, n_obs, m_max;
    double t_max;
    int32_t *msteps, *moffs, *obsrow;
    double *K, *disc, *target, *sw;
};

int upload_mc_grid(sabr_ctx *c, const sabr_market &m, int spy, int weighting, McGrid &g) {
    std::vector<int32_t> ms(m.n_mat), mo(m.n_mat + 1), orow(m.offs[m.n_mat]);
    std::vector<double> K(m.offs[m.n_mat]), disc(m.n_mat), tg(m.offs[m.n_mat]), sw(m.offs[m.n_mat]);
    // rows sorted by step so that the kernels meet the maturities in order
    std::vector<int> order(m.n_mat);
    for (int i = 0; i < m.n_mat; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n_steps(m.T[a], spy) < n_steps(m.T[b], spy); });
    bool sorted = true;
    for (int i = 0; i < m.n_mat; ++i) sorted &= order[i] == i;
    if (!sorted) return fail(c, SABR_E_INVAL, "Monte Carlo grids must list maturities in increasing order");
    g.m_max = 0;
    for (int i = 0; i < m.n_mat; ++i) {
        ms[i] = n_steps(m.T[i], spy);
        g.m_max = std::max(g.m_max, ms[i]);
        mo[i] = m.offs[i];
        disc[i] = m.disc ? m.disc[i] : 1.0;
        for (int j = m.offs[i]; j < m.offs[i + 1]; ++j) {
            orow[j] = i;
            K[j] = m.K[j];
            tg[j] = m.target ? m.target[j] : 0.0;
            sw[j] = (weighting == SABR_W_RELATIVE && m.target) ? 1.0 / m.target[j] : 1.0;
        }
    }
    mo[m.n_mat] = m.offs[m.n_mat];
    g.t_max = 0.0;
    for (int i = 0; i < m.n_mat; ++i) g.t_max = std::max(g.t_max, m.T[i]);
    g.n_mat = m.n_mat;
    g.n_obs = m.offs[m.n_mat];
    int rc;
    if ((rc = upload(c, S_MSTEPS, ms, &g.msteps)) || (rc = upload(c, S_MOFFS, mo, &g.moffs)) ||
        (rc = upload(c, S_OBSROW, orow, &g.obsrow)) || (rc = upload(c, S_K, K, &g.K)) ||
        (rc = upload(c, S_DISC, disc, &g.disc)) || (rc = upload(c, S_TARGET, tg, &g.target)) ||
        (rc = upload(c, S_SW, sw, &g.sw)))
        return rc;
    return SABR_OK;
}

// Path blocks of the common-random-number kernel.  Direct: one round of
// paths (16) per block, each block's option sums written straight to
// HBM (chosen while those partials stay within 4 GB and half the context's
// budget or workspace); otherwise up to 256 paths per block summed in LDS
// first.
bool crn_direct(const sabr_ctx *c, int64_t n_chains, int64_t n_paths, int n_obs) {
    if (c->crn_variant != 0) return false;
    const int64_t tiles = (n_chains + 63) / 64;
    const int64_t np = mc_crn_direct_paths();
    const int64_t nb = (n_paths + np - 1) / np;
    const double bytes = 4.0 * 64 * (double)tiles * n_obs * (double)nb;
    return bytes <= 4294967296.0 && (c->budget == 0 || bytes <= 0.5 * (double)c->budget) &&
           (!c->ws || bytes <= 0.5 * (double)c->ws_bytes);
}

void crn_geometry(int64_t n_chains, int64_t n_paths, McCrnDesc &d, bool direct) {
    if (direct) {
        d.paths_per_block = mc_crn_direct_paths();
        d.n_pblocks = (int32_t)((n_paths + d.paths_per_block - 1) / d.paths_per_block);
        return;
    }
    const int64_t tiles = (n_chains + 63) / 64;
    int64_t nb = std::max<int64_t>(1, 4096 / tiles);
    int64_t ppb = (n_paths + nb - 1) / nb;
    ppb = std::max<int64_t>(ppb, 16);
    ppb = std::min<int64_t>(ppb, 256);
    nb = (n_paths + ppb - 1) / ppb;
    d.n_pblocks = (int32_t)nb;
    d.paths_per_block = ppb;
}

// f (and model prices) of n_x parameter vectors Ydev (device, row stride np) by CRN paths.
int mc_objective_device(sabr_ctx *c, const McGrid &g, int model, int n_par, int beta_free, double beta,
                        double f0, const sabr_mc &mc, int64_t n_x, const double *Ydev, double *fdev,
                        double *modeldev, bool want_f, bool dominant) {
    McCrnDesc d;
    std::memset(&d, 0, sizeof d);
    d.n_mat = g.n_mat;
    d.n_obs = g.n_obs;
    d.m_max = g.m_max;
    d.n_chains = n_x;
    d.n_paths = mc.n_paths;
    d.np_stride = n_par;
    d.beta_free = beta_free;
    d.dt = 1.0 / (double)mc.steps_per_year;
    d.f0 = f0;
    d.beta = beta;
    d.key0 = (uint32_t)(mc.seed & 0xffffffffu);
    d.key1 = (uint32_t)(mc.seed >> 32);
    d.model = model;
    d.anti = mc.scheme == SABR_MC_ANTITHETIC;
    d.t_max = g.t_max;
    const bool direct = crn_direct(c, n_x, mc.n_paths, g.n_obs);
    crn_geometry(n_x, mc.n_paths, d, direct);
    const int64_t tiles = (n_x + 63) / 64;
    void *part;
    int rc;
    if ((rc = get_buf(c, S_PART, sizeof(float) * (size_t)tiles * g.n_obs * d.n_pblocks * 64, &part))) return rc;
    const void *fn = direct ? mc_crn_direct_kernel_ptr(model) : mc_crn_kernel_ptr(model, c->crn_variant);
    const size_t smem = mc_crn_smem_bytes(g.n_obs, direct);
    if ((rc = set_smem(c, fn, smem))) return rc;
    const int32_t *ms = g.msteps, *mo = g.moffs;
    const double *K = g.K;
    void *a1[] = {&d, &Ydev, &ms, &mo, &K, &part};
    if ((rc = launch(c, dominant, "mc_crn_kernel", fn, dim3((unsigned)(tiles * d.n_pblocks)), dim3(64), a1, smem)))
        return rc;
    const int32_t *orow = g.obsrow;
    const double *disc = g.disc, *tg = g.target, *sw = g.sw;
    void *e2 = nullptr;
    int64_t e2_stride = tiles * 64;
    if (want_f && (rc = get_buf(c, S_E2, sizeof(double) * (size_t)e2_stride * g.n_obs, &e2))) return rc;
    void *a2[] = {&d, &part, &orow, &disc, &tg, &sw, &modeldev, &e2, &e2_stride};
    if ((rc = launch(c, false, "mc_crn_prices", mc_crn_prices_ptr(), dim3((unsigned)tiles, (unsigned)g.n_obs), dim3(256),
                     a2, 0)))
        return rc;
    if (!want_f) return SABR_OK;
    void *a3[] = {&d, &Ydev, &e2, &e2_stride, &fdev};
    return launch(c, false, "mc_crn_objective", mc_crn_objective_ptr(), dim3((unsigned)((n_x + 255) / 256)), dim3(256),
                  a3, 0);
}

int run_mc_request(sabr_ctx *c, const sabr_request &q, sabr_result &out) {
    const sabr_market &m = q.market;
    const sabr_problem &p = q.problem;
    const int NP = p.n_par;
    if (p.beta_free) return fail(c, SABR_E_INVAL, "the Monte Carlo objective needs a fixed beta");
    if (q.sa.n_chains > 1 << 20) return fail(c, SABR_E_INVAL, "too many chains");
    McGrid g;
    int rc;
    if ((rc = upload_mc_grid(c, m, q.mc.steps_per_year, q.obj.weighting, g))) return rc;
    McSaDesc d;
    std::memset(&d, 0, sizeof d);
    d.model = p.model;
    d.n_par = NP;
    d.n_chains = q.sa.n_chains;
    d.n_iters = q.sa.n_iters;
    d.chain_len = q.sa.chain_len;
    d.key0 = (uint32_t)(q.sa.seed & 0xffffffffu);
    d.key1 = (uint32_t)(q.sa.seed >> 32);
    d.T0 = q.sa.T0;
    double tmax = 0;
    for (int i = 0; i < m.n_mat; ++i) tmax = std::max(tmax, m.T[i]);
    d.t_max = tmax;
    for (int k = 0; k < NP; ++k) {
        d.lb[k] = p.lb[k];
        d.ub[k] = p.ub[k];
        d.x0[k] = p.x0 ? p.x0[k] : 0.5 * (p.lb[k] + p.ub[k]);
    }
    if (p.model == SABR_DYN_II && !case2_ok_host(d.x0, tmax))
        return fail(c, SABR_E_INFEASIBLE, "case II start point violates the constraints");
    const int n_levels = (q.sa.n_iters + q.sa.chain_len - 1) / q.sa.chain_len;
    std::vector<double> sg(n_levels), sh(n_levels);
    const double cL = std::pow(q.sa.cooling, (double)q.sa.chain_len);
    double gk = 1.0;
    for (int k = 0; k < n_levels; ++k) {
        sg[k] = gk;
        sh[k] = std::fmax(q.sa.step0 * std::sqrt(gk), q.sa.step_min);
        gk = gk * cL;
    }
    double *dsg, *dsh;
    if ((rc = upload(c, S_SCHED_G, sg, &dsg)) || (rc = upload(c, S_SCHED_H, sh, &dsh))) return rc;
    const size_t P = (size_t)q.sa.n_chains;
    void *Y, *cx, *cf, *bx, *bf, *fy, *st;
    if ((rc = get_buf(c, S_Y, sizeof(double) * P * NP, &Y)) || (rc = get_buf(c, S_CX, sizeof(double) * P * NP, &cx)) ||
        (rc = get_buf(c, S_CF, sizeof(double) * P, &cf)) || (rc = get_buf(c, S_BX, sizeof(double) * P * NP, &bx)) ||
        (rc = get_buf(c, S_BF, sizeof(double) * P, &bf)) || (rc = get_buf(c, S_FY, sizeof(double) * P, &fy)) ||
        (rc = get_buf(c, S_MCSTATE, sizeof(McSaState), &st)))
        return rc;
    // f(x0)
    if ((rc = copy_h2d(c, Y, d.x0, sizeof(double) * NP))) return rc;
    if ((rc = mc_objective_device(c, g, p.model, NP, 0, p.beta, m.fwd[0], q.mc, 1, (const double *)Y,
                                  (double *)fy, nullptr, true, false)))
        return rc;
    const void *step = mc_sa_step_ptr();
    int t = -1;
    void *sargs[] = {&d, &t, &dsg, &dsh, &fy, &Y, &st, &cx, &cf, &bx, &bf};
    if ((rc = launch(c, false, "mc_sa_step", step, dim3(1), dim3(1024), sargs, 0))) return rc;
    for (t = 0; t < q.sa.n_iters; ++t) {
        if ((rc = mc_objective_device(c, g, p.model, NP, 0, p.beta, m.fwd[0], q.mc, (int64_t)P, (const double *)Y,
                                      (double *)fy, nullptr, true, true)))
            return rc;
        if ((rc = launch(c, false, "mc_sa_step", step, dim3(1), dim3(1024), sargs, 0))) return rc;
    }
    void *fargs[] = {&d, &bx, &bf, &st};
    if ((rc = launch(c, false, "mc_sa_final", mc_sa_final_ptr(), dim3(1), dim3(64), fargs, 0))) return rc;
    McSaState hs;
    HIPCHK(c, hipMemcpyAsync(&hs, st, sizeof hs, hipMemcpyDeviceToHost, c->stream));
    if ((rc = sync_and_account(c))) return rc;
    std::memset(&out, 0, sizeof out);
    for (int k = 0; k < NP; ++k) out.x[k] = hs.best_x[k];
    out.f = hs.best_f;
    out.f_before_polish = hs.best_f;
    out.n_accept = (int64_t)hs.n_accept;
    out.n_evals = 1 + (int64_t)P * q.sa.n_iters;
    out.status = SABR_OK;
    return SABR_OK;
}

// Validation of a calibration call: out[r].status gets each request's error.
int validate_requests(sabr_ctx *c, int n_req, const sabr_request *reqs, sabr_result *out) {
    int bad = 0;
    std::string first_err;
    for (int r = 0; r < n_req; ++r) {
        const sabr_request &q = reqs[r];
        std::memset(&out[r], 0, sizeof out[r]);
        int rc;
        const bool mc = q.obj.kind == SABR_OBJ_MC;
        if ((rc = check_request(c, q))) {
            out[r].status = rc;
            if (!bad) first_err = c->err;
            ++bad;
            continue;
        }
        if (q.problem.model == SABR_DYN_II && !mc) {
            double x0[kMaxPar], tmax = 0;
            for (int k = 0; k < q.problem.n_par; ++k)
                x0[k] = q.problem.x0 ? q.problem.x0[k] : 0.5 * (q.problem.lb[k] + q.problem.ub[k]);
            for (int i = 0; i < q.market.n_mat; ++i) tmax = std::max(tmax, q.market.T[i]);
            if (!case2_ok_host(x0, tmax)) {
                out[r].status = SABR_E_INFEASIBLE;
                if (!bad) first_err = "case II start point violates the constraints";
                ++bad;
            }
        }
    }
    if (bad) {
        c->err = first_err;
        return SABR_E_INVAL;
    }
    return SABR_OK;
}

// Formula requests grouped by kernel variant, in request order.
void group_formula_requests(sabr_ctx *c, int n_req, const sabr_request *reqs, std::vector<Group> &groups) {
    for (int r = 0; r < n_req; ++r) {
        const sabr_request &q = reqs[r];
        if (q.obj.kind != SABR_OBJ_FORMULA) continue;
        const int formula = q.problem.model == SABR_STATIC ? q.obj.formula : F_HAGAN;
        const int fp32 = q.obj.precision == SABR_FP32;
        const int bfree = q.problem.beta_free ? 1 : 0;
        const int lpc = lanes_per_chain(c, q);
        Group *gp = nullptr;
        for (auto &g : groups)
            if (g.model == q.problem.model && g.formula == formula && g.fp32 == fp32 && g.bfree == bfree &&
                g.lpc == lpc)
                gp = &g;
        if (!gp) {
            groups.push_back(Group{q.problem.model, formula, fp32, bfree, lpc, {}});
            gp = &groups.back();
        }
        gp->reqs.push_back(r);
    }
}

}  // namespace

// =====================================================================================
// C ABI
// =====================================================================================
// A prepared batch: the plans and device inputs of its annealing launches.
struct sabr_batch {
    sabr_ctx *ctx = nullptr;
    int n_req = 0;
    std::vector<GroupPlan> plans;
    std::vector<GroupDev> devs;
    std::vector<void *> owned;   // device allocations, freed by sabr_batch_destroy
};

extern "C" {

int sabr_ctx_create(int device, size_t hbm_budget_bytes, void *stream, sabr_ctx **out) {
    if (!out) return SABR_E_INVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        hipGetLastError();
        return SABR_E_INVAL;
    }
    sabr_ctx *c = new (std::nothrow) sabr_ctx();
    if (!c) return SABR_E_NOMEM;
    c->device = device;
    c->budget = hbm_budget_bytes;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return SABR_E_DEVICE;
    }
    scratch_setup(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return SABR_E_DEVICE;
    }
    c->n_cu = prop.multiProcessorCount;
    if (const char *e = std::getenv("SABR_LANES_PER_CHAIN")) {
        const int v = std::atoi(e);
        c->force_lpc = (v == 1 || v == 2 || v == 4 || v == 8 || v == 16) ? v : 0;
    }
    if (const char *e = std::getenv("SABR_CRN_VARIANT")) {
        const int v = std::atoi(e);
        c->crn_variant = (v >= 0 && v <= 9) ? v : 0;
    }
    if (const char *e = std::getenv("SABR_ROW_SPLIT")) {
        const int v = std::atoi(e);
        c->force_rsplit = (v == 1 || v == 2 || v == 4 || v == 8 || v == 16) ? v : 0;
    }
    if (const char *e = std::getenv("SABR_EXCHANGE_SPINS")) {
        const int v = std::atoi(e);
        c->spin_limit = (v >= 0 && v <= (1 << 22)) ? v : (1 << 22);
    }
    int smem = 0;
    hipDeviceGetAttribute(&smem, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    c->max_smem = (size_t)smem;
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return SABR_E_DEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return SABR_OK;
}

void sabr_ctx_destroy(sabr_ctx *c) {
    if (!c) return;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    for (auto &b : c->bufs)
        if (b.p && b.owned) hipFree(b.p);
    for (auto &e : c->pool) {
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
    }
    for (auto &e : c->pending) {
        hipEventDestroy(e.a);
        hipEventDestroy(e.b);
    }
    if (c->own_stream) hipStreamDestroy(c->stream);
    if (c->stage) hipHostFree(c->stage);
    delete c;
}

const char *sabr_ctx_last_error(const sabr_ctx *c) { return c ? c->err.c_str() : "no context"; }

int sabr_ctx_set_workspace(sabr_ctx *c, void *dev_ptr, size_t bytes) {
    if (!c) return SABR_E_INVAL;
    c->err.clear();
    hipSetDevice(c->device);
    if (dev_ptr) {
        hipPointerAttribute_t a;
        std::memset(&a, 0, sizeof a);
        if (hipPointerGetAttributes(&a, dev_ptr) != hipSuccess) hipGetLastError();
        if (a.type != hipMemoryTypeDevice || a.device != c->device)
            return fail(c, SABR_E_INVAL, "the workspace must be device memory of device %d", c->device);
        if (bytes < 4096) return fail(c, SABR_E_INVAL, "a workspace needs at least 4096 bytes");
    }
    hipStreamSynchronize(c->stream);
    for (auto &b : c->bufs) {
        if (b.p && b.owned) {
            hipFree(b.p);
            c->held -= b.bytes;
        }
        b = DevBuf{};
    }
    c->ws = (unsigned char *)dev_ptr;
    c->ws_bytes = dev_ptr ? bytes : 0;
    c->ws_used = 0;
    return SABR_OK;
}

int sabr_ctx_enable_timing(sabr_ctx *c, int enable) {
    if (!c) return SABR_E_INVAL;
    c->timing = enable != 0;
    return SABR_OK;
}

int sabr_ctx_timing(sabr_ctx *c, int reset, double *kernel_ms, int64_t *launches, char *name, size_t name_len) {
    if (!c) return SABR_E_INVAL;
    if (kernel_ms) *kernel_ms = c->kernel_ms;
    if (launches) *launches = c->launches;
    if (name && name_len) {
        std::strncpy(name, c->kernel_name.c_str(), name_len - 1);
        name[name_len - 1] = 0;
    }
    if (reset) {
        c->kernel_ms = 0.0;
        c->launches = 0;
    }
    return SABR_OK;
}

int sabr_calibrate_many(sabr_ctx *c, int32_t n_req, const sabr_request *reqs, sabr_result *out) {
    if (!c) return SABR_E_INVAL;
    begin_call(c);
    if (n_req < 1 || !reqs || !out) return fail(c, SABR_E_INVAL, "need n_req >= 1 and non-NULL arrays");
    c->err.clear();
    hipSetDevice(c->device);
    int rc;
    if ((rc = validate_requests(c, n_req, reqs, out))) return rc;
    std::vector<Group> groups;
    group_formula_requests(c, n_req, reqs, groups);
    for (auto &g : groups) {
        if ((rc = run_formula_group(c, reqs, g, out))) {
            for (int r : g.reqs) out[r].status = rc;
            return rc;
        }
    }
    for (int r = 0; r < n_req; ++r) {
        if (reqs[r].obj.kind != SABR_OBJ_MC) continue;
        if ((rc = run_mc_request(c, reqs[r], out[r]))) {
            out[r].status = rc;
            return rc;
        }
    }
    return SABR_OK;
}

int sabr_calibrate(sabr_ctx *c, const sabr_market *market, const sabr_problem *problem, const sabr_objspec *obj,
                   const sabr_sa *sa, const sabr_mc *mc, sabr_result *out) {
    if (!c) return SABR_E_INVAL;
    if (!market || !problem || !obj || !sa || !out)
        return fail(c, SABR_E_INVAL, "market, problem, objspec, sa and out must not be NULL");
    if (obj->kind == SABR_OBJ_MC && !mc) return fail(c, SABR_E_INVAL, "the Monte Carlo objective needs mc settings");
    sabr_request q;
    std::memset(&q, 0, sizeof q);
    q.market = *market;
    q.problem = *problem;
    q.obj = *obj;
    q.sa = *sa;
    if (mc) q.mc = *mc;
    const int rc = sabr_calibrate_many(c, 1, &q, out);
    return (rc == SABR_E_INVAL && out->status < 0) ? out->status : rc;   // e.g. SABR_E_INFEASIBLE
}

int sabr_batch_prepare(sabr_ctx *c, int32_t n_req, const sabr_request *reqs, sabr_batch **out) {
    if (!c) return SABR_E_INVAL;
    if (!out) return fail(c, SABR_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n_req < 1 || !reqs) return fail(c, SABR_E_INVAL, "need n_req >= 1 and a non-NULL request array");
    c->err.clear();
    hipSetDevice(c->device);
    for (int r = 0; r < n_req; ++r)
        if (reqs[r].obj.kind == SABR_OBJ_MC)
            return fail(c, SABR_E_INVAL, "request %d uses the Monte Carlo objective; a prepared batch holds formula "
                                         "requests only (use sabr_calibrate_many)", r);
    std::vector<sabr_result> tmp(n_req);
    int rc;
    if ((rc = validate_requests(c, n_req, reqs, tmp.data()))) return rc;
    std::vector<Group> groups, parts;
    group_formula_requests(c, n_req, reqs, groups);
    for (const Group &g : groups) split_group(c, reqs, g, parts);
    sabr_batch *b = new sabr_batch;
    b->ctx = c;
    b->n_req = n_req;
    b->plans.resize(parts.size());
    b->devs.resize(parts.size());
    for (size_t i = 0; i < parts.size() && !rc; ++i) {
        Alloc al{c, &b->owned};
        if ((rc = plan_group(c, reqs, parts[i], b->plans[i]))) break;
        if ((rc = upload_group(c, b->plans[i], b->devs[i], al))) break;
        // the host copies of the grids are no longer needed
        b->plans[i].pk = Packed{};
    }
    if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) {
        hipGetLastError();
        rc = fail(c, SABR_E_DEVICE, "upload of the batch failed");
    }
    if (rc) {
        sabr_batch_destroy(b);
        return rc;
    }
    *out = b;
    return SABR_OK;
}

int sabr_batch_run(sabr_batch *b, sabr_result *out) {
    if (!b) return SABR_E_INVAL;
    sabr_ctx *c = b->ctx;
    if (!out) return fail(c, SABR_E_INVAL, "out is NULL");
    c->err.clear();
    hipSetDevice(c->device);
    for (int r = 0; r < b->n_req; ++r) std::memset(&out[r], 0, sizeof out[r]);
    for (size_t i = 0; i < b->plans.size(); ++i) {
        const GroupPlan &pl = b->plans[i];
        int rc;
        if ((rc = set_smem(c, pl.fn, pl.smem)) || (!pl.pol.empty() && (rc = set_smem(c, pl.pf, pl.psm))) ||
            (rc = exec_group(c, pl, b->devs[i], out))) {
            for (int r : pl.grp.reqs) out[r].status = rc;
            return rc;
        }
    }
    return SABR_OK;
}

void sabr_batch_destroy(sabr_batch *b) {
    if (!b) return;
    hipSetDevice(b->ctx->device);
    hipStreamSynchronize(b->ctx->stream);
    for (void *p : b->owned) hipFree(p);
    delete b;
}

int sabr_objective_batch(sabr_ctx *c, const sabr_market *market, const sabr_problem *problem,
                         const sabr_objspec *obj, const sabr_mc *mc, int64_t n_x, const double *X, double *f,
                         double *model) {
    if (!c) return SABR_E_INVAL;
    begin_call(c);
    c->err.clear();
    hipSetDevice(c->device);
    int rc;
    if ((rc = check_obj(c, obj, problem ? problem->model : 0))) return rc;
    const bool is_mc = obj->kind == SABR_OBJ_MC;
    if ((rc = check_problem(c, problem, false))) return rc;
    if ((rc = check_market(c, market, false, is_mc, obj->weighting))) return rc;
    if (is_mc && (rc = check_mc(c, mc))) return rc;
    if (n_x < 0) return fail(c, SABR_E_INVAL, "n_x must be >= 0");
    if (n_x == 0) return SABR_OK;
    if (!X) return fail(c, SABR_E_INVAL, "X is NULL");
    const bool want_f = market->target != nullptr;
    if (!want_f && !model) return fail(c, SABR_E_INVAL, "no target and no model output: nothing to compute");
    if (want_f && !f) return fail(c, SABR_E_INVAL, "f is NULL");
    const int NP = problem->n_par;
    const int n_obs = market->offs[market->n_mat];
    const bool xd = is_device_ptr(X), fd = is_device_ptr(f), md = is_device_ptr(model);
    const double *Xdev = X;
    double *fdev = f, *mdev = model;
    void *p;
    if (!xd) {
        if ((rc = get_buf(c, S_X, sizeof(double) * (size_t)n_x * NP, &p))) return rc;
        if ((rc = copy_h2d(c, p, X, sizeof(double) * (size_t)n_x * NP))) return rc;
        Xdev = (const double *)p;
    }
    if (want_f && !fd) {
        if ((rc = get_buf(c, S_F, sizeof(double) * (size_t)n_x, &p))) return rc;
        fdev = (double *)p;
    }
    if (model && !md) {
        if ((rc = get_buf(c, S_MODEL, sizeof(double) * (size_t)n_x * n_obs, &p))) return rc;
        mdev = (double *)p;
    }
    if (!is_mc) {
        Packed pk;
        int pt_off, mat_off;
        pack_grid(pk, *market, *problem, *obj, pt_off, mat_off);
        DevGrid g;
        if ((rc = upload_grids(c, pk, g))) return rc;
        ReqDesc d;
        fill_desc(d, *market, *problem, *obj, pt_off, mat_off);
        std::vector<ReqDesc> dv(1, d);
        ReqDesc *dreq;
        if ((rc = upload(c, S_REQ, dv, &dreq))) return rc;
        const bool fp32 = obj->precision == SABR_FP32;
        const int formula = problem->model == SABR_STATIC ? obj->formula : F_HAGAN;
        const void *fn = objective_kernel_ptr(problem->model, formula, fp32, problem->beta_free != 0);
        if (!fn) return fail(c, SABR_E_INVAL, "no objective kernel for this model/formula");
        const size_t smem = grid_smem_bytes(fp32, d.n_pts, d.n_mat);
        if ((rc = set_smem(c, fn, smem))) return rc;
        const int64_t blocks = std::min<int64_t>((n_x + 255) / 256, 65535);
        PointsD P = g.P;
        MatsD Mt = g.Mt;
        int wf = want_f ? 1 : 0;
        void *args[] = {&dreq, &P, &Mt, &Xdev, &n_x, &fdev, &mdev, &wf};
        if ((rc = launch(c, true, "objective_kernel", fn, dim3((unsigned)blocks), dim3(256), args, smem))) return rc;
    } else {
        if (problem->beta_free) return fail(c, SABR_E_INVAL, "the Monte Carlo objective needs a fixed beta");
        McGrid g;
        if ((rc = upload_mc_grid(c, *market, mc->steps_per_year, obj->weighting, g))) return rc;
        if ((rc = mc_objective_device(c, g, problem->model, NP, 0, problem->beta, market->fwd[0], *mc, n_x, Xdev,
                                      fdev, mdev, want_f, true)))
            return rc;
    }
    if (want_f && !fd) HIPCHK(c, hipMemcpyAsync(f, fdev, sizeof(double) * (size_t)n_x, hipMemcpyDeviceToHost, c->stream));
    if (model && !md)
        HIPCHK(c, hipMemcpyAsync(model, mdev, sizeof(double) * (size_t)n_x * n_obs, hipMemcpyDeviceToHost, c->stream));
    return sync_and_account(c);
}

int sabr_mc_price(sabr_ctx *c, const sabr_market *market, const sabr_problem *problem, const sabr_mc *mc,
                  int32_t precision, double *price, double *std_err) {
    if (!c) return SABR_E_INVAL;
    begin_call(c);
    c->err.clear();
    hipSetDevice(c->device);
    int rc;
    if ((rc = check_problem(c, problem, false))) return rc;
    if (!problem->x0) return fail(c, SABR_E_INVAL, "problem->x0 (the parameters) is NULL");
    if ((rc = check_market(c, market, false, true, SABR_W_ABSOLUTE))) return rc;
    if ((rc = check_mc(c, mc))) return rc;
    if (precision != SABR_FP32 && precision != SABR_FP64) return fail(c, SABR_E_INVAL, "bad precision");
    if (!price) return fail(c, SABR_E_INVAL, "price is NULL");
    McGrid g;
    if ((rc = upload_mc_grid(c, *market, mc->steps_per_year, SABR_W_ABSOLUTE, g))) return rc;
    McDesc d;
    std::memset(&d, 0, sizeof d);
    d.model = problem->model;
    d.n_mat = g.n_mat;
    d.n_obs = g.n_obs;
    d.m_max = g.m_max;
    d.n_paths = mc->n_paths;
    d.dt = 1.0 / (double)mc->steps_per_year;
    d.f0 = market->fwd[0];
    const int NP = problem->n_par;
    d.beta = problem->beta_free ? problem->x0[NP - 1] : problem->beta;
    for (int k = 0; k < base_npar(problem->model); ++k) d.x[k] = problem->x0[k];
    d.key0 = (uint32_t)(mc->seed & 0xffffffffu);
    d.key1 = (uint32_t)(mc->seed >> 32);
    d.anti = mc->scheme == SABR_MC_ANTITHETIC;
    const bool fp32 = precision == SABR_FP32;
    const int64_t tiles = (mc->n_paths + 255) / 256;
    const int n_blocks = (int)std::min<int64_t>(tiles, 2048);
    void *ps, *pq, *pr, *se;
    if ((rc = get_buf(c, S_PART, sizeof(double) * (size_t)n_blocks * g.n_obs, &ps)) ||
        (rc = get_buf(c, S_PARTQ, sizeof(double) * (size_t)n_blocks * g.n_obs, &pq)) ||
        (rc = get_buf(c, S_PRICE, sizeof(double) * g.n_obs, &pr)) || (rc = get_buf(c, S_SE, sizeof(double) * g.n_obs, &se)))
        return rc;
    const void *fn = mc_price_kernel_ptr(fp32);
    const size_t smem = mc_price_smem_bytes(fp32, g.m_max, g.n_obs);
    if ((rc = set_smem(c, fn, smem))) return rc;
    const int32_t *ms = g.msteps, *mo = g.moffs;
    const double *K = g.K;
    void *a1[] = {&d, &ms, &mo, &K, &ps, &pq};
    if ((rc = launch(c, true, "mc_price_kernel", fn, dim3(n_blocks), dim3(256), a1, smem))) return rc;
    int n_obs = g.n_obs;
    int64_t np = mc->n_paths;
    const int32_t *orow = g.obsrow;
    const double *disc = g.disc;
    int nblk = n_blocks;
    int anti = d.anti;
    void *a2[] = {&n_obs, &nblk, &np, &anti, &ps, &pq, &orow, &disc, &pr, &se};
    if ((rc = launch(c, false, "mc_price_finalize", mc_price_finalize_ptr(), dim3((n_obs + 255) / 256), dim3(256), a2, 0)))
        return rc;
    HIPCHK(c, hipMemcpyAsync(price, pr, sizeof(double) * n_obs, hipMemcpyDeviceToHost, c->stream));
    if (std_err) HIPCHK(c, hipMemcpyAsync(std_err, se, sizeof(double) * n_obs, hipMemcpyDeviceToHost, c->stream));
    return sync_and_account(c);
}

int sabr_mc_price_noalloc(sabr_ctx *c, const sabr_market *market, const sabr_problem *problem, const sabr_mc *mc,
                         int32_t precision, double *price, double *std_err) {
    if (!c) return SABR_E_INVAL;
    c->err.clear();
    hipSetDevice(c->device);
    int rc;
    if ((rc = check_problem(c, problem, false))) return rc;
    if (!problem->x0) return fail(c, SABR_E_INVAL, "problem->x0 (the parameters) is NULL");
    if ((rc = check_market(c, market, false, true, SABR_W_ABSOLUTE))) return rc;
    if ((rc = check_mc(c, mc))) return rc;
    if (precision != SABR_FP32 && precision != SABR_FP64) return fail(c, SABR_E_INVAL, "bad precision");
    if (!price) return fail(c, SABR_E_INVAL, "price is NULL");
    const int n_mat = market->n_mat, n_obs = market->offs[n_mat];
    int m_max = 0, prev = 0;
    for (int i = 0; i < n_mat; ++i) {
        const int m = n_steps(market->T[i], mc->steps_per_year);
        if (m < prev) return fail(c, SABR_E_INVAL, "Monte Carlo grids must list maturities in increasing order");
        prev = m;
        m_max = std::max(m_max, m);
    }
    unsigned char *base = c->device < kMaxDevices ? g_scratch[c->device] : nullptr;
    if (!base)
        return fail(c, SABR_E_DEVICE, "no address for the static scratch array on device %d: %s", c->device,
                    hipGetErrorString(c->device < kMaxDevices ? g_scratch_err[c->device] : hipErrorInvalidDevice));
    const int64_t tiles = (mc->n_paths + 255) / 256;
    const int n_blocks = (int)std::min<int64_t>(tiles, 2048);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o_ps = 0, o_pq = o_ps + al(sizeof(double) * (size_t)n_blocks * n_obs);
    const size_t o_pr = o_pq + al(sizeof(double) * (size_t)n_blocks * n_obs);
    const size_t o_se = o_pr + al(sizeof(double) * n_obs), o_K = o_se + al(sizeof(double) * n_obs);
    const size_t o_disc = o_K + al(sizeof(double) * n_obs), o_T = o_disc + al(sizeof(double) * n_mat);
    const size_t o_din = o_T + al(sizeof(double) * n_mat), o_offs = o_din + al(sizeof(double) * n_mat);
    const size_t o_ms = o_offs + al(sizeof(int32_t) * (n_mat + 1)), o_row = o_ms + al(sizeof(int32_t) * n_mat);
    const size_t total = o_row + al(sizeof(int32_t) * n_obs);
    if (total > kScratchBytes)
        return fail(c, SABR_E_BUDGET, "the call needs %zu bytes of device scratch, the static array has %zu", total,
                    kScratchBytes);
    double *ps = (double *)(base + o_ps), *pq = (double *)(base + o_pq), *pr = (double *)(base + o_pr);
    double *se = (double *)(base + o_se), *K = (double *)(base + o_K), *disc = (double *)(base + o_disc);
    double *T = (double *)(base + o_T), *din = market->disc ? (double *)(base + o_din) : nullptr;
    int32_t *offs = (int32_t *)(base + o_offs), *ms = (int32_t *)(base + o_ms), *orow = (int32_t *)(base + o_row);
    // the caller's host arrays go straight to the device (no staging buffer)
    HIPCHK(c, hipMemcpyAsync(T, market->T, sizeof(double) * n_mat, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(offs, market->offs, sizeof(int32_t) * (n_mat + 1), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(K, market->K, sizeof(double) * n_obs, hipMemcpyHostToDevice, c->stream));
    if (din) HIPCHK(c, hipMemcpyAsync(din, market->disc, sizeof(double) * n_mat, hipMemcpyHostToDevice, c->stream));
    int spy = mc->steps_per_year, nm = n_mat;
    void *ag[] = {&nm, &T, &offs, &spy, &din, &ms, &orow, &disc};
    if ((rc = launch(c, false, "mc_grid_kernel", mc_grid_kernel_ptr(), dim3((n_obs + 255) / 256), dim3(256), ag, 0)))
        return rc;
    McDesc d;
    std::memset(&d, 0, sizeof d);
    d.model = problem->model;
    d.n_mat = n_mat;
    d.n_obs = n_obs;
    d.m_max = m_max;
    d.n_paths = mc->n_paths;
    d.dt = 1.0 / (double)mc->steps_per_year;
    d.f0 = market->fwd[0];
    const int NP = problem->n_par;
    d.beta = problem->beta_free ? problem->x0[NP - 1] : problem->beta;
    for (int k = 0; k < base_npar(problem->model); ++k) d.x[k] = problem->x0[k];
    d.key0 = (uint32_t)(mc->seed & 0xffffffffu);
    d.key1 = (uint32_t)(mc->seed >> 32);
    d.anti = mc->scheme == SABR_MC_ANTITHETIC;
    const bool fp32 = precision == SABR_FP32;
    const void *fn = mc_price_kernel_ptr(fp32);
    const size_t smem = mc_price_smem_bytes(fp32, m_max, n_obs);
    if ((rc = set_smem(c, fn, smem))) return rc;
    void *a1[] = {&d, &ms, &offs, &K, &ps, &pq};
    if ((rc = launch(c, false, "mc_price_kernel", fn, dim3(n_blocks), dim3(256), a1, smem))) return rc;
    int no = n_obs, nblk = n_blocks;
    int64_t np = mc->n_paths;
    int anti = d.anti;
    void *a2[] = {&no, &nblk, &np, &anti, &ps, &pq, &orow, &disc, &pr, &se};
    if ((rc = launch(c, false, "mc_price_finalize", mc_price_finalize_ptr(), dim3((n_obs + 255) / 256), dim3(256), a2, 0)))
        return rc;
    HIPCHK(c, hipMemcpyAsync(price, pr, sizeof(double) * n_obs, hipMemcpyDeviceToHost, c->stream));
    if (std_err) HIPCHK(c, hipMemcpyAsync(std_err, se, sizeof(double) * n_obs, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SABR_OK;
}

int sabr_atm_seed(sabr_ctx *c, const sabr_market *market, const sabr_problem *problem, double *x0) {
    if (!c) return SABR_E_INVAL;
    begin_call(c);
    c->err.clear();
    hipSetDevice(c->device);
    int rc;
    if ((rc = check_problem(c, problem, true)) || (rc = check_market(c, market, true, false, SABR_W_ABSOLUTE)))
        return rc;
    if (!x0) return fail(c, SABR_E_INVAL, "x0 is NULL");
    const sabr_market &m = *market;
    for (int i = 0; i < m.n_mat; ++i)
        for (int j = m.offs[i]; j < m.offs[i + 1]; ++j) {
            if (!(m.target[j] > 0)) return fail(c, SABR_E_INVAL, "target[%d] must be a positive vol", j);
            if (j > m.offs[i] && !(m.K[j] > m.K[j - 1]))
                return fail(c, SABR_E_INVAL, "strikes of maturity %d must increase", i);
        }
    const int n_obs = m.offs[m.n_mat];
    std::vector<double> T(m.T, m.T + m.n_mat), fwd(m.fwd, m.fwd + m.n_mat), K(m.K, m.K + n_obs),
        tg(m.target, m.target + n_obs);
    std::vector<int32_t> offs(m.offs, m.offs + m.n_mat + 1);
    double *dT, *dF, *dK, *dV;
    int32_t *dO;
    void *dx;
    if ((rc = upload(c, S_T, T, &dT)) || (rc = upload(c, S_FWD, fwd, &dF)) || (rc = upload(c, S_K, K, &dK)) ||
        (rc = upload(c, S_TARGET, tg, &dV)) || (rc = upload(c, S_OFFS, offs, &dO)) ||
        (rc = get_buf(c, S_X, sizeof(double) * kMaxPar, &dx)))
        return rc;
    AtmDesc d;
    std::memset(&d, 0, sizeof d);
    d.n_mat = m.n_mat;
    d.n_par = problem->n_par;
    d.beta_free = problem->beta_free ? 1 : 0;
    d.beta = problem->beta;
    for (int k = 0; k < problem->n_par; ++k) {
        d.lb[k] = problem->lb[k];
        d.ub[k] = problem->ub[k];
    }
    void *args[] = {&d, &dT, &dF, &dO, &dK, &dV, &dx};
    if ((rc = launch(c, false, "atm_seed_kernel", atm_seed_kernel_ptr(), dim3(1), dim3(64), args, 0))) return rc;
    HIPCHK(c, hipMemcpyAsync(x0, dx, sizeof(double) * problem->n_par, hipMemcpyDeviceToHost, c->stream));
    return sync_and_account(c);
}

int sabr_mc_cliquet(sabr_ctx *c, const sabr_problem *problem, double f0, double disc, int32_t n_reset,
                    const double *reset_T, double local_floor, double local_cap, double global_floor,
                    double global_cap, const sabr_mc *mc, int32_t precision, double *price, double *std_err) {
    if (!c) return SABR_E_INVAL;
    begin_call(c);
    c->err.clear();
    hipSetDevice(c->device);
    int rc;
    if ((rc = check_problem(c, problem, false))) return rc;
    if (!problem->x0) return fail(c, SABR_E_INVAL, "problem->x0 (the parameters) is NULL");
    if ((rc = check_mc(c, mc))) return rc;
    if (precision != SABR_FP32 && precision != SABR_FP64) return fail(c, SABR_E_INVAL, "bad precision");
    if (!price) return fail(c, SABR_E_INVAL, "price is NULL");
    if (!(f0 > 0) || !std::isfinite(f0) || !(disc > 0) || !std::isfinite(disc))
        return fail(c, SABR_E_INVAL, "f0 and disc must be finite and > 0");
    if (n_reset < 2 || !reset_T) return fail(c, SABR_E_INVAL, "a cliquet needs at least two reset dates");
    if (!(local_floor <= local_cap) || !(global_floor <= global_cap) || !std::isfinite(local_floor) || !std::isfinite(local_cap) ||
        !std::isfinite(global_floor) || !std::isfinite(global_cap))
        return fail(c, SABR_E_INVAL, "floors must be finite and not above their caps");
    std::vector<int32_t> rs(n_reset);
    for (int i = 0; i < n_reset; ++i) {
        if (!(reset_T[i] > 0) || !std::isfinite(reset_T[i])) return fail(c, SABR_E_INVAL, "reset_T[%d] must be > 0", i);
        rs[i] = n_steps(reset_T[i], mc->steps_per_year);
        if (i > 0 && rs[i] <= rs[i - 1])
            return fail(c, SABR_E_INVAL, "reset dates must fall on increasing steps of 1/%d y", mc->steps_per_year);
    }
    CliqDesc d;
    std::memset(&d, 0, sizeof d);
    d.model = problem->model;
    d.n_reset = n_reset;
    d.m_max = rs[n_reset - 1];
    d.n_paths = mc->n_paths;
    d.dt = 1.0 / (double)mc->steps_per_year;
    d.f0 = f0;
    const int NP = problem->n_par;
    d.beta = problem->beta_free ? problem->x0[NP - 1] : problem->beta;
    for (int k = 0; k < base_npar(problem->model); ++k) d.x[k] = problem->x0[k];
    d.local_floor = local_floor;
    d.local_cap = local_cap;
    d.global_floor = global_floor;
    d.global_cap = global_cap;
    d.key0 = (uint32_t)(mc->seed & 0xffffffffu);
    d.key1 = (uint32_t)(mc->seed >> 32);
    d.anti = mc->scheme == SABR_MC_ANTITHETIC;
    const bool fp32 = precision == SABR_FP32;
    const int64_t tiles = (mc->n_paths + 255) / 256;
    const int n_blocks = (int)std::min<int64_t>(tiles, 2048);
    int32_t *drs, *drow;
    double *ddisc;
    void *ps, *pq, *pr, *se;
    std::vector<int32_t> row0(1, 0);
    std::vector<double> dv(1, disc);
    if ((rc = upload(c, S_RESET, rs, &drs)) || (rc = upload(c, S_OBSROW, row0, &drow)) ||
        (rc = upload(c, S_DISC, dv, &ddisc)) || (rc = get_buf(c, S_PART, sizeof(double) * (size_t)n_blocks, &ps)) ||
        (rc = get_buf(c, S_PARTQ, sizeof(double) * (size_t)n_blocks, &pq)) ||
        (rc = get_buf(c, S_PRICE, sizeof(double), &pr)) || (rc = get_buf(c, S_SE, sizeof(double), &se)))
        return rc;
    const void *fn = mc_cliquet_kernel_ptr(fp32);
    const size_t smem = mc_cliquet_smem_bytes(fp32, d.m_max);
    if ((rc = set_smem(c, fn, smem))) return rc;
    void *a1[] = {&d, &drs, &ps, &pq};
    if ((rc = launch(c, true, "mc_cliquet_kernel", fn, dim3(n_blocks), dim3(256), a1, smem))) return rc;
    int one = 1, nblk = n_blocks;
    int64_t np = mc->n_paths;
    int anti = d.anti;
    void *a2[] = {&one, &nblk, &np, &anti, &ps, &pq, &drow, &ddisc, &pr, &se};
    if ((rc = launch(c, false, "mc_price_finalize", mc_price_finalize_ptr(), dim3(1), dim3(64), a2, 0))) return rc;
    HIPCHK(c, hipMemcpyAsync(price, pr, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (std_err) HIPCHK(c, hipMemcpyAsync(std_err, se, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return sync_and_account(c);
}

}  // extern "C"
