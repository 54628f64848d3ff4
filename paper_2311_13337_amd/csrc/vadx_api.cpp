// vadx_api.cpp -- host side of the C ABI declared in include/vadx.h: argument
// checks, model conversion, connectome and batch bookkeeping, the workspace
// planner (instance grouping, ring depths, delay tables) and the launch
// sequence of one run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "analysis_engine.h"
#include "engine.h"
#include "kmodel.h"
#include "mlp_engine.h"
#include "vadx.h"

using namespace vadx;

namespace {

// Groups sharing a block length: [first, first + n_groups) of the group table
// (one launch of workgroups of `threads` lanes each in the one-workgroup-per-
// group mode; the persistent launch takes every class at once).
struct BlockClass {
    int block;
    int32_t first, n_groups;
    int threads;
};

struct HostConn {
    int32_t n = 0, nnz = 0;
    double len_min = 0.0, len_max = 0.0;   // over edges with w != 0
    int64_t row_off = 0, edge_off = 0, sc_off = 0;
    int64_t ref_off = -1;                  // reference FC slot (floats), -1: none
    int64_t ref_slot = -1;                 // slot reserved at the first reference
};

template <class T> struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t count)
    {
        if (count <= n && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc((void **)&p, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) n = count;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

} // namespace

struct vadx_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    vadx_model model{};
    bool have_model = false;
    // connectomes (device copies grow as connectomes are added)
    std::vector<HostConn> conns;
    std::vector<int32_t> h_rowptr_sizes;
    int64_t total_rows = 0, total_edges = 0, total_sc = 0;
    DevBuf<int32_t> rowptr, colidx;
    DevBuf<float> weight;
    DevBuf<double> edge_len, sc;
    DevBuf<ConnDev> d_conns;
    DevBuf<float> refs;                  // reference FC matrices (fitness)
    int64_t total_ref = 0;
    // ranking (vadx_top_k)
    SelScratch sel;
    DevBuf<int64_t> topk_idx;
    // BOLD tables
    DevBuf<int64_t> b_samp, b_out;
    DevBuf<int32_t> b_n, b_rbase, b_reg, b_emit;
    // batch
    std::vector<float> S, be, ae, v;
    std::vector<int32_t> conn_of;
    std::vector<uint32_t> noise_key;     // Philox key word per instance (default: batch index)
    std::vector<double> iparam[6];       // per-instance model parameters (empty: the model's)
    bool batch_same = true;              // every instance's populations see the same inputs
    std::vector<int64_t> traced;
    // plan
    bool planned = false;
    vadx_run plan_run{};
    int block = 1;                       // longest block length of the plan
    int block_lcm = 1;                   // least common multiple of the plan's block lengths
    int wg_threads = 64;                 // widest workgroup of the plan
    std::vector<BlockClass> classes;     // groups of one block length, launched together
    std::vector<InstDev> h_inst;
    std::vector<int32_t> h_perm;
    std::vector<GroupDev> h_groups;
    std::vector<DelayTableDev> h_tables;
    int max_nnz = 0;
    int64_t packed_total = 0;
    int64_t n_samples = 0;
    size_t ws_bytes = 0;
    size_t off_stats = 0, off_flags = 0, off_queue = 0;
    DevBuf<InstDev> d_inst;
    DevBuf<int32_t> d_perm;
    DevBuf<GroupDev> d_groups;
    DevBuf<DelayTableDev> d_tables;
    DevBuf<int32_t> d_packed;
    DevBuf<KModel> d_kmodel;             // model constants of the run being integrated
    // last run
    void *ws = nullptr;
    bool ran = false;
    // timing
    bool timing = false;
    int64_t n_int = 0, n_fc = 0;
    double ms_int = 0.0, ms_fc = 0.0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_int, ev_fc;
    AnTimer an_timer;                    // analysis launches (when timing is on)
    // launch shape: 0 = persistent work queue (default), 1 = one workgroup per group
    int launch_mode = 0;
    // graph replay of whole runs
    bool use_graph = false;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;
    void *g_ws = nullptr;
    uint64_t g_epoch = 0, plan_epoch = 0;
    int wg_instances_override = 0;
    int wg_lanes = 256;                  // lane budget per workgroup (autotuned)
    std::map<int, int> class_lanes;      // lane budget per region count (autotuned; else wg_lanes)
    int occ = 2;                         // waves per SIMD of the persistent kernel (autotuned)
    int slack = 0;                       // half-length blocks where they stay long (autotuned)
    int item_steps = 1000;
    int cus = 0;
};

// Per-device address of the scratch array of vadx_top_k_noalloc (defined below).
static hipError_t noalloc_scratch(int device, void **p);

// Errors of calls made without a context (vadx_create) land here.
static thread_local std::string g_err = "";

static vadx_status fail(vadx_ctx *c, vadx_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    else g_err = buf;
    return st;
}

#define HIP_TRY(c, expr)                                                                       \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((c), e_ == hipErrorOutOfMemory ? VADX_E_OOM : VADX_E_HIP, "%s: %s", #expr, \
                        hipGetErrorString(e_));                                                \
    } while (0)

static const double kRS[10] = {-48.9, 5.1, -25.0, 1.4, -0.41, 10.5, -36.0, 7.4, 1.2, 40.7};
static const double kFS[10] = {-51.4, 0.4, -8.3, 0.2, -0.5, 1.4, -14.6, 4.5, 2.8, 15.3};

extern "C" {

vadx_status vadx_model_defaults(int preset, vadx_model *m)
{
    if (!m || (preset != VADX_PRESET_LITERATURE_B && preset != VADX_PRESET_PAPER_T1))
        return VADX_E_ARG;
    std::memset(m, 0, sizeof(*m));
    m->C_m = 200.0; m->g_L = 10.0; m->E_e = 0.0; m->E_i = -80.0;
    m->Q_e = 1.5; m->Q_i = 5.0; m->tau_e = 5.0; m->tau_i = 5.0;
    m->K_e = 400.0; m->K_i = 100.0; m->N_e = 8000.0; m->N_i = 2000.0; m->T = 20.0;
    m->E_L_e = -64.0; m->E_L_i = -65.0; m->tau_w_e = 500.0; m->tau_w_i = 1.0;
    m->b_i = 0.0; m->a_i = 0.0;
    m->cF_ee = 0.5e-3; m->cF_ei = 0.0; m->cF_ie = 0.5e-3; m->cF_ii = 0.0;   // Table 4's upper drive
    m->tau_OU = 5.0; m->sigma_OU = 1e-3; m->w_noise = 1e-3;
    m->muV0 = -60.0; m->dmuV0 = 10.0; m->sV0 = 4.0; m->dsV0 = 6.0; m->tN0 = 0.5; m->dtN0 = 1.0;
    m->rate_max = 1.0; m->E_init = 0.004; m->I_init = 0.01; m->x_floor = 1e-6;
    std::memcpy(m->P_e, kRS, sizeof(kRS));
    std::memcpy(m->P_i, kFS, sizeof(kFS));
    if (preset == VADX_PRESET_LITERATURE_B) {
        m->P_e[0] = -49.8;
        m->P_i[1] = 4.0;
        m->P_e[9] = -m->P_e[9];
        m->P_i[9] = -m->P_i[9];
    }
    return VADX_OK;
}

vadx_status vadx_create(int device, void *hip_stream, vadx_ctx **out)
{
    if (!out) return fail(nullptr, VADX_E_ARG, "null output");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0)
        return fail(nullptr, VADX_E_HIP, "hipGetDeviceCount: %s (%d devices)", hipGetErrorString(e), ndev);
    if (device < 0 || device >= ndev) return fail(nullptr, VADX_E_ARG, "device %d out of range", device);
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, VADX_E_HIP, "hipSetDevice: %s", hipGetErrorString(e));
    void *scratch_p = nullptr;
    e = noalloc_scratch(device, &scratch_p);
    if (e != hipSuccess)
        return fail(nullptr, VADX_E_HIP, "address of the top-k scratch: %s", hipGetErrorString(e));
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess || cus <= 0) return fail(nullptr, VADX_E_HIP, "CU count: %s", hipGetErrorString(e));
    vadx_ctx *c = new vadx_ctx();
    c->device = device;
    c->cus = cus;
    c->stream = (hipStream_t)hip_stream;
    vadx_model_defaults(VADX_PRESET_LITERATURE_B, &c->model);
    c->have_model = true;
    *out = c;
    return VADX_OK;
}

void vadx_destroy(vadx_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto &e : c->ev_int) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto &e : c->ev_fc) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto &v : c->an_timer.ev)
        for (auto &e : v) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    c->rowptr.release(); c->colidx.release(); c->weight.release(); c->edge_len.release();
    c->sc.release(); c->d_conns.release(); c->d_inst.release(); c->d_perm.release();
    c->d_groups.release(); c->d_tables.release(); c->d_packed.release(); c->d_kmodel.release();
    delete c;
}

const char *vadx_last_error(const vadx_ctx *c)
{
    if (!c) return g_err.c_str();
    return c->err.c_str();
}

static bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

vadx_status vadx_set_model(vadx_ctx *c, const vadx_model *m)
{
    if (!c || !m) return fail(c, VADX_E_ARG, "null argument");
    const double pos[] = {m->C_m, m->g_L, m->Q_e, m->Q_i, m->tau_e, m->tau_i, m->K_e, m->K_i,
                          m->N_e, m->N_i, m->T, m->tau_w_e, m->tau_w_i, m->tau_OU, m->dmuV0,
                          m->dsV0, m->dtN0, m->rate_max};
    for (double x : pos)
        if (!(std::isfinite(x) && x > 0.0)) return fail(c, VADX_E_ARG, "model constant must be > 0");
    const double any[] = {m->E_e, m->E_i, m->E_L_e, m->E_L_i, m->b_i, m->a_i, m->cF_ee, m->cF_ei,
                          m->cF_ie, m->cF_ii, m->sigma_OU, m->w_noise, m->muV0, m->sV0, m->tN0,
                          m->E_init, m->I_init, m->x_floor};
    for (double x : any)
        if (!std::isfinite(x)) return fail(c, VADX_E_ARG, "model constant not finite");
    for (int i = 0; i < 10; ++i)
        if (!std::isfinite(m->P_e[i]) || !std::isfinite(m->P_i[i]))
            return fail(c, VADX_E_ARG, "threshold coefficient not finite");
    if (!(m->x_floor > 0.0)) return fail(c, VADX_E_ARG, "x_floor must be > 0");
    if (m->E_init < 0 || m->E_init > m->rate_max || m->I_init < 0 || m->I_init > m->rate_max)
        return fail(c, VADX_E_ARG, "initial rates outside [0, rate_max]");
    c->model = *m;
    c->have_model = true;
    ++c->plan_epoch;   // a recorded run graph holds the previous constants
    return VADX_OK;
}

// Device copy of the connectome table (after a connectome or a reference changes).
static vadx_status upload_conns(vadx_ctx *c)
{
    std::vector<ConnDev> dc;
    for (auto &h : c->conns)
        dc.push_back(ConnDev{h.n, h.nnz, h.row_off, h.edge_off, h.sc_off, h.ref_off});
    HIP_TRY(c, c->d_conns.ensure(dc.size()));
    HIP_TRY(c, hipMemcpyAsync(c->d_conns.p, dc.data(), dc.size() * sizeof(ConnDev),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return VADX_OK;
}

vadx_status vadx_add_connectome(vadx_ctx *c, int32_t n, const double *w, const double *len,
                                int32_t *conn_id)
{
    if (!c || !w || !len || !conn_id) return fail(c, VADX_E_ARG, "null argument");
    if (n < 2) return fail(c, VADX_E_ARG, "need at least 2 regions");
    if (n > 512)
        return fail(c, VADX_E_UNSUPPORTED,
                    "at most 512 regions per connectome (one lane per region, whole instances per workgroup)");
    HostConn hc;
    hc.n = n;
    int64_t nnz = 0;
    double lmin = INFINITY, lmax = 0.0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j) {
            const double x = w[(int64_t)k * n + j], L = len[(int64_t)k * n + j];
            if (!finite_nonneg(x)) return fail(c, VADX_E_ARG, "weights must be finite and >= 0");
            if (!std::isfinite(L) || L < 0.0) return fail(c, VADX_E_ARG, "tract lengths must be finite and >= 0");
            if (x != 0.0) {
                if (k == j) return fail(c, VADX_E_ARG, "self-connection w[%d][%d] != 0", k, k);
                if (!(L > 0.0)) return fail(c, VADX_E_ARG, "edge %d-%d has no positive length", k, j);
                ++nnz;
                lmin = std::min(lmin, L);
                lmax = std::max(lmax, L);
            }
        }
    hc.nnz = (int32_t)nnz;
    hc.len_min = nnz ? lmin : 0.0;
    hc.len_max = lmax;
    hc.row_off = c->total_rows;
    hc.edge_off = c->total_edges;
    hc.sc_off = c->total_sc;
    HIP_TRY(c, hipSetDevice(c->device));
    // grow device arrays, keeping earlier connectomes
    auto grow = [&](auto &buf, size_t need) -> hipError_t {
        using T = std::remove_pointer_t<decltype(buf.p)>;
        if (need <= buf.n) return hipSuccess;
        T *np = nullptr;
        hipError_t e = hipMalloc((void **)&np, need * sizeof(T) * 2);
        if (e != hipSuccess) return e;
        if (buf.p) {
            e = hipMemcpyAsync(np, buf.p, buf.n * sizeof(T), hipMemcpyDeviceToDevice, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            (void)hipFree(buf.p);
            if (e != hipSuccess) { (void)hipFree(np); buf.p = nullptr; buf.n = 0; return e; }
        }
        buf.p = np;
        buf.n = need * 2;
        return hipSuccess;
    };
    HIP_TRY(c, grow(c->rowptr, (size_t)(c->total_rows + n + 1)));
    HIP_TRY(c, grow(c->colidx, (size_t)(c->total_edges + nnz + 1)));
    HIP_TRY(c, grow(c->weight, (size_t)(c->total_edges + nnz + 1)));
    HIP_TRY(c, grow(c->edge_len, (size_t)(c->total_edges + nnz + 1)));
    HIP_TRY(c, grow(c->sc, (size_t)(c->total_sc + (int64_t)n * n)));
    double *dlen = nullptr;
    HIP_TRY(c, hipMalloc((void **)&dlen, sizeof(double) * n * n));
    hipError_t e = hipMemcpyAsync(c->sc.p + hc.sc_off, w, sizeof(double) * n * n,
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(dlen, len, sizeof(double) * n * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = launch_conn_prepare(n, c->sc.p + hc.sc_off, dlen, c->rowptr.p + hc.row_off,
                                c->weight.p + hc.edge_off, c->edge_len.p + hc.edge_off,
                                c->colidx.p + hc.edge_off, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(dlen);
    if (e != hipSuccess) return fail(c, VADX_E_HIP, "connectome upload: %s", hipGetErrorString(e));
    c->total_rows += n + 1;
    c->total_edges += nnz;
    c->total_sc += (int64_t)n * n;
    c->conns.push_back(hc);
    vadx_status st = upload_conns(c);
    if (st) return st;
    *conn_id = (int32_t)c->conns.size() - 1;
    c->planned = false;
    return VADX_OK;
}

vadx_status vadx_set_batch(vadx_ctx *c, int64_t n, const float *S, const float *b_e,
                           const float *a_e, const float *v, const int32_t *conn)
{
    if (!c) return VADX_E_ARG;
    if (n < 0 || (n > 0 && (!S || !b_e || !a_e || !v))) return fail(c, VADX_E_ARG, "bad batch arrays");
    if (n > (int64_t)1 << 31) return fail(c, VADX_E_UNSUPPORTED, "batch too large");
    for (int64_t i = 0; i < n; ++i) {
        if (!finite_nonneg(S[i])) return fail(c, VADX_E_ARG, "S[%lld] must be finite and >= 0", (long long)i);
        if (!std::isfinite(b_e[i]) || !std::isfinite(a_e[i]))
            return fail(c, VADX_E_ARG, "b_e/a_e[%lld] not finite", (long long)i);
        if (!(std::isfinite(v[i]) && v[i] > 0.0f))
            return fail(c, VADX_E_ARG, "v[%lld] must be finite and > 0", (long long)i);
        const int32_t ci = conn ? conn[i] : 0;
        if (ci < 0 || ci >= (int32_t)c->conns.size())
            return fail(c, VADX_E_ARG, "conn_id[%lld] = %d unknown", (long long)i, ci);
    }
    c->S.assign(S, S + n);
    c->be.assign(b_e, b_e + n);
    c->ae.assign(a_e, a_e + n);
    c->v.assign(v, v + n);
    c->conn_of.assign((size_t)n, 0);
    if (conn) c->conn_of.assign(conn, conn + n);
    c->noise_key.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) c->noise_key[(size_t)i] = (uint32_t)i;
    for (auto &p : c->iparam) p.clear();
    c->traced.clear();
    c->planned = false;
    c->ran = false;
    return VADX_OK;
}

vadx_status vadx_set_noise_keys(vadx_ctx *c, int64_t n, const uint32_t *keys)
{
    if (!c) return VADX_E_ARG;
    if (n != (int64_t)c->S.size() || (n > 0 && !keys))
        return fail(c, VADX_E_ARG, "need one noise key per instance of the batch");
    c->noise_key.assign(keys, keys + n);
    c->planned = false;
    c->ran = false;
    return VADX_OK;
}

vadx_status vadx_set_trace(vadx_ctx *c, int64_t n, const int64_t *inst)
{
    if (!c || n < 0 || n > 1024 || (n > 0 && !inst)) return fail(c, VADX_E_ARG, "bad trace selection");
    for (int64_t i = 0; i < n; ++i)
        if (inst[i] < 0 || inst[i] >= (int64_t)c->S.size())
            return fail(c, VADX_E_ARG, "trace instance %lld out of range", (long long)inst[i]);
    c->traced.assign(inst, inst + n);
    c->planned = false;
    return VADX_OK;
}

static bool run_ok(vadx_ctx *c, const vadx_run *r)
{
    if (!r) return false;
    if (!(std::isfinite(r->dt_ms) && r->dt_ms > 0.0)) return false;
    if (r->n_steps < 0 || r->transient_steps < 0 || r->tavg_steps <= 0 || r->n_trace_steps < 0)
        return false;
    if (r->transient_steps > r->n_steps) return false;
    if (r->integrator != VADX_HEUN && r->integrator != VADX_EULER) return false;
    if (r->chunk_steps < 0) return false;
    if (!(std::isfinite(r->fc_min_std) && r->fc_min_std >= 0.0)) return false;
    (void)c;
    return true;
}

// Delay in steps as the delays kernel computes it (FP64, round half to even).
static int64_t host_delay(double L, float v, double dt)
{
    double q = std::nearbyint(L / ((double)v * dt));
    return q < 1.0 ? 1 : (int64_t)q;
}

vadx_status vadx_plan(vadx_ctx *c, const vadx_run *r, size_t *bytes)
{
    if (!c || !bytes) return fail(c, VADX_E_ARG, "null argument");
    if (!run_ok(c, r)) return fail(c, VADX_E_ARG, "invalid run settings");
    const int64_t ni = (int64_t)c->S.size();
    if (ni == 0) return fail(c, VADX_E_STATE, "no batch set");
    const int64_t ns = (r->n_steps - r->transient_steps) / r->tavg_steps;
    // ring depths and block lengths: a block of B steps from step s reads
    // histories up to slot s + B - 1 - d_min, so B <= d_min + 1 (each
    // instance's own shortest delay) keeps every read at or before the block's
    // first slot. The waves of a group wait before a block only until the
    // others have written that slot (d_min of the group), so they may drift up
    // to d_min + 1 - B steps apart; with wave slack B <= (d_min + 1) / 2 where
    // that is still >= kSlackMinBlock steps. A wave then writes at most
    // d_min + 1 slots ahead of the next block start of any other wave of its
    // instance, which reads back to d_max slots before that: rings hold
    // d_max + d_min + 2 slots.
    std::vector<int64_t> dmax(ni), dmin(ni);
    std::vector<int> blk(ni);
    int bmax = 1;
    for (int64_t i = 0; i < ni; ++i) {
        const HostConn &hc = c->conns[c->conn_of[i]];
        const int64_t dm = hc.nnz ? host_delay(hc.len_min, c->v[i], r->dt_ms) : 1;
        dmax[i] = hc.nnz ? host_delay(hc.len_max, c->v[i], r->dt_ms) : 1;
        dmin[i] = std::min(dm, dmax[i]);
        if (dmax[i] >= (1 << 20) - 2 * kMaxBlock - 2)
            return fail(c, VADX_E_UNSUPPORTED, "delay of %lld steps too long", (long long)dmax[i]);
        // the longest of 1, 2, 4, 8, 12, 16, 24, 32 steps within the bound
        int B = 1, Bh = 1;
        for (int cand : {2, 4, 8, 12, 16, 24, 32}) {
            if (cand <= kMaxBlock && cand <= dm + 1) B = cand;
            if (cand <= kMaxBlock && 2 * cand <= dm + 1) Bh = cand;
        }
        blk[i] = (c->slack && Bh >= kSlackMinBlock) ? Bh : B;
        bmax = std::max(bmax, blk[i]);
    }
    c->block = bmax;
    // launch and item lengths are multiples of every block length present
    c->block_lcm = 1;
    for (int64_t i = 0; i < ni; ++i) c->block_lcm = std::lcm(c->block_lcm, blk[i]);
    // delay tables: one per distinct (connectome, speed)
    std::map<std::pair<int32_t, uint32_t>, int32_t> tab;
    c->h_tables.clear();
    std::vector<int32_t> tab_of(ni);
    int64_t poff = 0;
    c->max_nnz = 0;
    for (int64_t i = 0; i < ni; ++i) {
        uint32_t vb;
        std::memcpy(&vb, &c->v[i], 4);
        auto key = std::make_pair(c->conn_of[i], vb);
        auto it = tab.find(key);
        if (it == tab.end()) {
            const HostConn &hc = c->conns[c->conn_of[i]];
            DelayTableDev t{c->conn_of[i], c->v[i], poff};
            poff += hc.nnz;
            c->max_nnz = std::max(c->max_nnz, hc.nnz);
            it = tab.emplace(key, (int32_t)c->h_tables.size()).first;
            c->h_tables.push_back(t);
        }
        tab_of[i] = it->second;
    }
    c->packed_total = poff;
    // groups: instances of one block length and one connectome, ordered by ring
    // depth, up to `per` instances (and the lane budget) per workgroup; one
    // launch per block length (longest first)
    std::vector<int32_t> order(ni);
    for (int64_t i = 0; i < ni; ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (blk[a] != blk[b]) return blk[a] > blk[b];
        if (c->conn_of[a] != c->conn_of[b]) return c->conn_of[a] < c->conn_of[b];
        if (dmin[a] != dmin[b]) return dmin[a] < dmin[b];
        return dmax[a] < dmax[b];
    });
    c->h_groups.clear();
    c->h_perm = order;
    c->classes.clear();
    for (int64_t s = 0; s < ni;) {
        const int32_t cid = c->conn_of[order[s]];
        const int B = blk[order[s]];
        const int n = c->conns[cid].n;
        const auto cl = c->class_lanes.find(n);
        int per = std::max(1, (cl != c->class_lanes.end() ? cl->second : c->wg_lanes) / n);
        if (c->wg_instances_override > 0) per = std::min(per, c->wg_instances_override);
        int64_t e = s;
        int64_t gmin = dmin[order[s]];
        while (e < ni && e - s < per && c->conn_of[order[e]] == cid && blk[order[e]] == B) {
            gmin = std::min(gmin, dmin[order[e]]);
            ++e;
        }
        if (c->classes.empty() || c->classes.back().block != B)
            c->classes.push_back(BlockClass{B, (int32_t)c->h_groups.size(), 0, 64});
        BlockClass &bc = c->classes.back();
        c->h_groups.push_back(GroupDev{(int32_t)s, (int32_t)(e - s), n, B, (int32_t)gmin});
        bc.n_groups += 1;
        bc.threads = std::max(bc.threads, (int)(((e - s) * n + 63) / 64 * 64));
        s = e;
    }
    // within each block length, the groups of different connectomes take
    // turns in the queue, so that the workgroups sharing a CU tend to hold
    // rows of different lengths and their gathers' memory waits overlap less
    // (uneven batch: 1 % faster; results do not depend on the order)
    for (BlockClass &bc : c->classes) {
        std::vector<GroupDev> g(c->h_groups.begin() + bc.first, c->h_groups.begin() + bc.first + bc.n_groups);
        std::map<int, std::vector<GroupDev>> by_conn;
        for (const GroupDev &x : g) by_conn[c->conn_of[c->h_perm[x.first]]].push_back(x);
        std::vector<GroupDev> turns;
        for (size_t r = 0; turns.size() < g.size(); ++r)
            for (auto &kv : by_conn)
                if (r < kv.second.size()) turns.push_back(kv.second[r]);
        std::copy(turns.begin(), turns.end(), c->h_groups.begin() + bc.first);
    }
    c->wg_threads = 64;
    for (const BlockClass &bc : c->classes) c->wg_threads = std::max(c->wg_threads, bc.threads);
    // workspace layout (floats unless noted), each section 256-byte aligned
    c->h_inst.assign(ni, InstDev{});
    int64_t f_state = 0, f_acc = 0, f_ring = 0, f_samp = 0, f_fc = 0, f_trace = 0;
    for (int64_t i = 0; i < ni; ++i) {
        const HostConn &hc = c->conns[c->conn_of[i]];
        InstDev &d = c->h_inst[i];
        d.S = c->S[i]; d.be = c->be[i]; d.ae = c->ae[i];
        auto ip = [&](int p, double model_value) {
            return c->iparam[p].empty() ? model_value : c->iparam[p][(size_t)i];
        };
        d.w_noise = (float)ip(VADX_P_W_NOISE, c->model.w_noise);
        d.inv_tauw_e = (float)(1.0 / ip(VADX_P_TAU_W_E, c->model.tau_w_e));
        d.cF[0] = (float)ip(VADX_P_CF_EE, c->model.cF_ee);
        d.cF[1] = (float)ip(VADX_P_CF_EI, c->model.cF_ei);
        d.cF[2] = (float)ip(VADX_P_CF_IE, c->model.cF_ie);
        d.cF[3] = (float)ip(VADX_P_CF_II, c->model.cF_ii);
        d.n = hc.n;
        d.D = (int32_t)(dmax[i] + dmin[i] + 2);
        d.Dp = d.D + blk[i] - 1;
        d.conn = c->conn_of[i];
        d.id = c->noise_key[(size_t)i];
        d.table_off = c->h_tables[tab_of[i]].off;
        d.trace_off = -1;
        d.state_off = f_state; f_state += 16LL * hc.n;   // 8 doubles per region
        d.acc_off = f_acc; f_acc += hc.n;
        d.ring_off = f_ring; f_ring += (int64_t)hc.n * d.Dp;
        d.samp_off = f_samp; f_samp += (ns > 0 ? ns : 0) * hc.n;
        d.fc_off = f_fc; f_fc += (int64_t)hc.n * hc.n;
    }
    c->batch_same = true;
    for (const auto &d : c->h_inst)
        if (!(d.cF[0] == d.cF[2] && d.cF[1] == d.cF[3])) c->batch_same = false;
    if (r->n_trace_steps > 0)
        for (int64_t t : c->traced) {
            InstDev &d = c->h_inst[t];
            d.trace_off = f_trace;
            f_trace += r->n_trace_steps * 8 * d.n;
        }
    size_t off = 0;
    auto section = [&](int64_t floats) { size_t o = off; off = align_up(off + floats * 4, 256); return o; };
    const size_t o_state = section(f_state), o_acc = section(f_acc), o_ring = section(f_ring);
    const size_t o_samp = section(f_samp), o_fc = section(f_fc), o_trace = section(f_trace);
    c->off_stats = off; off = align_up(off + (size_t)ni * sizeof(vadx_stats), 256);
    c->off_flags = off; off = align_up(off + (size_t)ni * 4, 256);
    c->off_queue = off; off = align_up(off + (size_t)(c->h_groups.size() + 2) * 4, 256);
    for (auto &d : c->h_inst) {
        d.state_off += o_state / 4; d.acc_off += o_acc / 4; d.ring_off += o_ring / 4;
        d.samp_off += o_samp / 4; d.fc_off += o_fc / 4;
        if (d.trace_off >= 0) d.trace_off += o_trace / 4;
    }
    c->n_samples = ns > 0 ? ns : 0;
    c->ws_bytes = off;
    // device metadata
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, c->d_inst.ensure(ni));
    HIP_TRY(c, c->d_perm.ensure(ni));
    HIP_TRY(c, c->d_groups.ensure(c->h_groups.size()));
    HIP_TRY(c, c->d_tables.ensure(c->h_tables.size()));
    HIP_TRY(c, c->d_packed.ensure((size_t)std::max<int64_t>(c->packed_total, 1)));
    HIP_TRY(c, c->d_kmodel.ensure(1));
    HIP_TRY(c, hipMemcpyAsync(c->d_inst.p, c->h_inst.data(), ni * sizeof(InstDev), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_perm.p, c->h_perm.data(), ni * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_groups.p, c->h_groups.data(), c->h_groups.size() * sizeof(GroupDev), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->d_tables.p, c->h_tables.data(), c->h_tables.size() * sizeof(DelayTableDev), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, launch_delays((int)c->h_tables.size(), c->d_tables.p, c->d_conns.p, c->colidx.p,
                             c->edge_len.p, r->dt_ms, c->d_packed.p, c->max_nnz, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->plan_run = *r;
    c->planned = true;
    ++c->plan_epoch;
    c->ran = false;
    *bytes = c->ws_bytes;
    return VADX_OK;
}

static vadx_status record(vadx_ctx *c, std::vector<std::pair<hipEvent_t, hipEvent_t>> &evs,
                          hipEvent_t *start)
{
    hipEvent_t a, b;
    HIP_TRY(c, hipEventCreate(&a));
    HIP_TRY(c, hipEventCreate(&b));
    evs.emplace_back(a, b);
    HIP_TRY(c, hipEventRecord(a, c->stream));
    *start = b;
    return VADX_OK;
}

// Enqueues one whole run (flag clear, integration chunks, FC and statistics)
// on `st`. With timing on, events bracket the launches (eager runs only).
static vadx_status enqueue_run(vadx_ctx *c, const vadx_run *r, void *ws, hipStream_t st,
                               bool timed)
{
    const int64_t ni = (int64_t)c->S.size();
    uint32_t *flags = (uint32_t *)((char *)ws + c->off_flags);
    HIP_TRY(c, launch_fill_u32(flags, ni, 0u, st));
    IntegrateArgs a{};
    a.M = make_kmodel(c->model);
    a.M.same_inputs = c->batch_same ? 1 : 0;
    HIP_TRY(c, launch_kmodel_store(a.M, c->d_kmodel.p, st));
    a.Mp = c->d_kmodel.p;
    a.inst = c->d_inst.p;
    a.perm = c->d_perm.p;
    a.groups = c->d_groups.p;
    a.conns = c->d_conns.p;
    a.rowptr = c->rowptr.p;
    a.weight = c->weight.p;
    a.packed = c->d_packed.p;
    a.ws = (float *)ws;
    a.flags = flags;
    a.n_steps_total = r->n_steps;
    a.transient_steps = r->transient_steps;
    a.tavg_steps = r->tavg_steps;
    a.n_trace_steps = r->n_trace_steps;
    a.n_samples = c->n_samples;
    a.dt = r->dt_ms;
    a.gdw_scale = r->noise_off ? 0.0 : c->model.sigma_OU / c->model.tau_OU * std::sqrt(r->dt_ms);
    a.E_init = c->model.E_init;
    a.I_init = c->model.I_init;
    a.seed = r->seed;
    a.integrator = r->integrator;
    // default launch length: the whole run for the persistent queue (its only
    // tail is then the end of the run), 10000 steps for one-workgroup-per-group.
    // Launch and item lengths are multiples of every block length of the plan
    // (their least common multiple), so blocks stay whole inside a run.
    int64_t chunk = r->chunk_steps > 0 ? r->chunk_steps
                                       : (c->launch_mode == 0 ? std::max<int64_t>(r->n_steps, 1) : 10000);
    // (a launch that reaches the end of the run may end on a partial block)
    const int64_t bl = c->block_lcm;
    chunk = chunk >= r->n_steps ? std::max<int64_t>(r->n_steps, 1)
                                : std::max<int64_t>(chunk / bl, 1) * bl;
    const int64_t item_steps = std::max<int64_t>(c->item_steps / bl, 1) * bl;
    uint32_t *status = (uint32_t *)((char *)ws + c->off_queue) + 1;
    HIP_TRY(c, launch_fill_u32(status, 1, 0u, st));
    a.status = status;
    a.wait_spins = 1u << 24;
    for (int64_t n0 = 0; n0 < r->n_steps; n0 += chunk) {
        a.n_begin = n0;
        a.n_end = std::min<int64_t>(r->n_steps, n0 + chunk);
        if (c->launch_mode == 0) {
            // one persistent launch over the groups of every block length
            a.block = c->block;
            a.groups = c->d_groups.p;
            const int ng = (int)c->h_groups.size();
            hipEvent_t stop = nullptr;
            if (timed) { vadx_status e = record(c, c->ev_int, &stop); if (e) return e; }
            int *qb = (int *)((char *)ws + c->off_queue);
            QueueArgs q{};
            q.next = qb;
            q.status = status;
            q.done = qb + 2;
            q.n_groups = ng;
            q.item_steps = item_steps;
            q.max_spins = 1u << 26;
            const int per_cu = persistent_blocks_per_cu(c->block, c->wg_threads, c->occ);
            if (per_cu <= 0)
                return fail(c, VADX_E_UNSUPPORTED, "workgroup of %d threads does not fit a CU", c->wg_threads);
            const int grid = std::min(ng, per_cu * c->cus);
            q.n_items = (int)(ng * ((a.n_end - a.n_begin + q.item_steps - 1) / q.item_steps));
            HIP_TRY(c, launch_integrate_persistent(a, c->wg_threads, q, grid, c->occ, st));
            if (timed) HIP_TRY(c, hipEventRecord(stop, st));
            continue;
        }
        // one launch per block length, longest first, on the same stream
        for (const BlockClass &bc : c->classes) {
            a.block = bc.block;
            a.groups = c->d_groups.p + bc.first;
            const int ng = bc.n_groups;
            hipEvent_t stop = nullptr;
            if (timed) { vadx_status e = record(c, c->ev_int, &stop); if (e) return e; }
            HIP_TRY(c, launch_integrate(a, ng, bc.threads, st));
            if (timed) HIP_TRY(c, hipEventRecord(stop, st));
        }
    }
    FcArgs f{};
    f.inst = c->d_inst.p;
    f.conns = c->d_conns.p;
    f.sc = c->sc.p;
    f.ref = c->refs.p;
    f.ws = (float *)ws;
    f.stats = (float *)((char *)ws + c->off_stats);
    f.flags = flags;
    f.n_samples = c->n_samples;
    f.min_var = r->fc_min_std * r->fc_min_std;
    f.max_n = 1;
    for (const HostConn &hc : c->conns) f.max_n = std::max(f.max_n, hc.n);
    hipEvent_t stop = nullptr;
    if (timed) { vadx_status e = record(c, c->ev_fc, &stop); if (e) return e; }
    HIP_TRY(c, launch_fc_stats(f, ni, st));
    if (timed) HIP_TRY(c, hipEventRecord(stop, st));
    return VADX_OK;
}

static void drop_graph(vadx_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->g_ws = nullptr;
}

vadx_status vadx_integrate(vadx_ctx *c, const vadx_run *r, void *ws, size_t ws_bytes)
{
    if (!c) return VADX_E_ARG;
    if (!run_ok(c, r)) return fail(c, VADX_E_ARG, "invalid run settings");
    if (!c->planned || std::memcmp(&c->plan_run, r, sizeof(vadx_run)) != 0)
        return fail(c, VADX_E_STATE, "run differs from the last vadx_plan (call vadx_plan first)");
    if (!ws || ((uintptr_t)ws & 255u)) return fail(c, VADX_E_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < c->ws_bytes)
        return fail(c, VADX_E_OOM, "workspace of %zu bytes < planned %zu", ws_bytes, c->ws_bytes);
    HIP_TRY(c, hipSetDevice(c->device));
    if (!c->use_graph || c->timing) {
        vadx_status e = enqueue_run(c, r, ws, c->stream, c->timing);
        if (e) return e;
    } else {
        if (!c->gexec || c->g_ws != ws || c->g_epoch != c->plan_epoch) {
            drop_graph(c);
            if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            vadx_status e = enqueue_run(c, r, ws, c->cap_stream, false);
            hipGraph_t g = nullptr;
            hipError_t ce = hipStreamEndCapture(c->cap_stream, &g);
            if (e) { if (g) (void)hipGraphDestroy(g); return e; }
            if (ce != hipSuccess) return fail(c, VADX_E_HIP, "graph capture: %s", hipGetErrorString(ce));
            hipError_t ie = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (ie != hipSuccess) {
                c->gexec = nullptr;
                return fail(c, VADX_E_HIP, "graph instantiate: %s", hipGetErrorString(ie));
            }
            c->g_ws = ws;
            c->g_epoch = c->plan_epoch;
        }
        HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
    }
    c->ws = ws;
    c->ran = true;
    return VADX_OK;
}

vadx_status vadx_set_waves_per_simd(vadx_ctx *c, int32_t waves)
{
    if (!c) return VADX_E_ARG;
    if (waves != 0 && waves != 2 && waves != 3) return fail(c, VADX_E_ARG, "waves per SIMD must be 2 or 3");
    c->occ = waves == 0 ? 2 : waves;
    c->planned = false;
    return VADX_OK;
}

vadx_status vadx_wave_slack(vadx_ctx *c, int32_t slack, int32_t *current)
{
    if (!c) return VADX_E_ARG;
    if (slack < -1 || slack > 1) return fail(c, VADX_E_ARG, "wave slack must be 0, 1 or -1");
    if (slack >= 0 && slack != c->slack) {
        c->slack = slack;
        c->planned = false;
    }
    if (current) *current = c->slack;
    return VADX_OK;
}

vadx_status vadx_launch_info(vadx_ctx *c, int32_t *groups, int32_t *block_threads,
                             int32_t *grid, int32_t *steps_per_block)
{
    if (!c) return VADX_E_ARG;
    if (!c->planned) return fail(c, VADX_E_STATE, "no plan");
    int g = 0;
    if (c->launch_mode == 0) {
        const int per_cu = persistent_blocks_per_cu(c->block, c->wg_threads, c->occ);
        g = std::min((int)c->h_groups.size(), per_cu * c->cus);
    } else {
        for (const BlockClass &bc : c->classes) g = std::max(g, bc.n_groups);
    }
    if (groups) *groups = (int32_t)c->h_groups.size();
    if (block_threads) *block_threads = c->wg_threads;
    if (grid) *grid = g;
    if (steps_per_block) *steps_per_block = c->block;
    return VADX_OK;
}

vadx_status vadx_set_graph(vadx_ctx *c, int32_t on)
{
    if (!c) return VADX_E_ARG;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->use_graph = on != 0;
    return VADX_OK;
}

vadx_status vadx_sync(vadx_ctx *c)
{
    if (!c) return VADX_E_ARG;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->ran) {
        uint32_t status = 0;
        HIP_TRY(c, hipMemcpy(&status, (char *)c->ws + c->off_queue + 4, 4, hipMemcpyDeviceToHost));
        if (status & 1u) return fail(c, VADX_E_HIP, "integration scheduler: a wait for a previous chunk timed out");
        if (status & 2u) return fail(c, VADX_E_HIP, "integration: a wait for another wave's block timed out");
    }
    return VADX_OK;
}

vadx_status vadx_set_launch(vadx_ctx *c, int32_t mode, int32_t wg_instances, int32_t item_steps)
{
    if (!c) return VADX_E_ARG;
    if ((mode != 0 && mode != 1) || wg_instances < 0 || item_steps < 0)
        return fail(c, VADX_E_ARG, "bad launch shape");
    c->launch_mode = mode;
    c->wg_instances_override = wg_instances;
    c->item_steps = item_steps > 0 ? item_steps : 1000;
    c->planned = false;
    return VADX_OK;
}

static vadx_status copy_out(vadx_ctx *c, void *dst, const void *src, size_t bytes, int32_t where)
{
    if (where != VADX_HOST && where != VADX_DEVICE) return fail(c, VADX_E_ARG, "bad `where`");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(dst, src, bytes,
                              where == VADX_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                              c->stream));
    if (where == VADX_HOST) HIP_TRY(c, hipStreamSynchronize(c->stream));
    return VADX_OK;
}

static vadx_status check_read(vadx_ctx *c, int64_t inst, void *out)
{
    if (!c->ran) return fail(c, VADX_E_STATE, "no results: call vadx_integrate first");
    if (!out) return fail(c, VADX_E_ARG, "null output");
    if (inst < 0 || inst >= (int64_t)c->h_inst.size()) return fail(c, VADX_E_ARG, "instance out of range");
    return VADX_OK;
}

vadx_status vadx_read_stats(vadx_ctx *c, int64_t first, int64_t count, vadx_stats *out, int32_t where)
{
    if (!c) return VADX_E_ARG;
    if (count == 0) return VADX_OK;
    vadx_status st = check_read(c, first, out);
    if (st) return st;
    if (count < 0 || first + count > (int64_t)c->h_inst.size()) return fail(c, VADX_E_ARG, "range out of bounds");
    return copy_out(c, out, (char *)c->ws + c->off_stats + first * sizeof(vadx_stats),
                    count * sizeof(vadx_stats), where);
}

vadx_status vadx_read_fc(vadx_ctx *c, int64_t inst, float *out, int32_t where)
{
    if (!c) return VADX_E_ARG;
    vadx_status st = check_read(c, inst, out);
    if (st) return st;
    const InstDev &d = c->h_inst[inst];
    return copy_out(c, out, (float *)c->ws + d.fc_off, sizeof(float) * d.n * d.n, where);
}

vadx_status vadx_read_samples(vadx_ctx *c, int64_t inst, float *out, int32_t where)
{
    if (!c) return VADX_E_ARG;
    vadx_status st = check_read(c, inst, out);
    if (st) return st;
    const InstDev &d = c->h_inst[inst];
    if (c->n_samples == 0) return VADX_OK;
    return copy_out(c, out, (float *)c->ws + d.samp_off, sizeof(float) * d.n * c->n_samples, where);
}

vadx_status vadx_read_state(vadx_ctx *c, int64_t inst, double *out, int32_t where)
{
    if (!c) return VADX_E_ARG;
    vadx_status st = check_read(c, inst, out);
    if (st) return st;
    const InstDev &d = c->h_inst[inst];
    if (c->plan_run.n_steps == 0) return fail(c, VADX_E_STATE, "no steps were integrated");
    return copy_out(c, out, (float *)c->ws + d.state_off, sizeof(double) * 8 * d.n, where);
}

vadx_status vadx_read_trace(vadx_ctx *c, int64_t slot, float *out, int32_t where)
{
    if (!c) return VADX_E_ARG;
    if (slot < 0 || slot >= (int64_t)c->traced.size()) return fail(c, VADX_E_ARG, "trace slot out of range");
    vadx_status st = check_read(c, c->traced[slot], out);
    if (st) return st;
    const InstDev &d = c->h_inst[c->traced[slot]];
    if (d.trace_off < 0) return fail(c, VADX_E_STATE, "no trace recorded");
    return copy_out(c, out, (float *)c->ws + d.trace_off,
                    sizeof(float) * 8 * d.n * c->plan_run.n_trace_steps, where);
}

vadx_status vadx_instance_shape(vadx_ctx *c, int64_t inst, int32_t *n_regions, int64_t *n_samples)
{
    if (!c || !n_regions || !n_samples) return fail(c, VADX_E_ARG, "null argument");
    if (!c->planned) return fail(c, VADX_E_STATE, "no plan");
    if (inst < 0 || inst >= (int64_t)c->h_inst.size()) return fail(c, VADX_E_ARG, "instance out of range");
    *n_regions = c->h_inst[inst].n;
    *n_samples = c->n_samples;
    return VADX_OK;
}

vadx_status vadx_enable_timing(vadx_ctx *c, int32_t on)
{
    if (!c) return VADX_E_ARG;
    c->timing = on != 0;
    return VADX_OK;
}

static vadx_status drain(vadx_ctx *c, std::vector<std::pair<hipEvent_t, hipEvent_t>> &evs,
                         int64_t &n, double &ms)
{
    for (auto &e : evs) {
        float t = 0.f;
        HIP_TRY(c, hipEventSynchronize(e.second));
        HIP_TRY(c, hipEventElapsedTime(&t, e.first, e.second));
        ms += t;
        ++n;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    evs.clear();
    return VADX_OK;
}

vadx_status vadx_kernel_time(vadx_ctx *c, int64_t *n_int, double *ms_int, int64_t *n_fc, double *ms_fc)
{
    if (!c || !n_int || !ms_int || !n_fc || !ms_fc) return fail(c, VADX_E_ARG, "null argument");
    HIP_TRY(c, hipSetDevice(c->device));
    vadx_status st = drain(c, c->ev_int, c->n_int, c->ms_int);
    if (st) return st;
    st = drain(c, c->ev_fc, c->n_fc, c->ms_fc);
    if (st) return st;
    *n_int = c->n_int; *ms_int = c->ms_int; *n_fc = c->n_fc; *ms_fc = c->ms_fc;
    c->n_int = c->n_fc = 0;
    c->ms_int = c->ms_fc = 0.0;
    return VADX_OK;
}

} // extern "C"

// ---------------------------------------------------------------- autotuner
// Key of a batch for the tuning cache: device, block length and the mix of
// region counts (instance counts rounded to powers of two).
static std::string tune_key(vadx_ctx *c)
{
    hipDeviceProp_t prop{};
    std::string dev = "unknown";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) dev = prop.gcnArchName;
    std::map<int, int64_t> cls;
    for (int32_t ci : c->conn_of) cls[c->conns[ci].n] += 1;
    std::ostringstream k;
    for (char ch : dev)
        if (ch != '"' && ch != '\\' && ch != ':') k << ch;
    k << "|B" << c->block;
    for (auto &e : cls) {
        int64_t p2 = 1;
        while (p2 < e.second) p2 <<= 1;
        k << "|n" << e.first << "x" << p2;
    }
    return k.str();
}

// Lane budgets per region count as "n:lanes,n:lanes".
static std::string lanes_str(const std::map<int, int> &m)
{
    std::ostringstream o;
    for (auto it = m.begin(); it != m.end(); ++it) o << (it == m.begin() ? "" : ",") << it->first << ":" << it->second;
    return o.str();
}

static bool lanes_parse(const std::string &t, std::map<int, int> *m)
{
    std::map<int, int> r;
    std::istringstream in(t);
    std::string tok;
    while (std::getline(in, tok, ',')) {
        int n = 0, l = 0;
        if (std::sscanf(tok.c_str(), "%d:%d", &n, &l) != 2 || n < 1 || l < 64 || l > 512) return false;
        r[n] = l;
    }
    if (r.empty()) return false;
    *m = r;
    return true;
}

static bool tune_lookup(const char *path, const std::string &key, std::map<int, int> *lanes, int *items,
                        int *occ, int *slack)
{
    if (!path) return false;
    std::ifstream f(path);
    std::string line, q = "\"" + key + "\"";
    while (std::getline(f, line)) {
        const size_t at = line.find(q);
        if (at == std::string::npos) continue;
        int it = 0, w = 0;
        const size_t pl = line.find("\"class_lanes\": \"", at), pi = line.find("\"item_steps\":", at);
        const size_t pw = line.find("\"waves_per_simd\":", at);
        if (pl == std::string::npos || pi == std::string::npos || pw == std::string::npos) continue;
        const size_t l0 = pl + 16, l1 = line.find('"', l0);
        std::map<int, int> m;
        if (l1 != std::string::npos && lanes_parse(line.substr(l0, l1 - l0), &m) &&
            std::sscanf(line.c_str() + pi + 13, "%d", &it) == 1 &&
            std::sscanf(line.c_str() + pw + 17, "%d", &w) == 1 && it > 0 && w >= 2 && w <= 3) {
            // entries written before the slack setting existed were tuned without it
            int sl = 0;
            const size_t ps = line.find("\"wave_slack\":", at);
            if (ps != std::string::npos && (std::sscanf(line.c_str() + ps + 13, "%d", &sl) != 1 || sl < 0 || sl > 1))
                continue;
            *lanes = m;
            *items = it;
            *occ = w;
            *slack = sl;
            return true;
        }
    }
    return false;
}

static void tune_store(const char *path, const std::string &key, const std::map<int, int> &lanes,
                       int items, int occ, int slack, double ms)
{
    if (!path) return;
    std::vector<std::string> keep;
    {
        std::ifstream f(path);
        std::string line, q = "\"" + key + "\"";
        while (std::getline(f, line))
            if (line.find("\"class_lanes\":") != std::string::npos && line.find(q) == std::string::npos) {
                while (!line.empty() && (line.back() == ',' || line.back() == ' ')) line.pop_back();
                keep.push_back(line);
            }
    }
    char buf[640];
    std::snprintf(buf, sizeof(buf),
                  "  \"%s\": {\"class_lanes\": \"%s\", \"item_steps\": %d, \"waves_per_simd\": %d, "
                  "\"wave_slack\": %d, \"trial_ms\": %.3f}",
                  key.c_str(), lanes_str(lanes).c_str(), items, occ, slack, ms);
    keep.push_back(buf);
    std::ofstream o(path, std::ios::trunc);
    o << "{\n";
    for (size_t i = 0; i < keep.size(); ++i) o << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
    o << "}\n";
}

extern "C" vadx_status vadx_autotune(vadx_ctx *c, const vadx_run *r, void *ws, size_t ws_bytes,
                                     const char *cache_path, int32_t trial_steps,
                                     int32_t *lanes_out, int32_t *item_steps_out,
                                     int32_t *waves_out)
{
    if (!c || !r || !ws || ((uintptr_t)ws & 255u) || trial_steps < 0)
        return fail(c, VADX_E_ARG, "bad autotune arguments");
    if (c->S.empty()) return fail(c, VADX_E_STATE, "no batch set");
    if (!run_ok(c, r)) return fail(c, VADX_E_ARG, "invalid run settings");
    HIP_TRY(c, hipSetDevice(c->device));
    // trial runs: the same model and steps, no samples, no traces
    vadx_run t = *r;
    t.n_steps = trial_steps > 0 ? trial_steps : 2000;
    t.transient_steps = t.n_steps;
    t.n_trace_steps = 0;
    t.chunk_steps = 0;
    size_t need = 0;
    const int saved_mode = c->launch_mode, saved_override = c->wg_instances_override;
    const int saved_occ = c->occ, saved_slack = c->slack;
    const bool saved_graph = c->use_graph, saved_timing = c->timing;
    std::vector<int64_t> saved_traced = c->traced;
    c->traced.clear();
    c->launch_mode = 0;
    c->wg_instances_override = 0;
    c->use_graph = false;
    c->timing = false;
    // the region-count classes of the batch
    std::map<int, int> lanes;
    for (int32_t ci : c->conn_of) lanes[c->conns[ci].n] = 256;
    vadx_status result = VADX_OK;
    std::map<int, int> best_l = lanes;
    // lane budgets and slack are compared at items of an eighth of the trial
    // run (500..3000 steps), so that each group still runs several items
    const int i0 = (int)std::min<int64_t>(3000, std::max<int64_t>(500, t.n_steps / 8));
    int best_i = i0, best_w = 2, best_s = 0;
    double best_ms = -1.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto restore = [&]() {
        c->occ = saved_occ;
        c->slack = saved_slack;
        c->launch_mode = saved_mode;
        c->wg_instances_override = saved_override;
        c->use_graph = saved_graph;
        c->timing = saved_timing;
        c->traced = saved_traced;
        c->planned = false;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    // VADX_TUNE_LOG set: each trial's shape and time go to stderr
    const bool tune_log = std::getenv("VADX_TUNE_LOG") != nullptr;
    auto trial = [&](const std::map<int, int> &l, int items, int occ, int slack, double *ms) -> vadx_status {
        c->class_lanes = l;
        c->item_steps = items;
        c->occ = occ;
        c->slack = slack;
        c->planned = false;
        vadx_status st = vadx_plan(c, &t, &need);
        if (st) return st;
        // a shape whose plan needs more workspace than given (deeper rings
        // under wave slack) is left out
        if (need > ws_bytes) {
            *ms = std::numeric_limits<double>::infinity();
            return VADX_OK;
        }
        HIP_TRY(c, hipEventRecord(e0, c->stream));
        st = enqueue_run(c, &t, ws, c->stream, false);
        if (st) return st;
        HIP_TRY(c, hipEventRecord(e1, c->stream));
        st = vadx_sync(c);
        if (st) return st;
        float f = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&f, e0, e1));
        *ms = f;
        if (tune_log)
            std::fprintf(stderr, "[vadx autotune] lanes %s slack %d waves %d items %d: %.3f ms\n",
                         lanes_str(l).c_str(), slack, occ, items, f);
        return VADX_OK;
    };
    // the key needs the block length of this batch: plan once (without slack)
    c->class_lanes = lanes;
    c->slack = 0;
    c->planned = false;
    result = vadx_plan(c, &t, &need);
    if (result) { restore(); return result; }
    const std::string key = tune_key(c);
    std::map<int, int> cl;
    int ci = 0, cw = 0;
    int cs = 0;
    if (tune_lookup(cache_path, key, &cl, &ci, &cw, &cs)) {
        for (auto &e : lanes)
            if (cl.count(e.first)) e.second = cl[e.first];
        best_l = lanes;
        best_i = ci;
        best_w = cw;
        best_s = cs;
    } else {
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            restore();
            return fail(c, VADX_E_HIP, "event creation failed");
        }
        double ms = 0.0;
        result = trial(lanes, i0, 2, 0, &ms);    // warm-up (code load, caches)
        if (result == VADX_OK) result = trial(lanes, i0, 2, 0, &ms);
        if (result == VADX_OK) best_ms = ms;
        // with and without wave slack, each region-count class's lane budget
        // in turn (the others at their best so far for that slack):
        // floor(budget / n) instances per workgroup, one candidate per
        // distinct instance count
        for (int sl : {0, 1}) {
            std::map<int, int> sl_l = lanes;
            double sl_ms = -1.0;
            if (sl == 1 && result == VADX_OK) result = trial(sl_l, i0, 2, 1, &sl_ms);
            if (sl == 0) sl_ms = best_ms;
            for (auto &e : lanes) {
                const int n = e.first;
                for (int l = std::max(64, (n + 63) / 64 * 64); l <= 512 && result == VADX_OK; l += 64) {
                    if (l + 64 <= 512 && std::max(1, l / n) == std::max(1, (l + 64) / n)) continue;
                    if (l == sl_l[n]) continue;
                    std::map<int, int> cand = sl_l;
                    cand[n] = l;
                    result = trial(cand, i0, 2, sl, &ms);
                    if (result == VADX_OK && ms < sl_ms) { sl_ms = ms; sl_l = cand; }
                }
            }
            if (result == VADX_OK && sl_ms < best_ms) { best_ms = sl_ms; best_l = sl_l; best_s = sl; }
        }
        // the register budget at the chosen lane budgets and slack
        if (result == VADX_OK) {
            result = trial(best_l, i0, 3, best_s, &ms);
            if (result == VADX_OK && ms < best_ms) { best_ms = ms; best_w = 3; }
        }
        // the item length, over trial runs as long as the run itself (at most
        // max(trial_steps, 60000) steps): the queue's tail is a share of the
        // run that grows with the item length, so short trials would favour
        // short items
        t.n_steps = std::min<int64_t>(r->n_steps, std::max<int64_t>(t.n_steps, 60000));
        t.transient_steps = t.n_steps;
        best_ms = std::numeric_limits<double>::infinity();
        for (int it : {500, 1000, 2000, 3000, 4000, 8000}) {
            if (result) break;
            result = trial(best_l, it, best_w, best_s, &ms);
            if (result == VADX_OK && ms < best_ms) { best_ms = ms; best_i = it; }
        }
        if (result == VADX_OK) tune_store(cache_path, key, best_l, best_i, best_w, best_s, best_ms);
    }
    restore();
    if (result) return result;
    c->class_lanes = best_l;
    c->item_steps = best_i;
    c->occ = best_w;
    c->slack = best_s;
    int widest = 64;
    for (auto &e : best_l) widest = std::max(widest, e.second);
    if (waves_out) *waves_out = best_w;
    if (lanes_out) *lanes_out = widest;
    if (item_steps_out) *item_steps_out = best_i;
    return VADX_OK;
}

extern "C" vadx_status vadx_class_lanes(vadx_ctx *c, int32_t n_regions, int32_t lanes, int32_t *current)
{
    if (!c) return VADX_E_ARG;
    if (n_regions < 1 || (lanes != 0 && lanes != -1 && (lanes < 64 || lanes > 512)))
        return fail(c, VADX_E_ARG, "bad lane budget");
    if (lanes > 0) {
        c->class_lanes[n_regions] = lanes;
        c->planned = false;
    } else if (lanes == 0) {
        c->class_lanes.erase(n_regions);
        c->planned = false;
    }
    if (current) {
        const auto it = c->class_lanes.find(n_regions);
        *current = it != c->class_lanes.end() ? it->second : c->wg_lanes;
    }
    return VADX_OK;
}

// ---------------------------------------------------------------- analysis
extern "C" vadx_status vadx_analyze_series(vadx_ctx *c, const float *samples, int64_t n_inst,
                                           int32_t n, int64_t n_samples, double sample_period_ms,
                                           const vadx_analysis_cfg *cfg, void *ws, size_t ws_bytes,
                                           vadx_analysis *out, float *psd_out, float *pli_out)
{
    if (!c) return VADX_E_ARG;
    if (n_inst < 0) return fail(c, VADX_E_ARG, "negative instance count");
    if (n < 1 || n > 512) return fail(c, VADX_E_ARG, "region count must be in [1, 512]");
    std::vector<int64_t> off((size_t)n_inst);
    std::vector<int32_t> ns((size_t)n_inst, n);
    for (int64_t i = 0; i < n_inst; ++i) off[(size_t)i] = i * n_samples * n;
    AnInstances in{samples, off.data(), ns.data(), n_inst, n_samples};
    std::string err;
    vadx_status st = run_analysis(c->device, c->stream, in, sample_period_ms, cfg, ws, ws_bytes, out,
                                  psd_out, pli_out, c->timing ? &c->an_timer : nullptr, err);
    if (st) return fail(c, st, "%s", err.c_str());
    return VADX_OK;
}

extern "C" vadx_status vadx_analyze(vadx_ctx *c, const vadx_analysis_cfg *cfg, void *ws,
                                    size_t ws_bytes, vadx_analysis *out)
{
    if (!c) return VADX_E_ARG;
    if (!c->ran) return fail(c, VADX_E_STATE, "no samples: call vadx_integrate first");
    const size_t ni = c->h_inst.size();
    std::vector<int64_t> off(ni);
    std::vector<int32_t> ns(ni);
    for (size_t i = 0; i < ni; ++i) {
        off[i] = c->h_inst[i].samp_off;
        ns[i] = c->h_inst[i].n;
    }
    AnInstances in{(const float *)c->ws, off.data(), ns.data(), (int64_t)ni, c->n_samples};
    const double period = (double)c->plan_run.tavg_steps * c->plan_run.dt_ms;
    std::string err;
    vadx_status st = run_analysis(c->device, c->stream, in, period, cfg, ws, ws_bytes, out, nullptr,
                                  nullptr, c->timing ? &c->an_timer : nullptr, err);
    if (st) return fail(c, st, "%s", err.c_str());
    return VADX_OK;
}

extern "C" vadx_status vadx_analysis_kernel_time(vadx_ctx *c, int64_t *launches, double *ms)
{
    if (!c || !launches || !ms) return fail(c, VADX_E_ARG, "null argument");
    HIP_TRY(c, hipSetDevice(c->device));
    for (int k = 0; k < kAnKernels; ++k) {
        vadx_status st = drain(c, c->an_timer.ev[k], c->an_timer.n[k], c->an_timer.ms[k]);
        if (st) return st;
        launches[k] = c->an_timer.n[k];
        ms[k] = c->an_timer.ms[k];
        c->an_timer.n[k] = 0;
        c->an_timer.ms[k] = 0.0;
    }
    return VADX_OK;
}

// ------------------------------------------------------- fitness and ranking
extern "C" vadx_status vadx_set_reference_fc(vadx_ctx *c, int32_t conn_id, const float *fc)
{
    if (!c) return VADX_E_ARG;
    if (conn_id < 0 || conn_id >= (int32_t)c->conns.size()) return fail(c, VADX_E_ARG, "no such connectome");
    HostConn &h = c->conns[(size_t)conn_id];
    const int64_t nn = (int64_t)h.n * h.n;
    if (!fc) {
        h.ref_off = -1;
        ++c->plan_epoch;
        return upload_conns(c);
    }
    for (int64_t i = 0; i < nn; ++i)
        if (!std::isfinite(fc[i])) return fail(c, VADX_E_ARG, "non-finite reference FC entry");
    HIP_TRY(c, hipSetDevice(c->device));
    if (h.ref_slot < 0) {
        // grow the reference store, keeping the matrices already there
        const int64_t need = c->total_ref + nn;
        if ((size_t)need > c->refs.n) {
            float *np = nullptr;
            HIP_TRY(c, hipMalloc((void **)&np, sizeof(float) * (size_t)need));
            if (c->refs.p && c->total_ref > 0) {
                HIP_TRY(c, hipMemcpyAsync(np, c->refs.p, sizeof(float) * (size_t)c->total_ref,
                                          hipMemcpyDeviceToDevice, c->stream));
                HIP_TRY(c, hipStreamSynchronize(c->stream));
            }
            if (c->refs.p) (void)hipFree(c->refs.p);
            c->refs.p = np;
            c->refs.n = (size_t)need;
        }
        h.ref_slot = c->total_ref;
        c->total_ref += nn;
    }
    HIP_TRY(c, hipMemcpyAsync(c->refs.p + h.ref_slot, fc, sizeof(float) * (size_t)nn,
                              hipMemcpyHostToDevice, c->stream));
    h.ref_off = h.ref_slot;
    ++c->plan_epoch;                  // a recorded graph holds the old reference pointer
    return upload_conns(c);
}

extern "C" vadx_status vadx_top_k(vadx_ctx *c, const float *score, int64_t n, int32_t k,
                                  int64_t *idx, float *val)
{
    if (!c) return VADX_E_ARG;
    if (n < 0 || k < 0 || (n > 0 && !score) || (k > 0 && !idx))
        return fail(c, VADX_E_ARG, "bad top-k arguments");
    if (k > 1024) return fail(c, VADX_E_UNSUPPORTED, "k above 1024");
    if (k > n) return fail(c, VADX_E_ARG, "k above the number of scores");
    if (k == 0) return VADX_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, c->topk_idx.ensure((size_t)k));
    int64_t n_sel = 0;
    std::string err;
    vadx_status st = select_run(c->stream, c->sel, score, n, k, 0.f, 0u, c->topk_idx.p, nullptr, k,
                                &n_sel, err);
    if (st) return fail(c, st, "%s", err.c_str());
    if (n_sel != k) return fail(c, VADX_E_ARG, "selection returned %lld of %d", (long long)n_sel, k);
    HIP_TRY(c, launch_rank_sort(score, c->topk_idx.p, k, idx, val, c->stream));
    return VADX_OK;
}

// ---------------------------------------------------------------- top k without allocation
// vadx_top_k_noalloc keeps its scratch (the selection's histogram, per-tile
// counts and bases, the k candidate indices) in one file-scope device array
// of fixed size instead of allocating. Each device holds its own copy; host
// code reaches it only through the address hipGetSymbolAddress gives on that
// device (kept per device in g_noalloc_ptr), never through the array's name.
constexpr int64_t kNoAllocMaxPoints = (int64_t)1 << 24;
constexpr int64_t kNoAllocTiles = kNoAllocMaxPoints / 4096;     // selection tiles of 4096 points
constexpr size_t kNoAllocSelBytes = 256 * 4 + kNoAllocTiles * 4 + 2 * kNoAllocTiles * 8;
constexpr size_t kNoAllocBytes = ((kNoAllocSelBytes + 255) / 256) * 256 + 1024 * sizeof(int64_t);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[kNoAllocMaxDevices];

// Address of this device's scratch copy; resolved once per device with the
// device current (vadx_create calls it). Returns hipSuccess or the error.
static hipError_t noalloc_scratch(int device, void **p)
{
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void *q = nullptr;
        hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_noalloc_ptr[device] = q;
    }
    *p = g_noalloc_ptr[device];
    return hipSuccess;
}

extern "C" vadx_status vadx_top_k_noalloc(vadx_ctx *c, const float *score, int64_t n, int32_t k,
                                          int64_t *idx, float *val)
{
    if (!c) return VADX_E_ARG;
    if (n < 0 || k < 0 || (n > 0 && !score) || (k > 0 && !idx))
        return fail(c, VADX_E_ARG, "bad top-k arguments");
    if (k > 1024) return fail(c, VADX_E_UNSUPPORTED, "k above 1024");
    if (k > n) return fail(c, VADX_E_ARG, "k above the number of scores");
    if (n > kNoAllocMaxPoints)
        return fail(c, VADX_E_UNSUPPORTED, "%lld scores: vadx_top_k_noalloc takes at most %lld",
                    (long long)n, (long long)kNoAllocMaxPoints);
    if (k == 0) return VADX_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    if (select_tiles(n) > kNoAllocTiles) return fail(c, VADX_E_UNSUPPORTED, "selection tiles exceed the scratch");
    void *base = nullptr;
    HIP_TRY(c, noalloc_scratch(c->device, &base));
    // host staging of the per-tile counts: static, one set per calling thread
    static thread_local uint32_t h_counts[kNoAllocTiles];
    static thread_local int64_t h_bases[kNoAllocTiles];
    SelScratch sc;
    sc.p = base;
    sc.tiles = kNoAllocTiles;
    int64_t *cand = (int64_t *)((char *)base + ((kNoAllocSelBytes + 255) / 256) * 256);
    int64_t n_sel = 0;
    std::string err;
    vadx_status st = select_run(c->stream, sc, score, n, k, 0.f, 0u, cand, nullptr, k, &n_sel, err,
                                h_counts, h_bases);
    if (st) return fail(c, st, "%s", err.c_str());
    if (n_sel != k) return fail(c, VADX_E_ARG, "selection returned %lld of %d", (long long)n_sel, k);
    HIP_TRY(c, launch_rank_sort(score, cand, k, idx, val, c->stream));
    return VADX_OK;
}

extern "C" vadx_status vadx_set_instance_param(vadx_ctx *c, int32_t param, int64_t n,
                                               const double *values)
{
    if (!c) return VADX_E_ARG;
    if (param < 0 || param >= 6) return fail(c, VADX_E_ARG, "unknown parameter %d", param);
    if (n != (int64_t)c->S.size()) return fail(c, VADX_E_ARG, "n must equal the batch size");
    if (!values) {
        c->iparam[param].clear();
    } else {
        for (int64_t i = 0; i < n; ++i) {
            const double v = values[i];
            const bool ok = param == VADX_P_TAU_W_E ? (std::isfinite(v) && v > 0.0)
                                                    : (std::isfinite(v) && v >= 0.0);
            if (!ok) return fail(c, VADX_E_ARG, "parameter %d of instance %lld out of range", param,
                                 (long long)i);
        }
        c->iparam[param].assign(values, values + n);
    }
    c->planned = false;
    c->ran = false;
    return VADX_OK;
}

// ------------------------------------------------------------------- BOLD
extern "C" vadx_status vadx_bold_defaults(vadx_bold_cfg *p)
{
    if (!p) return VADX_E_ARG;
    p->kappa = 0.65;
    p->gamma = 0.41;
    p->tau0 = 0.98;
    p->alpha = 0.32;
    p->E0 = 0.34;
    p->V0 = 0.02;
    p->k1 = 7.0 * 0.34;
    p->k2 = 2.0;
    p->k3 = 2.0 * 0.34 - 0.2;
    p->tr_ms = 2000.0;
    return VADX_OK;
}

static int32_t bold_count(int64_t n_samples, double period_ms, double tr_ms)
{
    return (int32_t)std::floor((double)n_samples * period_ms / tr_ms + 1e-9);
}

static vadx_status run_bold(vadx_ctx *c, const float *samples, const std::vector<int64_t> &off,
                            const std::vector<int32_t> &ns, int64_t n_samples, double period_ms,
                            const vadx_bold_cfg *p, float *out, int32_t *n_tr_out)
{
    if (!p || !n_tr_out) return fail(c, VADX_E_ARG, "null argument");
    auto pos = [](double x) { return std::isfinite(x) && x > 0.0; };
    if (!(std::isfinite(p->kappa) && p->kappa >= 0.0 && pos(p->gamma) && pos(p->tau0) &&
          pos(p->alpha) && pos(p->E0) && p->E0 < 1.0 && std::isfinite(p->V0) &&
          std::isfinite(p->k1) && std::isfinite(p->k2) && std::isfinite(p->k3) && pos(p->tr_ms)))
        return fail(c, VADX_E_ARG, "invalid BOLD parameters");
    if (!pos(period_ms) || n_samples < 0) return fail(c, VADX_E_ARG, "invalid sample period or count");
    const int32_t n_tr = bold_count(n_samples, period_ms, p->tr_ms);
    *n_tr_out = n_tr;
    const size_t ni = ns.size();
    if (ni == 0 || n_tr == 0) return VADX_OK;
    if (!samples || !out) return fail(c, VADX_E_ARG, "null samples or output");
    std::vector<int32_t> rb(ni), emit((size_t)n_tr), reg;
    std::vector<int64_t> oo(ni);
    int64_t r = 0, o = 0;
    for (size_t i = 0; i < ni; ++i) {
        rb[i] = (int32_t)r;
        oo[i] = o;
        for (int k = 0; k < ns[i]; ++k) reg.push_back((int32_t)i);
        r += ns[i];
        o += (int64_t)n_tr * ns[i];
    }
    const double steps = p->tr_ms / period_ms;
    for (int32_t m = 0; m < n_tr; ++m) emit[(size_t)m] = (int32_t)std::nearbyint((m + 1) * steps);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, c->b_samp.ensure(ni));
    HIP_TRY(c, c->b_out.ensure(ni));
    HIP_TRY(c, c->b_n.ensure(ni));
    HIP_TRY(c, c->b_rbase.ensure(ni));
    HIP_TRY(c, c->b_reg.ensure((size_t)r));
    HIP_TRY(c, c->b_emit.ensure((size_t)n_tr));
    HIP_TRY(c, hipMemcpyAsync(c->b_samp.p, off.data(), 8 * ni, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->b_out.p, oo.data(), 8 * ni, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->b_n.p, ns.data(), 4 * ni, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->b_rbase.p, rb.data(), 4 * ni, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->b_reg.p, reg.data(), 4 * (size_t)r, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->b_emit.p, emit.data(), 4 * (size_t)n_tr, hipMemcpyHostToDevice,
                              c->stream));
    BoldArgs a{};
    a.samples = samples;
    a.samp_off = c->b_samp.p;
    a.n = c->b_n.p;
    a.rbase = c->b_rbase.p;
    a.reg_inst = c->b_reg.p;
    a.out_off = c->b_out.p;
    a.emit = c->b_emit.p;
    a.n_reg = r;
    a.n_samples = n_samples;
    a.n_tr = n_tr;
    a.kappa = (float)p->kappa;
    a.gamma = (float)p->gamma;
    a.inv_tau0 = (float)(1.0 / p->tau0);
    a.inv_alpha = (float)(1.0 / p->alpha);
    a.inv_E0 = (float)(1.0 / p->E0);
    a.l2_1mE0 = (float)std::log2(1.0 - p->E0);
    a.h = period_ms / 1000.0;
    a.V0 = p->V0;
    a.k1 = p->k1;
    a.k2 = p->k2;
    a.k3 = p->k3;
    a.out = out;
    HIP_TRY(c, launch_bold(a, c->stream));
    return VADX_OK;
}

extern "C" vadx_status vadx_bold_series(vadx_ctx *c, const float *samples, int64_t n_inst,
                                        int32_t n, int64_t n_samples, double sample_period_ms,
                                        const vadx_bold_cfg *cfg, float *out, int32_t *n_tr)
{
    if (!c) return VADX_E_ARG;
    if (n_inst < 0 || n < 1 || n > 512) return fail(c, VADX_E_ARG, "bad sizes");
    std::vector<int64_t> off((size_t)n_inst);
    std::vector<int32_t> ns((size_t)n_inst, n);
    for (int64_t i = 0; i < n_inst; ++i) off[(size_t)i] = i * n_samples * n;
    return run_bold(c, samples, off, ns, n_samples, sample_period_ms, cfg, out, n_tr);
}

extern "C" vadx_status vadx_bold(vadx_ctx *c, const vadx_bold_cfg *cfg, float *out, int32_t *n_tr)
{
    if (!c) return VADX_E_ARG;
    if (!c->ran) return fail(c, VADX_E_STATE, "no samples: call vadx_integrate first");
    const size_t ni = c->h_inst.size();
    std::vector<int64_t> off(ni);
    std::vector<int32_t> ns(ni);
    for (size_t i = 0; i < ni; ++i) {
        off[i] = c->h_inst[i].samp_off;
        ns[i] = c->h_inst[i].n;
    }
    const double period = (double)c->plan_run.tavg_steps * c->plan_run.dt_ms;
    return run_bold(c, (const float *)c->ws, off, ns, c->n_samples, period, cfg, out, n_tr);
}
