// hmc_api.hip -- the C ABI of libhmc.so (include/hmc.h): argument checks,
// workspace layout, form selection and stream-ordered launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "hmc_internal.hpp"

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace hmc {
hmc_status fail(hmc_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}
}  // namespace hmc
using hmc::fail;

namespace {

hmc_status check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return HMC_OK;
    return fail(HMC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
}  // namespace

struct hmc_ctx {
    hmc::PlainArgs a;
    hmc_config cfg;
    hipStream_t stream;
    uint64_t t;
    int32_t form;            // effective form
    hipGraphExec_t graph_exec;
    bool graph_ready;
    hmc::KernelTimer timer;  // armed by hmc_kernel_timer_start (a.timer points here)
};

namespace hmc {

size_t elem_size(int32_t dtype) { return dtype == HMC_F64 ? 8 : (dtype == HMC_BF16 ? 2 : 4); }

hmc_status check_adapt(const hmc_adapt* ad) {
    if (!ad || !ad->enabled) return HMC_OK;
    if (!(ad->target_accept > 0.0 && ad->target_accept < 1.0))
        return fail(HMC_E_INVALID, "adaptation target_accept must be in (0, 1)");
    if (ad->kind == HMC_ADAPT_DUAL_AVERAGING) {
        if (!(ad->gamma > 0.0) || !(ad->t0 >= 0.0) || !(ad->kappa > 0.0))
            return fail(HMC_E_INVALID, "dual-averaging parameters out of range");
        return HMC_OK;
    }
    if (ad->kind == HMC_ADAPT_SIMPLE) {
        if (!(ad->rate > 0.0 && ad->rate <= 1.0)) return fail(HMC_E_INVALID, "adaptation rate must be in (0, 1]");
        return HMC_OK;
    }
    return fail(HMC_E_INVALID, "unknown adaptation kind");
}

Workspace carve_workspace(void* base, const TargetDev& tg, const hmc_config& cfg, size_t* total) {
    const int64_t C = cfg.num_chains, D = tg.D;
    const size_t es = elem_size(cfg.state_dtype);
    const size_t state = (size_t)C * D * es;
    const bool bf16 = cfg.grad_dtype == HMC_BF16;
    int64_t nsplit = tg.kind == HMC_TGT_LOGREG ? logreg_nsplit_cap(tg.N, C) : 0;
    int64_t nsplit_lp = nsplit;
    if (bf16) {
        nsplit = nsplit > 8 ? nsplit : 8;          // BF16 split counts 1, 2, 4, 8
        nsplit_lp = nsplit > lb_logp_nsplit(tg.N, C, D) ? nsplit : lb_logp_nsplit(tg.N, C, D);
    }
    char* p = (char*)base;
    size_t off = 0;
    auto take = [&](size_t n) {
        void* r = p ? (void*)(p + off) : nullptr;
        off += align256(n);
        return r;
    };
    Workspace w;
    w.x = take(state);
    w.g = take(state);
    w.logp = (double*)take((size_t)C * 8);
    w.eps = (double*)take((size_t)C * 8);
    w.da = (DualAvg*)take((size_t)C * sizeof(DualAvg));
    w.xq = take(state);
    w.pq = take(state);
    w.gq = take(state);
    w.lpq = (double*)take((size_t)C * 8);
    w.h0 = (double*)take((size_t)C * 8);
    w.part_g = (float*)take((size_t)nsplit * C * D * 4);
    w.part_lp = (double*)take((size_t)nsplit_lp * C * 8);
    w.lr_cnt = (int32_t*)take(tg.kind == HMC_TGT_LOGREG ? (size_t)((C + 63) / 64) * 4 : 0);
    int64_t np = 0;
    const size_t padb = bf16 ? lb_pad_bytes(tg.N, D, &np, nullptr) : 0;
    w.xt = bf16 ? take(padb) : nullptr;
    w.xp = bf16 ? take(padb) : nullptr;
    w.yp = bf16 ? take((size_t)np) : nullptr;
    w.bk_x = take(state);
    w.bk_g = take(state);
    w.bk_logp = (double*)take((size_t)C * 8);
    w.bk_eps = (double*)take((size_t)C * 8);
    w.bk_da = (DualAvg*)take((size_t)C * sizeof(DualAvg));
    w.ctrl = (Ctrl*)take(sizeof(Ctrl));
    w.beta_buf = (double*)take((size_t)C * 8);
    w.beta = nullptr;
    w.scale_buf = (double*)take((size_t)D * 8);
    w.scale = nullptr;
    w.bytes = off;
    if (total) *total = off;
    return w;
}

}  // namespace hmc

using namespace hmc;

hmc_status hmc::validate_args(const hmc_target* tg, const hmc_config* cfg, TargetDev* out) {
    if (!tg || !cfg) return fail(HMC_E_INVALID, "target and config must not be NULL");
    if (tg->dim < 1) return fail(HMC_E_INVALID, "target dim must be >= 1");
    if (cfg->num_chains < 1) return fail(HMC_E_INVALID, "num_chains must be >= 1");
    if (cfg->num_chains > (int64_t)0x7fffffff) return fail(HMC_E_INVALID, "num_chains must be < 2^31");
    if (cfg->num_leapfrog_steps < 1) return fail(HMC_E_INVALID, "num_leapfrog_steps must be >= 1");
    if (cfg->state_dtype != HMC_F32 && cfg->state_dtype != HMC_F64)
        return fail(HMC_E_UNSUPPORTED, "state_dtype must be HMC_F32 or HMC_F64");
    if (cfg->grad_dtype != HMC_F32 && cfg->grad_dtype != HMC_BF16)
        return fail(HMC_E_UNSUPPORTED, "grad_dtype must be HMC_F32 or HMC_BF16");
    if (cfg->form < HMC_FORM_AUTO || cfg->form > HMC_FORM_GRAPH) return fail(HMC_E_INVALID, "unknown form");
    TargetDev t{};
    t.kind = tg->kind;
    t.D = tg->dim;
    t.prec = tg->prec;
    t.X = tg->X;
    t.N = tg->n_rows;
    t.y = tg->y;
    t.inv_var = 1.0;
    switch (tg->kind) {
    case HMC_TGT_STD_NORMAL:
        break;
    case HMC_TGT_GAUSS_DIAG:
    case HMC_TGT_GAUSS_DENSE:
        if (!tg->prec) return fail(HMC_E_INVALID, "Gaussian target needs prec");
        if (tg->kind == HMC_TGT_GAUSS_DENSE && cfg->state_dtype != HMC_F32)
            return fail(HMC_E_UNSUPPORTED, "dense Gaussian runs in FP32 state");
        if (tg->kind == HMC_TGT_GAUSS_DENSE && tg->dim > 1024)
            return fail(HMC_E_UNSUPPORTED, "dense Gaussian supports D <= 1024");
        break;
    case HMC_TGT_LOGREG:
        if (!tg->X || !tg->y) return fail(HMC_E_INVALID, "logistic regression needs X and y");
        if (tg->n_rows < 1) return fail(HMC_E_INVALID, "n_rows must be >= 1");
        if (!(tg->prior_scale > 0.0) || !std::isfinite(tg->prior_scale))
            return fail(HMC_E_INVALID, "prior_scale must be finite and > 0");
        if (tg->x_dtype != HMC_F32 && tg->x_dtype != HMC_BF16)
            return fail(HMC_E_UNSUPPORTED, "X must be HMC_F32 or HMC_BF16");
        if (cfg->state_dtype != HMC_F32) return fail(HMC_E_UNSUPPORTED, "logistic regression runs in FP32 state");
        if (tg->dim > 512) return fail(HMC_E_UNSUPPORTED, "logistic regression supports D <= 512");
        t.x_bf16 = tg->x_dtype == HMC_BF16;
        t.inv_var = 1.0 / (tg->prior_scale * tg->prior_scale);
        break;
    default:
        return fail(HMC_E_INVALID, "unknown target kind");
    }
    if (cfg->grad_dtype == HMC_BF16 && !(tg->kind == HMC_TGT_LOGREG && tg->x_dtype == HMC_BF16))
        return fail(HMC_E_UNSUPPORTED, "BF16 gradients need a logistic-regression target with BF16 X");
    if (cfg->grad_dtype == HMC_BF16 && !bf16_grad_supported(t))
        return fail(HMC_E_UNSUPPORTED, "BF16 gradients support D <= 512");
    if (cfg->grad_dtype == HMC_BF16 && cfg->form == HMC_FORM_FUSED)
        return fail(HMC_E_UNSUPPORTED, "BF16 gradients run in the plain or graph form");
    if (out) *out = t;
    return HMC_OK;
}

extern "C" {

const char* hmc_last_error(void) { return g_last_error.c_str(); }

hmc_status hmc_workspace_size(const hmc_target* target, const hmc_config* config, size_t* bytes) {
    TargetDev t;
    hmc_status st = validate_args(target, config, &t);
    if (st != HMC_OK) return st;
    if (!bytes) return fail(HMC_E_INVALID, "bytes must not be NULL");
    carve_workspace(nullptr, t, *config, bytes);
    return HMC_OK;
}

static hmc_status upload_eps(hmc_ctx* ctx, const double* step_size, int64_t len) {
    const int64_t C = ctx->a.C;
    std::vector<double> eps((size_t)C);
    for (int64_t c = 0; c < C; ++c) eps[(size_t)c] = step_size[len == 1 ? 0 : c];
    hmc_status st = check_hip(hipMemcpyAsync(ctx->a.ws.eps, eps.data(), (size_t)C * 8, hipMemcpyHostToDevice,
                                             ctx->stream), "upload step sizes");
    if (st != HMC_OK) return st;
    return check_hip(hipStreamSynchronize(ctx->stream), "upload step sizes");
}

static Ctrl base_ctrl(const hmc_ctx* ctx) {
    Ctrl c;
    memset(&c, 0, sizeof(c));
    c.t = ctx->t;
    c.t_begin = ctx->t;
    return c;
}

}  // extern "C"

// Argument checks of hmc_init that need no device: the target, the config,
// the initial state pointer and the step sizes.
static hmc_status check_init_args(const hmc_target* target, const hmc_config* config, const void* init_state,
                                  const double* step_size, int64_t step_size_len, TargetDev* t) {
    hmc_status st = validate_args(target, config, t);
    if (st != HMC_OK) return st;
    if (!init_state) return fail(HMC_E_INVALID, "init_state must not be NULL");
    if (!step_size) return fail(HMC_E_INVALID, "step_size must not be NULL");
    if (step_size_len != 1 && step_size_len != config->num_chains)
        return fail(HMC_E_INVALID, "step_size_len must be 1 or num_chains");
    for (int64_t i = 0; i < step_size_len; ++i)
        if (!(step_size[i] > 0.0) || !std::isfinite(step_size[i]))
            return fail(HMC_E_INVALID, "step sizes must be finite and > 0");
    return HMC_OK;
}

// hmc_init's device work on a context the caller owns: carve the workspace,
// pick the form, upload step sizes, bootstrap.  Arguments already checked.
static hmc_status init_ctx(hmc_ctx* ctx, const TargetDev& t, const hmc_config* config, const void* init_state,
                           const double* step_size, int64_t step_size_len, void* workspace, void* hip_stream) {
    hmc_status st = HMC_OK;
    ctx->cfg = *config;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->t = 0;
    ctx->graph_ready = false;
    ctx->graph_exec = nullptr;
    PlainArgs& a = ctx->a;
    a.tg = t;
    a.C = config->num_chains;
    a.L = config->num_leapfrog_steps;
    a.f64 = config->state_dtype == HMC_F64;
    a.bf16_grad = config->grad_dtype == HMC_BF16;
    a.key = make_key(config->seed);
    a.ws = carve_workspace(workspace, t, *config, nullptr);

    const bool can_fuse = fused_supported(a);
    switch (config->form) {
    case HMC_FORM_AUTO: ctx->form = can_fuse ? HMC_FORM_FUSED : HMC_FORM_PLAIN; break;
    case HMC_FORM_FUSED:
        if (!can_fuse) return fail(HMC_E_UNSUPPORTED, "no fused kernel for this target shape");
        ctx->form = HMC_FORM_FUSED;
        break;
    default: ctx->form = config->form;
    }

    st = upload_eps(ctx, step_size, step_size_len);
    if (st == HMC_OK && a.bf16_grad) st = check_hip(launch_pad_bf16(a, ctx->stream), "padded copies of X");
    if (st == HMC_OK) st = check_hip(launch_set_ctrl(base_ctrl(ctx), a.ws.ctrl, ctx->stream), "init control");
    if (st == HMC_OK) st = check_hip(launch_da_init(a, ctx->stream), "init adaptation");
    if (st == HMC_OK) st = check_hip(launch_bootstrap(a, init_state, ctx->stream), "bootstrap");
    if (st == HMC_OK) st = check_hip(hipStreamSynchronize(ctx->stream), "bootstrap");
    return st;
}

extern "C" {

hmc_status hmc_init(const hmc_target* target, const hmc_config* config, const void* init_state,
                    const double* step_size, int64_t step_size_len, void* workspace, size_t workspace_bytes,
                    void* hip_stream, hmc_ctx** out) {
    TargetDev t;
    hmc_status st = check_init_args(target, config, init_state, step_size, step_size_len, &t);
    if (st != HMC_OK) return st;
    if (!out) return fail(HMC_E_INVALID, "out must not be NULL");
    size_t need = 0;
    carve_workspace(nullptr, t, *config, &need);
    if (!workspace) return fail(HMC_E_INVALID, "workspace must not be NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(HMC_E_INVALID, "workspace must be 256-byte aligned");
    if (workspace_bytes < need) return fail(HMC_E_NOMEM, "workspace smaller than hmc_workspace_size()");
    hmc_ctx* ctx = new hmc_ctx();
    st = init_ctx(ctx, t, config, init_state, step_size, step_size_len, workspace, hip_stream);
    if (st != HMC_OK) {
        delete ctx;
        return st;
    }
    *out = ctx;
    return HMC_OK;
}

int32_t hmc_effective_form(const hmc_ctx* ctx) { return ctx ? ctx->form : -1; }

static hmc_status ensure_graph(hmc_ctx* ctx) {
    if (ctx->graph_ready) return HMC_OK;
    hipStream_t cs;
    hmc_status st = check_hip(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "graph stream");
    if (st != HMC_OK) return st;
    hipGraph_t graph = nullptr;
    st = check_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    if (st == HMC_OK) {
        PlainArgs ga = ctx->a;
        ga.timer = nullptr;      // no event nodes in the graph
        hipError_t le = launch_plain_transition(ga, false, cs);
        hipError_t ee = hipStreamEndCapture(cs, &graph);
        st = check_hip(le != hipSuccess ? le : ee, "capture transition");
    }
    if (st == HMC_OK) st = check_hip(hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0), "instantiate");
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    if (st == HMC_OK) ctx->graph_ready = true;
    return st;
}

static hmc_status run_transitions(hmc_ctx* ctx, int64_t n, bool copy_proposal) {
    if (ctx->form == HMC_FORM_GRAPH && !copy_proposal) {
        hmc_status st = ensure_graph(ctx);
        if (st != HMC_OK) return st;
        for (int64_t i = 0; i < n; ++i) {
            st = check_hip(hipGraphLaunch(ctx->graph_exec, ctx->stream), "graph launch");
            if (st != HMC_OK) return st;
        }
        return HMC_OK;
    }
    for (int64_t i = 0; i < n; ++i) {
        hmc_status st = check_hip(launch_plain_transition(ctx->a, copy_proposal, ctx->stream), "transition");
        if (st != HMC_OK) return st;
    }
    return HMC_OK;
}

hmc_status hmc_step(hmc_ctx* ctx, const hmc_step_out* out) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    hmc_step_out o;
    memset(&o, 0, sizeof(o));
    if (out) o = *out;
    hmc_status st;
    if (ctx->form == HMC_FORM_FUSED) {
        FusedRun r;
        memset(&r, 0, sizeof(r));
        r.t_begin = ctx->t;
        r.n_transitions = 1;
        r.out = o;
        timer_begin(ctx->a, ctx->stream);
        st = check_hip(launch_fused(ctx->a, r, ctx->stream), "fused step");
        timer_end(ctx->a, ctx->stream, "fused transition kernel");
    } else {
        Ctrl c = base_ctrl(ctx);
        c.out_acc = o.is_accepted;
        c.out_lar = o.log_accept_ratio;
        c.out_logp = o.target_log_prob;
        c.out_xprop = o.proposed_state;
        c.out_pprop = o.proposed_momentum;
        c.out_dh = o.delta_h;
        st = check_hip(launch_set_ctrl(c, ctx->a.ws.ctrl, ctx->stream), "step control");
        if (st == HMC_OK) st = run_transitions(ctx, 1, o.proposed_state || o.proposed_momentum);
    }
    if (st == HMC_OK) ctx->t += 1;
    return st;
}

hmc_status hmc_sample_chain(hmc_ctx* ctx, int64_t num_results, int64_t num_burnin_steps, const hmc_adapt* adapt,
                            void* samples, const hmc_trace* trace) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    if (num_results < 0 || num_burnin_steps < 0) return fail(HMC_E_INVALID, "negative transition count");
    const bool ad = adapt && adapt->enabled;
    if (ad && check_adapt(adapt) != HMC_OK) return HMC_E_INVALID;
    const int64_t total = num_results + num_burnin_steps;
    if (ctx->t + (uint64_t)total > 0xffffffffull) return fail(HMC_E_INVALID, "transition counter would exceed 2^32");
    hmc_trace tr;
    memset(&tr, 0, sizeof(tr));
    if (trace) tr = *trace;
    hmc_status st = HMC_OK;
    if (ad) st = check_hip(launch_da_init(ctx->a, ctx->stream), "adaptation init");
    if (st != HMC_OK) return st;
    if (total == 0) return HMC_OK;
    if (ctx->form == HMC_FORM_FUSED) {
        FusedRun r;
        memset(&r, 0, sizeof(r));
        r.t_begin = ctx->t;
        r.n_transitions = total;
        r.n_burnin = num_burnin_steps;
        r.m_offset = 0;
        r.adapt_total = num_burnin_steps;
        set_adapt(r, adapt);
        r.samples = samples;
        r.trace = tr;
        timer_begin(ctx->a, ctx->stream);
        st = check_hip(launch_fused(ctx->a, r, ctx->stream), "fused sample_chain");
        timer_end(ctx->a, ctx->stream, "fused transition kernel");
    } else {
        Ctrl c = base_ctrl(ctx);
        c.n_burnin = num_burnin_steps;
        c.n_results = num_results;
        set_adapt(c, adapt);
        c.samples = samples;
        c.tr_step = tr.step_size;
        c.tr_acc = tr.is_accepted;
        c.tr_lar = tr.log_accept_ratio;
        c.tr_logp = tr.target_log_prob;
        st = check_hip(launch_set_ctrl(c, ctx->a.ws.ctrl, ctx->stream), "sample_chain control");
        if (st == HMC_OK) st = run_transitions(ctx, total, false);
    }
    if (st == HMC_OK) ctx->t += (uint64_t)total;
    return st;
}

hmc_status hmc_get_state(hmc_ctx* ctx, void* state, double* step_size, uint64_t* t) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    const size_t es = ctx->a.f64 ? 8 : 4;
    hmc_status st = HMC_OK;
    if (state)
        st = check_hip(hipMemcpyAsync(state, ctx->a.ws.x, (size_t)ctx->a.C * ctx->a.tg.D * es,
                                      hipMemcpyDeviceToDevice, ctx->stream), "copy state");
    if (st == HMC_OK && step_size)
        st = check_hip(hipMemcpyAsync(step_size, ctx->a.ws.eps, (size_t)ctx->a.C * 8, hipMemcpyDeviceToDevice,
                                      ctx->stream), "copy step size");
    if (st == HMC_OK) st = check_hip(hipStreamSynchronize(ctx->stream), "get_state");
    if (st == HMC_OK && t) *t = ctx->t;
    return st;
}

hmc_status hmc_set_state(hmc_ctx* ctx, const void* state, const double* step_size, uint64_t t) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    if (!state) return fail(HMC_E_INVALID, "state must not be NULL");
    if (t > 0xffffffffull) return fail(HMC_E_INVALID, "t must be < 2^32");
    hmc_status st = HMC_OK;
    if (step_size)
        st = check_hip(hipMemcpyAsync(ctx->a.ws.eps, step_size, (size_t)ctx->a.C * 8, hipMemcpyDeviceToDevice,
                                      ctx->stream), "set step size");
    ctx->t = t;
    if (st == HMC_OK) st = check_hip(launch_set_ctrl(base_ctrl(ctx), ctx->a.ws.ctrl, ctx->stream), "set control");
    if (st == HMC_OK) st = check_hip(launch_bootstrap(ctx->a, state, ctx->stream), "bootstrap");
    return st;
}

static void timer_release(hmc_ctx* ctx) {
    KernelTimer& t = ctx->timer;
    if (t.ev) {
        for (int64_t i = 0; i < 2 * t.cap; ++i) (void)hipEventDestroy(t.ev[i]);
        delete[] t.ev;
    }
    t = KernelTimer{};
    ctx->a.timer = nullptr;
}

hmc_status hmc_destroy(hmc_ctx* ctx) {
    if (!ctx) return HMC_OK;
    hmc_status st = check_hip(hipStreamSynchronize(ctx->stream), "destroy");
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    timer_release(ctx);
    delete ctx;
    return st;
}

hmc_status hmc_kernel_timer_start(hmc_ctx* ctx, int64_t max_launches) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    if (max_launches < 1 || max_launches > (1 << 20)) return fail(HMC_E_INVALID, "max_launches must be in [1, 2^20]");
    hmc_status st = check_hip(hipStreamSynchronize(ctx->stream), "kernel timer");
    if (st != HMC_OK) return st;
    timer_release(ctx);
    KernelTimer& t = ctx->timer;
    t.ev = new hipEvent_t[(size_t)(2 * max_launches)];
    for (int64_t i = 0; i < 2 * max_launches; ++i) {
        st = check_hip(hipEventCreate(&t.ev[i]), "kernel timer events");
        if (st != HMC_OK) {
            t.cap = i / 2;       // events 0 .. 2 cap - 1 exist (an odd one is leaked to keep the pairs whole)
            timer_release(ctx);
            return st;
        }
    }
    t.cap = max_launches;
    ctx->a.timer = &t;
    return HMC_OK;
}

hmc_status hmc_kernel_timer_read(hmc_ctx* ctx, double* mean_ms, int64_t* launches, char* name, size_t name_len) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    KernelTimer& t = ctx->timer;
    if (!t.ev) return fail(HMC_E_INVALID, "kernel timer not started");
    hmc_status st = check_hip(hipStreamSynchronize(ctx->stream), "kernel timer");
    double total = 0.0;
    for (int64_t i = 0; st == HMC_OK && i < t.n; ++i) {
        float ms = 0.f;
        st = check_hip(hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]), "kernel timer elapsed");
        total += ms;
    }
    if (st == HMC_OK) {
        if (mean_ms) *mean_ms = t.n > 0 ? total / (double)t.n : 0.0;
        if (launches) *launches = t.n;
        if (name && name_len > 0) snprintf(name, name_len, "%s", t.name ? t.name : "");
    }
    timer_release(ctx);
    return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Sampling without device allocation: the workspace of hmc_sample_chain_noalloc
// is this file-scope array, one copy per GPU, held until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in for the symbol): the device address of each GPU's copy
// is looked up once per device with that device current and kept here.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[HMC_NOALLOC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

hmc_status scratch_for_device(int dev, void** out) {
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(HMC_E_DEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hmc_status st = check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch address");
        if (st != HMC_OK) return st;
        if (!ptr || ((uintptr_t)ptr & 255) != 0) return fail(HMC_E_DEVICE, "scratch address not 256-byte aligned");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HMC_OK;
}
}  // namespace

extern "C" {

hmc_status hmc_sample_chain_noalloc(const hmc_target* target, const hmc_config* config, const void* init_state,
                                    const double* step_size, int64_t step_size_len, int64_t num_results,
                                    int64_t num_burnin_steps, const hmc_adapt* adapt, void* samples,
                                    const hmc_trace* trace, void* final_state, double* final_step_size,
                                    void* hip_stream) {
    TargetDev t;
    hmc_status st = check_init_args(target, config, init_state, step_size, step_size_len, &t);
    if (st != HMC_OK) return st;
    if (config->form == HMC_FORM_GRAPH)
        return fail(HMC_E_UNSUPPORTED, "the graph form instantiates a graph, which allocates; use plain, fused or auto");
    if (num_results < 0 || num_burnin_steps < 0) return fail(HMC_E_INVALID, "negative transition count");
    if (num_results + num_burnin_steps > 0xffffffffll) return fail(HMC_E_INVALID, "more than 2^32 transitions");
    if (adapt && adapt->enabled && check_adapt(adapt) != HMC_OK) return HMC_E_INVALID;
    size_t need = 0;
    carve_workspace(nullptr, t, *config, &need);
    if (need > (size_t)HMC_NOALLOC_WORKSPACE_BYTES)
        return fail(HMC_E_NOMEM, "workspace of " + std::to_string(need) + " bytes exceeds the " +
                                     std::to_string((long long)HMC_NOALLOC_WORKSPACE_BYTES) +
                                     "-byte scratch of hmc_sample_chain_noalloc; use hmc_init with a workspace");

    // the stream's device must be the current one: its scratch copy is the one looked up
    int cur = -1, sdev = -1;
    st = check_hip(hipGetDevice(&cur), "current device");
    if (st == HMC_OK) st = check_hip(hipStreamGetDevice((hipStream_t)hip_stream, &sdev), "stream device");
    if (st != HMC_OK) return st;
    if (sdev != cur) return fail(HMC_E_INVALID, "hip_stream belongs to another device than the current one");
    void* ws = nullptr;
    st = scratch_for_device(cur, &ws);
    if (st != HMC_OK) return st;

    hmc_ctx ctx{};
    st = init_ctx(&ctx, t, config, init_state, step_size, step_size_len, ws, hip_stream);
    if (st == HMC_OK) st = hmc_sample_chain(&ctx, num_results, num_burnin_steps, adapt, samples, trace);
    const size_t es = ctx.a.f64 ? 8 : 4;
    if (st == HMC_OK && final_state)
        st = check_hip(hipMemcpyAsync(final_state, ctx.a.ws.x, (size_t)ctx.a.C * t.D * es, hipMemcpyDeviceToDevice,
                                      ctx.stream), "copy final state");
    if (st == HMC_OK && final_step_size)
        st = check_hip(hipMemcpyAsync(final_step_size, ctx.a.ws.eps, (size_t)ctx.a.C * 8, hipMemcpyDeviceToDevice,
                                      ctx.stream), "copy final step sizes");
    // the context ends with this call, so its work must have left the scratch
    const hmc_status sync = check_hip(hipStreamSynchronize((hipStream_t)hip_stream), "sample_chain_noalloc");
    return st != HMC_OK ? st : sync;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner: times the launch configurations that apply to this context with
// HIP events on its stream, restores the chain state after every trial, and
// keeps the fastest.  Choices are cached per (target family, D, log2 N,
// log2 C, dtypes, L, requested form) in memory and, when HMC_AUTOTUNE_CACHE
// names a file, on disk (one "key form lr_nsplit lr16_nsplit elem_gmult" line
// per entry).
// ---------------------------------------------------------------------------
namespace {
struct TuneChoice {
    int32_t form;
    Tune tune;
};
std::mutex g_tune_mu;
std::map<std::string, TuneChoice> g_tune_cache;
bool g_tune_loaded = false;

int ilog2(int64_t v) {
    int r = 0;
    while (v > 1) {
        v >>= 1;
        ++r;
    }
    return r;
}

std::string tune_key(const hmc_ctx* ctx) {
    std::ostringstream k;
    k << ctx->a.tg.kind << ":" << ctx->a.tg.D << ":" << ilog2(ctx->a.tg.N + 1) << ":" << ilog2(ctx->a.C) << ":"
      << ctx->cfg.state_dtype << ":" << ctx->cfg.grad_dtype << ":" << ctx->a.L << ":" << ctx->cfg.form;
    return k.str();
}

void load_cache_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("HMC_AUTOTUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string key;
    TuneChoice c;
    while (f >> key >> c.form >> c.tune.lr_nsplit >> c.tune.lr16_nsplit >> c.tune.elem_gmult) g_tune_cache[key] = c;
}

void store_cache_locked(const std::string& key, const TuneChoice& c) {
    g_tune_cache[key] = c;
    const char* path = std::getenv("HMC_AUTOTUNE_CACHE");
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << c.form << " " << c.tune.lr_nsplit << " " << c.tune.lr16_nsplit << " " << c.tune.elem_gmult
      << "\n";
}

hipError_t save_state(hmc_ctx* ctx, bool restore) {
    const Workspace& w = ctx->a.ws;
    const size_t state = (size_t)ctx->a.C * ctx->a.tg.D * (ctx->a.f64 ? 8 : 4);
    const size_t C = (size_t)ctx->a.C;
    struct {
        void* live;
        void* bk;
        size_t n;
    } parts[] = {{w.x, w.bk_x, state}, {w.g, w.bk_g, state}, {w.logp, w.bk_logp, C * 8},
                 {w.eps, w.bk_eps, C * 8}, {w.da, w.bk_da, C * sizeof(DualAvg)}};
    for (auto& p : parts) {
        hipError_t e = restore ? hipMemcpyAsync(p.live, p.bk, p.n, hipMemcpyDeviceToDevice, ctx->stream)
                               : hipMemcpyAsync(p.bk, p.live, p.n, hipMemcpyDeviceToDevice, ctx->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void drop_graph(hmc_ctx* ctx) {
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    ctx->graph_exec = nullptr;
    ctx->graph_ready = false;
}

// n burn-in transitions without adaptation, samples or traces (the state is restored afterwards)
hmc_status trial_run(hmc_ctx* ctx, int64_t n) {
    if (ctx->form == HMC_FORM_FUSED) {
        FusedRun r;
        memset(&r, 0, sizeof(r));
        r.t_begin = ctx->t;
        r.n_transitions = n;
        r.n_burnin = n;
        return check_hip(launch_fused(ctx->a, r, ctx->stream), "autotune trial");
    }
    Ctrl c = base_ctrl(ctx);
    c.n_burnin = n;
    hmc_status st = check_hip(launch_set_ctrl(c, ctx->a.ws.ctrl, ctx->stream), "autotune control");
    if (st == HMC_OK) st = run_transitions(ctx, n, false);
    return st;
}
}  // namespace

extern "C" hmc_status hmc_autotune(hmc_ctx* ctx, int32_t trial_transitions, char* report, size_t report_len) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    if (trial_transitions < 1) return fail(HMC_E_INVALID, "trial_transitions must be >= 1");
    const std::string key = tune_key(ctx);
    std::ostringstream rep;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_cache_locked();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            ctx->form = it->second.form;
            ctx->a.tune = it->second.tune;
            drop_graph(ctx);
            rep << "cached " << key << " form=" << ctx->form;
            if (report && report_len) snprintf(report, report_len, "%s", rep.str().c_str());
            return HMC_OK;
        }
    }
    std::vector<TuneChoice> cands;
    std::vector<int32_t> forms;
    if (ctx->cfg.form == HMC_FORM_AUTO) {
        if (fused_supported(ctx->a))
            forms.push_back(HMC_FORM_FUSED);
        forms.push_back(HMC_FORM_PLAIN);
        forms.push_back(HMC_FORM_GRAPH);
    } else {
        forms.push_back(ctx->form);
    }
    const bool elem = ctx->a.tg.kind == HMC_TGT_STD_NORMAL || ctx->a.tg.kind == HMC_TGT_GAUSS_DIAG;
    for (int32_t f : forms) {
        TuneChoice c{f, Tune{0, 0, 0}};
        if (f == HMC_FORM_FUSED && elem) {
            cands.push_back(c);
            c.tune.elem_gmult = 2;
            cands.push_back(c);
        } else if (f != HMC_FORM_FUSED && ctx->a.tg.kind == HMC_TGT_LOGREG && ctx->a.bf16_grad) {
            const int d = lb_grad_nsplit(ctx->a.tg.N, ctx->a.C, ctx->a.tg.D);
            for (int s : {d, 1, 2, 4, 8}) {
                bool seen = false;
                for (const TuneChoice& o : cands) seen |= o.form == f && o.tune.lr16_nsplit == s;
                if (seen) continue;
                c.tune.lr16_nsplit = s;
                cands.push_back(c);
            }
        } else if (f != HMC_FORM_FUSED && ctx->a.tg.kind == HMC_TGT_LOGREG) {
            const int64_t d = logreg_nsplit(ctx->a.tg.N, ctx->a.C);
            for (int64_t s : {d / 2, d, 2 * d})
                if (s >= 1 && s <= 64) {
                    c.tune.lr_nsplit = (int32_t)s;
                    cands.push_back(c);
                }
        } else {
            cands.push_back(c);
        }
    }
    const int32_t form0 = ctx->form;
    const Tune tune0 = ctx->a.tune;
    hmc_status st = check_hip(save_state(ctx, false), "autotune backup");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == HMC_OK) st = check_hip(hipEventCreate(&e0), "event");
    if (st == HMC_OK) st = check_hip(hipEventCreate(&e1), "event");
    float best = 1e30f;
    TuneChoice bestc{form0, tune0};
    for (size_t i = 0; st == HMC_OK && i < cands.size(); ++i) {
        ctx->form = cands[i].form;
        ctx->a.tune = cands[i].tune;
        drop_graph(ctx);
        st = trial_run(ctx, 1);   // warm-up (graph capture, code load)
        if (st == HMC_OK) st = check_hip(save_state(ctx, true), "autotune restore");
        if (st == HMC_OK) st = check_hip(hipEventRecord(e0, ctx->stream), "event");
        if (st == HMC_OK) st = trial_run(ctx, trial_transitions);
        if (st == HMC_OK) st = check_hip(hipEventRecord(e1, ctx->stream), "event");
        if (st == HMC_OK) st = check_hip(hipEventSynchronize(e1), "event");
        float ms = 0.f;
        if (st == HMC_OK) st = check_hip(hipEventElapsedTime(&ms, e0, e1), "event");
        if (st == HMC_OK) st = check_hip(save_state(ctx, true), "autotune restore");
        if (st != HMC_OK) break;
        rep << "form=" << cands[i].form << " lr_nsplit=" << cands[i].tune.lr_nsplit
            << " lr16_nsplit=" << cands[i].tune.lr16_nsplit << " elem_gmult=" << cands[i].tune.elem_gmult << ": "
            << ms / trial_transitions << " ms/transition\n";
        if (ms < best) {
            best = ms;
            bestc = cands[i];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ctx->form = st == HMC_OK ? bestc.form : form0;
    ctx->a.tune = st == HMC_OK ? bestc.tune : tune0;
    drop_graph(ctx);
    if (st == HMC_OK) st = check_hip(launch_set_ctrl(base_ctrl(ctx), ctx->a.ws.ctrl, ctx->stream), "control");
    if (st == HMC_OK) st = check_hip(hipStreamSynchronize(ctx->stream), "autotune");
    if (st == HMC_OK) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        store_cache_locked(key, bestc);
    }
    rep << "chosen form=" << ctx->form;
    if (report && report_len) snprintf(report, report_len, "%s", rep.str().c_str());
    return st;
}

// ---------------------------------------------------------------------------
// Replica exchange (paper Sec. 2.2): per-chain inverse temperatures on the
// plain / graph forms, the exchange step, and the driver that alternates one
// transition of every chain with one exchange step.
// ---------------------------------------------------------------------------
extern "C" {

hmc_status hmc_set_inverse_temperature(hmc_ctx* ctx, const double* beta) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    if (!beta) {
        ctx->a.ws.beta = nullptr;
        drop_graph(ctx);
        return HMC_OK;
    }
    std::vector<double> h((size_t)ctx->a.C);
    hmc_status st = check_hip(hipMemcpyAsync(h.data(), beta, h.size() * 8, hipMemcpyDeviceToHost, ctx->stream),
                              "read inverse temperatures");
    if (st == HMC_OK) st = check_hip(hipStreamSynchronize(ctx->stream), "read inverse temperatures");
    if (st != HMC_OK) return st;
    for (double b : h)
        if (!(b > 0.0) || !std::isfinite(b)) return fail(HMC_E_INVALID, "inverse temperatures must be finite and > 0");
    st = check_hip(hipMemcpyAsync(ctx->a.ws.beta_buf, h.data(), h.size() * 8, hipMemcpyHostToDevice, ctx->stream),
                   "set inverse temperatures");
    if (st == HMC_OK) st = check_hip(hipStreamSynchronize(ctx->stream), "set inverse temperatures");
    if (st != HMC_OK) return st;
    ctx->a.ws.beta = ctx->a.ws.beta_buf;
    drop_graph(ctx);    // captured launches hold the workspace pointers by value
    return HMC_OK;
}

static hmc_status remc_check(const hmc_ctx* ctx, int64_t num_replicas) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    if (num_replicas < 1 || ctx->a.C % num_replicas != 0)
        return fail(HMC_E_INVALID, "num_replicas must be >= 1 and divide the number of chains");
    return HMC_OK;
}

hmc_status hmc_remc_swap(hmc_ctx* ctx, int64_t num_replicas, uint64_t swap_index, uint8_t* swapped) {
    hmc_status st = remc_check(ctx, num_replicas);
    if (st != HMC_OK) return st;
    if (swap_index > 0xffffffffull) return fail(HMC_E_INVALID, "swap_index must be < 2^32");
    st = check_hip(launch_remc_swap(ctx->a, num_replicas, ctx->a.C / num_replicas, (uint32_t)swap_index,
                                        swapped, nullptr, ctx->stream), "exchange step");
    return st;
}

hmc_status hmc_remc_sample_chain(hmc_ctx* ctx, int64_t num_replicas, int64_t num_results, int64_t num_burnin_steps,
                                 const hmc_adapt* adapt, void* samples, const hmc_trace* trace,
                                 uint8_t* swapped) {
    hmc_status st = remc_check(ctx, num_replicas);
    if (st != HMC_OK) return st;
    if (num_results < 0 || num_burnin_steps < 0) return fail(HMC_E_INVALID, "negative transition count");
    const bool ad = adapt && adapt->enabled;
    if (ad && check_adapt(adapt) != HMC_OK) return HMC_E_INVALID;
    const int64_t total = num_results + num_burnin_steps;
    if (ctx->t + (uint64_t)total > 0xffffffffull) return fail(HMC_E_INVALID, "transition counter would exceed 2^32");
    const int64_t C = ctx->a.C, M = C / num_replicas;
    const size_t rowb = (size_t)C * ctx->a.tg.D * (ctx->a.f64 ? 8 : 4);
    hmc_trace tr;
    memset(&tr, 0, sizeof(tr));
    if (trace) tr = *trace;
    if (ad) st = check_hip(launch_da_init(ctx->a, ctx->stream), "adaptation init");
    if (ctx->form == HMC_FORM_FUSED && fused_remc_inline(ctx->a, num_replicas)) {
        // every replica of a chain index in one wavefront (element-wise) or workgroup (dense, logistic)
        // of the fused kernel, which exchanges between transitions itself -- one launch for the run
        FusedRun r;
        memset(&r, 0, sizeof(r));
        r.t_begin = ctx->t;
        r.n_transitions = total;
        r.n_burnin = num_burnin_steps;
        r.adapt_total = num_burnin_steps;
        set_adapt(r, adapt);
        r.samples = samples;
        r.trace = tr;
        r.remc_K = (int32_t)num_replicas;
        r.remc_M = M;
        r.swapped = swapped;
        if (st == HMC_OK && total > 0) st = check_hip(launch_fused(ctx->a, r, ctx->stream), "fused replica exchange");
        if (st == HMC_OK) ctx->t += (uint64_t)total;
        return st;
    }
    if (ctx->form == HMC_FORM_FUSED) {
        // one fused launch per transition (its trace row), then the exchange, which writes the kept sample row
        for (int64_t i = 0; i < total && st == HMC_OK; ++i) {
            const uint64_t t = ctx->t + (uint64_t)i;
            const bool kept = i >= num_burnin_steps;
            const size_t row = kept ? (size_t)(i - num_burnin_steps) * C : 0;
            FusedRun r;
            memset(&r, 0, sizeof(r));
            r.t_begin = t;
            r.n_transitions = 1;
            r.n_burnin = kept ? 0 : 1;
            r.m_offset = i;
            r.adapt_total = num_burnin_steps;
            set_adapt(r, adapt);
            if (kept) {
                r.trace.step_size = tr.step_size ? tr.step_size + row : nullptr;
                r.trace.is_accepted = tr.is_accepted ? tr.is_accepted + row : nullptr;
                r.trace.log_accept_ratio = tr.log_accept_ratio ? tr.log_accept_ratio + row : nullptr;
                r.trace.target_log_prob = tr.target_log_prob ? tr.target_log_prob + row : nullptr;
            }
            st = check_hip(launch_fused(ctx->a, r, ctx->stream), "fused remc transition");
            uint8_t* sw = (kept && swapped) ? swapped + row : nullptr;
            void* srow = (kept && samples) ? (char*)samples + (size_t)(i - num_burnin_steps) * rowb : nullptr;
            if (st == HMC_OK)
                st = check_hip(launch_remc_swap(ctx->a, num_replicas, M, (uint32_t)t, sw, srow, ctx->stream),
                               "exchange step");
        }
        if (st == HMC_OK) ctx->t += (uint64_t)total;
        return st;
    }
    // the transitions write the traces; the samples are taken after each exchange
    Ctrl c = base_ctrl(ctx);
    c.n_burnin = num_burnin_steps;
    c.n_results = num_results;
    set_adapt(c, adapt);
    c.samples = nullptr;
    c.tr_step = tr.step_size;
    c.tr_acc = tr.is_accepted;
    c.tr_lar = tr.log_accept_ratio;
    c.tr_logp = tr.target_log_prob;
    if (st == HMC_OK) st = check_hip(launch_set_ctrl(c, ctx->a.ws.ctrl, ctx->stream), "remc control");
    for (int64_t i = 0; i < total && st == HMC_OK; ++i) {
        const uint64_t t = ctx->t + (uint64_t)i;
        const bool kept = i >= num_burnin_steps;
        uint8_t* sw = (kept && swapped) ? swapped + (size_t)(i - num_burnin_steps) * C : nullptr;
        void* srow = (kept && samples) ? (char*)samples + (size_t)(i - num_burnin_steps) * rowb : nullptr;
        st = run_transitions(ctx, 1, false);
        if (st == HMC_OK)
            st = check_hip(launch_remc_swap(ctx->a, num_replicas, M, (uint32_t)t, sw, srow, ctx->stream),
                           "exchange step");
    }
    if (st == HMC_OK) ctx->t += (uint64_t)total;
    return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Streaming expectations: burn-in, then the kept transitions in chunks of the
// ring's rows, each chunk written into the ring by the form's own kernels and
// folded into the moments by k_moments.
// ---------------------------------------------------------------------------
extern "C" hmc_status hmc_sample_chain_moments(hmc_ctx* ctx, int64_t num_results, int64_t num_burnin_steps,
                                               const hmc_adapt* adapt, const hmc_moments* moments,
                                               const hmc_trace* trace) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    if (!moments || !moments->mean || !moments->m2 || !moments->ring)
        return fail(HMC_E_INVALID, "moments, mean, m2 and ring must not be NULL");
    if (moments->ring_rows < 1) return fail(HMC_E_INVALID, "ring_rows must be >= 1");
    if (num_results < 0 || num_burnin_steps < 0) return fail(HMC_E_INVALID, "negative transition count");
    if (moments->batch_sum && (moments->batch_len < 1 || num_results % moments->batch_len != 0))
        return fail(HMC_E_INVALID, "batch_len must be >= 1 and divide num_results");
    if (adapt && adapt->enabled && check_adapt(adapt) != HMC_OK) return HMC_E_INVALID;
    if (ctx->t + (uint64_t)(num_results + num_burnin_steps) > 0xffffffffull)
        return fail(HMC_E_INVALID, "transition counter would exceed 2^32");
    const int64_t n_el = ctx->a.C * ctx->a.tg.D;
    hmc_status st = check_hip(launch_fill_f64(moments->mean, 2 * n_el, ctx->stream), "clear moments");
    if (st == HMC_OK) st = check_hip(launch_fill_f64(moments->m2, 2 * n_el, ctx->stream), "clear moments");
    if (st == HMC_OK && moments->batch_sum)
        st = check_hip(launch_fill_f64(moments->batch_sum, (num_results / moments->batch_len) * n_el, ctx->stream),
                       "clear batch sums");
    if (st == HMC_OK && num_burnin_steps > 0) st = hmc_sample_chain(ctx, 0, num_burnin_steps, adapt, nullptr, nullptr);
    for (int64_t r0 = 0; r0 < num_results && st == HMC_OK; r0 += moments->ring_rows) {
        const int64_t q = std::min<int64_t>(moments->ring_rows, num_results - r0);
        hmc_trace tr;
        memset(&tr, 0, sizeof(tr));
        if (trace) {
            const size_t off = (size_t)r0 * ctx->a.C;
            tr.step_size = trace->step_size ? trace->step_size + off : nullptr;
            tr.is_accepted = trace->is_accepted ? trace->is_accepted + off : nullptr;
            tr.log_accept_ratio = trace->log_accept_ratio ? trace->log_accept_ratio + off : nullptr;
            tr.target_log_prob = trace->target_log_prob ? trace->target_log_prob + off : nullptr;
        }
        st = hmc_sample_chain(ctx, q, 0, nullptr, moments->ring, &tr);
        if (st == HMC_OK)
            st = check_hip(launch_moments(ctx->a, moments->ring, q, r0, num_results, *moments, ctx->stream),
                           "fold moments");
    }
    return st;
}

// ---------------------------------------------------------------------------
// Transformed kernel (paper Sec. 4.1) with the diagonal affine bijector
// x = shift + scale z.  The plain kernels run in x: the momentum lives in z,
// so scale multiplies the momentum in every drift and the gradient in every
// kick (the shift drops out).  The fused kernels run in z = x / scale against
// the pulled-back target (precision S P S; logistic: X S and the prior's
// precision scaled per dim).  FP32 gradients.
// ---------------------------------------------------------------------------
extern "C" hmc_status hmc_set_transform_scale(hmc_ctx* ctx, const double* scale) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    if (!scale) {
        ctx->a.ws.scale = nullptr;
        drop_graph(ctx);
        return HMC_OK;
    }
    if (ctx->a.bf16_grad) return fail(HMC_E_UNSUPPORTED, "the transformed kernel needs FP32 gradients");
    std::vector<double> h((size_t)ctx->a.tg.D);
    hmc_status st = check_hip(hipMemcpyAsync(h.data(), scale, h.size() * 8, hipMemcpyDeviceToHost, ctx->stream),
                              "read scale");
    if (st == HMC_OK) st = check_hip(hipStreamSynchronize(ctx->stream), "read scale");
    if (st != HMC_OK) return st;
    for (double v : h)
        if (!(v > 0.0) || !std::isfinite(v)) return fail(HMC_E_INVALID, "scale must be finite and > 0");
    st = check_hip(hipMemcpyAsync(ctx->a.ws.scale_buf, h.data(), h.size() * 8, hipMemcpyHostToDevice, ctx->stream),
                   "set scale");
    if (st == HMC_OK) st = check_hip(hipStreamSynchronize(ctx->stream), "set scale");
    if (st != HMC_OK) return st;
    ctx->a.ws.scale = ctx->a.ws.scale_buf;
    drop_graph(ctx);
    return HMC_OK;
}

// ---------------------------------------------------------------------------
// No-U-Turn sampler (paper Sec. 2.3): the unrolled tree on the plain kernels,
// all chains in lockstep, a chain masked once its trajectory stops; the host
// reads the number of chains still running after every doubling.
// ---------------------------------------------------------------------------
extern "C" hmc_status hmc_nuts_workspace_size(const hmc_ctx* ctx, int32_t max_depth, size_t* bytes) {
    if (!ctx || !bytes) return fail(HMC_E_INVALID, "ctx and bytes must not be NULL");
    if (max_depth < 0 || max_depth > 10) return fail(HMC_E_INVALID, "max_depth must be in 0..10");
    carve_nuts(nullptr, ctx->a.C, ctx->a.tg.D, max_depth, ctx->a.f64 ? 8 : 4, nuts_l2_rows(ctx->a), bytes);
    return HMC_OK;
}

extern "C" hmc_status hmc_nuts_sample_chain(hmc_ctx* ctx, int32_t max_depth, int64_t num_results,
                                            int64_t num_burnin_steps, const hmc_adapt* adapt, void* nuts_workspace,
                                            size_t nuts_workspace_bytes, void* samples, int32_t* tree_depth,
                                            int32_t* n_leapfrog, double* accept_stat) {
    if (!ctx) return fail(HMC_E_INVALID, "ctx must not be NULL");
    if (hmc_status st = check_adapt(adapt)) return st;
    if (max_depth < 0 || max_depth > 10) return fail(HMC_E_INVALID, "max_depth must be in 0..10");
    if (num_results < 0 || num_burnin_steps < 0) return fail(HMC_E_INVALID, "negative transition count");
    if (ctx->a.ws.beta || ctx->a.ws.scale)
        return fail(HMC_E_UNSUPPORTED, "NUTS runs without inverse temperatures or a transform");
    if (!nuts_workspace) return fail(HMC_E_INVALID, "nuts_workspace must not be NULL");
    size_t need = 0;
    NutsWs nw = carve_nuts(nuts_workspace, ctx->a.C, ctx->a.tg.D, max_depth, ctx->a.f64 ? 8 : 4,
                           nuts_l2_rows(ctx->a), &need);
    if (nuts_workspace_bytes < need) return fail(HMC_E_NOMEM, "NUTS workspace smaller than hmc_nuts_workspace_size");
    const int64_t total = num_results + num_burnin_steps;
    if (ctx->t + (uint64_t)total > 0xffffffffull) return fail(HMC_E_INVALID, "transition counter would exceed 2^32");
    NutsAdapt ad{};
    set_adapt(ad, adapt);
    ad.n_burnin = num_burnin_steps;
    hmc_status st = HMC_OK;
    if (ad.adapt && ad.adapt_kind == HMC_ADAPT_DUAL_AVERAGING)
        st = check_hip(launch_da_init(ctx->a, ctx->stream), "adaptation init");
    if (st != HMC_OK) return st;
    if ((ctx->form == HMC_FORM_FUSED || ctx->cfg.form == HMC_FORM_AUTO) && nuts_fused_supported(ctx->a)) {
        // element-wise targets: one persistent launch for all transitions
        st = check_hip(launch_nuts_fused(ctx->a, nw, ad, (uint32_t)ctx->t, total, max_depth, samples, tree_depth,
                                         n_leapfrog, accept_stat, ctx->stream),
                       "nuts persistent");
        if (st == HMC_OK) ctx->t += (uint64_t)total;
        return st;
    }
    PlainArgs leap = ctx->a;
    leap.ws.eps = nw.seps;             // signed step v eps of each chain's current doubling
    for (int64_t it = 0; it < total && st == HMC_OK; ++it) {
        const uint32_t t = (uint32_t)(ctx->t + (uint64_t)it);
        st = check_hip(launch_nuts_begin(ctx->a, nw, t, ctx->stream), "nuts begin");
        for (int32_t j = 0; j < max_depth && st == HMC_OK; ++j) {
            st = check_hip(launch_nuts_dir(ctx->a, nw, t, j, ctx->stream), "nuts direction");
            for (int32_t i = 0; i < (1 << j) && st == HMC_OK; ++i) {
                st = check_hip(launch_nuts_halfkick(leap, nw, ctx->stream), "nuts half kick");
                if (st == HMC_OK) st = check_hip(launch_leapfrog_step(leap, 0.5, ctx->stream), "nuts leapfrog");
                if (st == HMC_OK) st = check_hip(launch_nuts_leaf(ctx->a, nw, t, j, i, ctx->stream), "nuts leaf");
            }
            if (st == HMC_OK) st = check_hip(launch_nuts_doubling_end(ctx->a, nw, t, j, ctx->stream), "nuts doubling");
            int32_t running = 0;
            if (st == HMC_OK)
                st = check_hip(hipMemcpyAsync(&running, nw.n_active, 4, hipMemcpyDeviceToHost, ctx->stream),
                               "nuts count");
            if (st == HMC_OK) st = check_hip(hipStreamSynchronize(ctx->stream), "nuts count");
            if (st != HMC_OK || running == 0) break;
        }
        const int64_t r = it >= num_burnin_steps ? it - num_burnin_steps : -1;   // kept draw, or -1
        if (st == HMC_OK)
            st = check_hip(launch_nuts_end(ctx->a, nw, ad, it, samples, r, tree_depth, n_leapfrog, accept_stat,
                                           ctx->stream),
                           "nuts end");
    }
    if (st == HMC_OK) ctx->t += (uint64_t)total;
    return st;
}
