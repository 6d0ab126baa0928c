// hmc_server.hip -- continuous batching of sampling requests on one GPU
// (hmc_server_* in include/hmc.h).
//
// One worker thread owns every HIP call.  Each loop iteration ("tick"):
//   1. admits queued requests whose memory fits the free part of the device
//      pool (first fit, arrival order with backfill), runs their bootstrap;
//   2. advances every active request by up to transitions_per_tick
//      transitions: elementwise requests of one shape class in a single ragged
//      launch (a device job table maps blocks to requests), every other request
//      on one of a few HIP streams so their kernels overlap on the device;
//   3. retires requests that reached burn-in + results transitions and frees
//      their memory (or keeps server-owned samples until hmc_server_take).
// Chain state, gradients, log-probabilities, step sizes and dual-averaging
// state stay in the pool between ticks; the fused kernels resume mid-run from
// that state, so a request's result is the same as one hmc_sample_chain call.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <tuple>
#include <mutex>
#include <thread>
#include <vector>

#include "hmc_internal.hpp"

using namespace hmc;

namespace {

constexpr int kStreams = 4;
constexpr int kMaxJobs = 256;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) with 256-byte granularity.
class PoolAlloc {
public:
    explicit PoolAlloc(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        used_ -= bytes;
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
    size_t used() const { return used_; }
    size_t size() const { return size_; }

private:
    size_t size_, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Request {
    uint64_t id;
    hmc_request req;
    PlainArgs a;
    int form;                 // HMC_FORM_FUSED or HMC_FORM_PLAIN
    int cls;                  // elementwise shape class or -1
    size_t ws_bytes, smp_bytes, off = 0;
    bool owns_samples = false;
    void* samples = nullptr;  // where samples go (caller's or pool)
    int64_t done = 0, total = 0;
    int state = HMC_REQ_QUEUED;
    std::vector<double> eps_host;
    std::chrono::steady_clock::time_point t_submit, t_done;
    bool memory_held = false;
};

}  // namespace

struct hmc_server {
    size_t budget;
    int K;
    int device = 0;
    void* pool = nullptr;
    PoolAlloc* alloc = nullptr;
    hipStream_t streams[kStreams] = {};
    ElemJob* jobs_host = nullptr;   // pinned
    ElemJob* jobs_dev = nullptr;
    Lr16Job* lr16_host = nullptr;   // pinned
    Lr16Job* lr16_dev = nullptr;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Request*> pending;
    std::vector<Request*> active;
    std::map<uint64_t, Request*> all;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    hmc_server_stats st{};
};

namespace {

size_t request_bytes(const hmc_request& r, const TargetDev& t, size_t* ws, size_t* smp, bool* owns) {
    carve_workspace(nullptr, t, r.config, ws);
    *owns = r.samples == nullptr && r.num_results > 0;
    *smp = *owns ? (size_t)r.num_results * r.config.num_chains * t.D * elem_size(r.config.state_dtype) : 0;
    return align256(*ws) + align256(*smp);
}

// bootstrap of one admitted request on stream s (mirrors hmc_init)
hipError_t admit(Request* q, void* pool, hipStream_t s) {
    PlainArgs& a = q->a;
    char* base = (char*)pool + q->off;
    a.ws = carve_workspace(base, a.tg, q->req.config, nullptr);
    q->samples = q->owns_samples ? (void*)(base + align256(q->ws_bytes)) : q->req.samples;
    q->eps_host.assign((size_t)a.C, q->req.step_size);
    hipError_t e = hipMemcpyAsync(a.ws.eps, q->eps_host.data(), (size_t)a.C * 8, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    if (a.bf16_grad && (e = launch_pad_bf16(a, s)) != hipSuccess) return e;
    Ctrl c;
    memset(&c, 0, sizeof(c));
    c.n_burnin = q->req.num_burnin;
    c.n_results = q->req.num_results;
    set_adapt(c, &q->req.adapt);
    c.samples = q->samples;
    c.tr_step = q->req.trace.step_size;
    c.tr_acc = q->req.trace.is_accepted;
    c.tr_lar = q->req.trace.log_accept_ratio;
    c.tr_logp = q->req.trace.target_log_prob;
    if ((e = launch_set_ctrl(c, a.ws.ctrl, s)) != hipSuccess) return e;
    if ((e = launch_bootstrap(a, q->req.init_state, s)) != hipSuccess) return e;
    return launch_da_init(a, s);
}

// a request whose gradient launch alone has a workgroup for every CU gains nothing
// from sharing launches and would hold back the small requests it shares them with
bool lr16_fills_gpu(const PlainArgs& a) {
    Lr16Job j;
    lr16_job_shape(a, &j);
    return j.nblk[LR16_KIND_GRAD] >= 256;
}

// the launch parameters of the next n transitions of a fused request
FusedRun tick_run(const Request* q, int64_t n) {
    FusedRun r;
    memset(&r, 0, sizeof(r));
    const int64_t B = q->req.num_burnin, C = q->a.C, D = q->a.tg.D;
    const size_t es = q->a.f64 ? 8 : 4;
    r.t_begin = (uint64_t)q->done;
    r.n_transitions = n;
    r.n_burnin = std::max<int64_t>(0, std::min<int64_t>(n, B - q->done));
    r.m_offset = std::min<int64_t>(q->done, B);
    r.adapt_total = B;
    set_adapt(r, &q->req.adapt);
    const int64_t kept_before = std::max<int64_t>(0, q->done - B);
    if (q->samples) r.samples = (char*)q->samples + (size_t)kept_before * C * D * es;
    const hmc_trace& tr = q->req.trace;
    if (tr.step_size) r.trace.step_size = tr.step_size + kept_before * C;
    if (tr.is_accepted) r.trace.is_accepted = tr.is_accepted + kept_before * C;
    if (tr.log_accept_ratio) r.trace.log_accept_ratio = tr.log_accept_ratio + kept_before * C;
    if (tr.target_log_prob) r.trace.target_log_prob = tr.target_log_prob + kept_before * C;
    return r;
}

void release_memory(hmc_server* srv, Request* q, bool keep_samples) {
    if (!q->memory_held) return;
    if (keep_samples && q->owns_samples) {
        // keep the sample buffer, give back the workspace part
        if (q->ws_bytes == 0) return;
        srv->alloc->release(q->off, q->ws_bytes);
        q->off += align256(q->ws_bytes);
        q->ws_bytes = 0;
        return;
    }
    srv->alloc->release(q->off, align256(q->ws_bytes) + align256(q->smp_bytes));
    q->memory_held = false;
}

void worker_loop(hmc_server* srv) {
    (void)hipSetDevice(srv->device);
    int rr = 0;
    for (;;) {
        std::vector<Request*> newly;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->cv.wait(lk, [&] { return srv->stop || !srv->pending.empty() || !srv->active.empty(); });
            if (srv->stop && srv->pending.empty() && srv->active.empty()) return;
            // admission in arrival order with backfill
            for (auto it = srv->pending.begin(); it != srv->pending.end();) {
                Request* q = *it;
                size_t off;
                if (srv->alloc->alloc(align256(q->ws_bytes) + align256(q->smp_bytes), &off)) {
                    q->off = off;
                    q->memory_held = true;
                    q->state = HMC_REQ_RUNNING;
                    newly.push_back(q);
                    it = srv->pending.erase(it);
                } else {
                    ++it;
                }
            }
            srv->st.bytes_in_use = srv->alloc->used();
            srv->st.peak_bytes_in_use = std::max(srv->st.peak_bytes_in_use, srv->st.bytes_in_use);
        }
        for (Request* q : newly) {
            const hipError_t e = admit(q, srv->pool, srv->streams[rr++ % kStreams]);
            std::lock_guard<std::mutex> lk(srv->mu);
            if (e != hipSuccess) {
                q->state = HMC_REQ_FAILED;
                release_memory(srv, q, false);
                srv->st.failed++;
                srv->cv_done.notify_all();
            } else {
                srv->active.push_back(q);
                srv->st.admitted++;
            }
        }
        for (int k = 0; k < kStreams; ++k) (void)hipStreamSynchronize(srv->streams[k]);
        std::vector<Request*> act;
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            act = srv->active;
            srv->st.active = (int64_t)act.size();
            srv->st.pending = (int64_t)srv->pending.size();
            srv->st.max_active = std::max(srv->st.max_active, (int64_t)act.size());
        }
        if (act.empty()) continue;

        // ---- one tick ----
        std::map<int, std::vector<Request*>> classes;
        std::map<std::tuple<int, int, int>, std::vector<Request*>> lr16_classes;
        std::vector<Request*> others;
        for (Request* q : act) {
            if (q->form == HMC_FORM_FUSED && q->cls >= 0) {
                classes[q->cls].push_back(q);
            } else if (q->form == HMC_FORM_PLAIN && lr16_batch_class(q->a) >= 0 && !lr16_fills_gpu(q->a)) {
                lr16_classes[std::make_tuple(lr16_batch_class(q->a), plain_chain_group(q->a.tg.D), q->a.L)]
                    .push_back(q);
            } else {
                others.push_back(q);
            }
        }
        for (auto& kv : lr16_classes)   // a class of one runs as an ordinary plain request
            if (kv.second.size() == 1) others.push_back(kv.second[0]);
        bool ok = true;
        int njob = 0;
        for (auto& kv : classes) {
            // one ragged launch per class (chunks of kMaxJobs)
            for (size_t b0 = 0; b0 < kv.second.size(); b0 += kMaxJobs) {
                const size_t b1 = std::min(kv.second.size(), b0 + kMaxJobs);
                const int first = njob;
                int64_t blocks = 0;
                for (size_t i = b0; i < b1; ++i) {
                    Request* q = kv.second[i];
                    ElemJob& j = srv->jobs_host[njob++];
                    j.a = q->a;
                    j.r = tick_run(q, std::min<int64_t>(srv->K, q->total - q->done));
                    j.block_begin = blocks;
                    blocks += elem_blocks(q->a);
                }
                const int n = njob - first;
                hipStream_t s = srv->streams[0];
                if (hipMemcpyAsync(srv->jobs_dev + first, srv->jobs_host + first, sizeof(ElemJob) * n,
                                   hipMemcpyHostToDevice, s) != hipSuccess ||
                    launch_fused_elem_multi(kv.first, srv->jobs_dev + first, n, blocks, s) != hipSuccess)
                    ok = false;
                if (n >= 2) srv->st.batched_launches++;
                if (njob + kMaxJobs > 4 * kMaxJobs) {   // job table reuse needs the copies done
                    (void)hipStreamSynchronize(s);
                    njob = 0;
                }
            }
        }
        // BF16-gradient logistic plain requests of one class: transition i of the tick
        // runs once for every member with more than i transitions left (chunks of kMaxJobs)
        // on the streams of the other requests (stream 0 carries the element-wise classes), so
        // that classes overlap
        int si = 1;
        int nlr = 0;
        for (auto& kv : lr16_classes) {
            if (kv.second.size() < 2) continue;
            for (size_t b0 = 0; b0 < kv.second.size() && ok; b0 += kMaxJobs) {
                const size_t b1 = std::min(kv.second.size(), b0 + kMaxJobs);
                hipStream_t s = srv->streams[si++ % kStreams];
                int first = -1, n = 0;
                for (int64_t i = 0; i < srv->K && ok; ++i) {
                    std::vector<Request*> mem;
                    for (size_t k = b0; k < b1; ++k)
                        if (kv.second[k]->total - kv.second[k]->done > i) mem.push_back(kv.second[k]);
                    if (mem.empty()) break;
                    if ((int)mem.size() != n) {   // the set only shrinks: a new table when it does
                        if (nlr + (int)mem.size() > 4 * kMaxJobs) {   // table reuse needs every copy done
                            for (int k = 0; k < kStreams; ++k) (void)hipStreamSynchronize(srv->streams[k]);
                            nlr = 0;
                        }
                        first = nlr;
                        n = (int)mem.size();
                        for (int k = 0; k < n; ++k) srv->lr16_host[first + k].a = mem[k]->a;
                        nlr += n;
                        if (!lr16_layout(srv->lr16_host + first, n) ||
                            hipMemcpyAsync(srv->lr16_dev + first, srv->lr16_host + first, sizeof(Lr16Job) * n,
                                           hipMemcpyHostToDevice, s) != hipSuccess) {
                            ok = false;
                            break;
                        }
                    }
                    if (n == 1) {
                        if (launch_plain_transition(mem[0]->a, false, s) != hipSuccess) ok = false;
                    } else {
                        if (launch_lr16_transition_multi(srv->lr16_host + first, srv->lr16_dev + first, n, s) !=
                            hipSuccess)
                            ok = false;
                        srv->st.batched_plain_transitions++;
                    }
                }
            }
        }
        for (Request* q : others) {
            hipStream_t s = srv->streams[si++ % kStreams];
            const int64_t n = std::min<int64_t>(srv->K, q->total - q->done);
            if (q->form == HMC_FORM_FUSED) {
                if (launch_fused(q->a, tick_run(q, n), s) != hipSuccess) ok = false;
            } else {
                for (int64_t i = 0; i < n && ok; ++i)
                    if (launch_plain_transition(q->a, false, s) != hipSuccess) ok = false;
            }
        }
        hipError_t se = hipSuccess;
        for (int k = 0; k < kStreams; ++k) {
            hipError_t e = hipStreamSynchronize(srv->streams[k]);
            if (e != hipSuccess) se = e;
        }
        const auto now = std::chrono::steady_clock::now();
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->st.ticks++;
        for (Request* q : act) {
            q->done = std::min<int64_t>(q->total, q->done + srv->K);
            if (!ok || se != hipSuccess) {
                q->state = HMC_REQ_FAILED;
                srv->st.failed++;
            } else if (q->done >= q->total) {
                q->state = HMC_REQ_DONE;
                q->t_done = now;
                srv->st.completed++;
            } else {
                continue;
            }
            release_memory(srv, q, q->state == HMC_REQ_DONE);
            srv->active.erase(std::find(srv->active.begin(), srv->active.end(), q));
        }
        srv->st.bytes_in_use = srv->alloc->used();
        srv->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

hmc_status hmc_server_create(size_t hbm_budget_bytes, int32_t transitions_per_tick, hmc_server** out) {
    if (!out) return fail(HMC_E_INVALID, "out must not be NULL");
    if (transitions_per_tick < 1) return fail(HMC_E_INVALID, "transitions_per_tick must be >= 1");
    if (hbm_budget_bytes < 4096) return fail(HMC_E_INVALID, "hbm budget too small");
    hmc_server* srv = new hmc_server();
    srv->budget = align256(hbm_budget_bytes);
    srv->K = transitions_per_tick;
    (void)hipGetDevice(&srv->device);
    bool ok = hipMalloc(&srv->pool, srv->budget) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&srv->jobs_host, sizeof(ElemJob) * 4 * kMaxJobs, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMalloc((void**)&srv->jobs_dev, sizeof(ElemJob) * 4 * kMaxJobs) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&srv->lr16_host, sizeof(Lr16Job) * 4 * kMaxJobs, hipHostMallocDefault) ==
                   hipSuccess;
    ok = ok && hipMalloc((void**)&srv->lr16_dev, sizeof(Lr16Job) * 4 * kMaxJobs) == hipSuccess;
    for (int k = 0; ok && k < kStreams; ++k)
        ok = hipStreamCreateWithFlags(&srv->streams[k], hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        if (srv->pool) (void)hipFree(srv->pool);
        if (srv->jobs_host) (void)hipHostFree(srv->jobs_host);
        if (srv->jobs_dev) (void)hipFree(srv->jobs_dev);
        if (srv->lr16_host) (void)hipHostFree(srv->lr16_host);
        if (srv->lr16_dev) (void)hipFree(srv->lr16_dev);
        for (int k = 0; k < kStreams; ++k)
            if (srv->streams[k]) (void)hipStreamDestroy(srv->streams[k]);
        delete srv;
        return fail(HMC_E_NOMEM, "cannot allocate the server pool");
    }
    srv->alloc = new PoolAlloc(srv->budget);
    srv->st.pool_bytes = srv->budget;
    srv->worker = std::thread(worker_loop, srv);
    *out = srv;
    return HMC_OK;
}

hmc_status hmc_server_submit(hmc_server* srv, const hmc_request* req, uint64_t* id) {
    if (!srv || !req || !id) return fail(HMC_E_INVALID, "server, request and id must not be NULL");
    TargetDev t;
    hmc_status stt = validate_args(&req->target, &req->config, &t);
    if (stt != HMC_OK) return stt;
    if (!req->init_state) return fail(HMC_E_INVALID, "init_state must not be NULL");
    if (!(req->step_size > 0.0) || !std::isfinite(req->step_size)) return fail(HMC_E_INVALID, "bad step size");
    if (req->num_results < 0 || req->num_burnin < 0) return fail(HMC_E_INVALID, "negative transition count");
    if (req->num_results + req->num_burnin > 0xffffffffll) return fail(HMC_E_INVALID, "too many transitions");
    if (check_adapt(&req->adapt) != HMC_OK) return HMC_E_INVALID;
    if (req->config.form == HMC_FORM_GRAPH) return fail(HMC_E_UNSUPPORTED, "serving runs the plain or fused form");
    Request* q = new Request();
    q->req = *req;
    PlainArgs& a = q->a;
    a.tg = t;
    a.C = req->config.num_chains;
    a.L = req->config.num_leapfrog_steps;
    a.f64 = req->config.state_dtype == HMC_F64;
    a.bf16_grad = req->config.grad_dtype == HMC_BF16;
    a.key = make_key(req->config.seed);
    const bool can_fuse = fused_supported(a);
    if (req->config.form == HMC_FORM_FUSED && !can_fuse) {
        delete q;
        return fail(HMC_E_UNSUPPORTED, "no fused kernel for this target shape");
    }
    q->form = (req->config.form == HMC_FORM_PLAIN || !can_fuse) ? HMC_FORM_PLAIN : HMC_FORM_FUSED;
    q->cls = q->form == HMC_FORM_FUSED ? elem_class(a) : -1;
    const size_t need = request_bytes(*req, t, &q->ws_bytes, &q->smp_bytes, &q->owns_samples);
    if (need > srv->budget) {
        delete q;
        return fail(HMC_E_NOMEM, "request needs more device memory than the whole server budget");
    }
    q->total = req->num_results + req->num_burnin;
    q->t_submit = std::chrono::steady_clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        q->id = srv->next_id++;
        srv->all[q->id] = q;
        if (q->total == 0) {
            q->state = HMC_REQ_DONE;
            q->t_done = q->t_submit;
            srv->st.completed++;
        } else {
            srv->pending.push_back(q);
        }
        srv->st.submitted++;
        *id = q->id;
    }
    srv->cv.notify_all();
    return HMC_OK;
}

static hmc_status report(hmc_server* srv, uint64_t id, int32_t* state, double* latency_s, bool wait) {
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->all.find(id);
    if (it == srv->all.end()) return fail(HMC_E_INVALID, "unknown request id");
    Request* q = it->second;
    if (wait) srv->cv_done.wait(lk, [&] { return q->state == HMC_REQ_DONE || q->state == HMC_REQ_FAILED; });
    if (state) *state = q->state;
    if (latency_s)
        *latency_s = q->state == HMC_REQ_DONE ? std::chrono::duration<double>(q->t_done - q->t_submit).count() : -1.0;
    return q->state == HMC_REQ_FAILED ? fail(HMC_E_DEVICE, "request failed on the device") : HMC_OK;
}

hmc_status hmc_server_poll(hmc_server* srv, uint64_t id, int32_t* state, double* latency_s) {
    if (!srv) return fail(HMC_E_INVALID, "server must not be NULL");
    return report(srv, id, state, latency_s, false);
}

hmc_status hmc_server_wait(hmc_server* srv, uint64_t id, int32_t* state, double* latency_s) {
    if (!srv) return fail(HMC_E_INVALID, "server must not be NULL");
    return report(srv, id, state, latency_s, true);
}

hmc_status hmc_server_take(hmc_server* srv, uint64_t id, void* dst_samples) {
    if (!srv || !dst_samples) return fail(HMC_E_INVALID, "server and dst must not be NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->all.find(id);
    if (it == srv->all.end()) return fail(HMC_E_INVALID, "unknown request id");
    Request* q = it->second;
    if (q->state != HMC_REQ_DONE) return fail(HMC_E_BUSY, "request not done");
    if (!q->owns_samples || !q->memory_held) return fail(HMC_E_INVALID, "request has no server-held samples");
    const size_t n = q->smp_bytes;
    const void* src = (char*)srv->pool + q->off;
    lk.unlock();
    hmc_status st = HMC_OK;
    if (hipMemcpy(dst_samples, src, n, hipMemcpyDeviceToDevice) != hipSuccess)
        st = fail(HMC_E_DEVICE, "copy of samples failed");
    lk.lock();
    srv->alloc->release(q->off, q->smp_bytes);
    q->memory_held = false;
    srv->st.bytes_in_use = srv->alloc->used();
    return st;
}

hmc_status hmc_server_get_stats(hmc_server* srv, hmc_server_stats* out) {
    if (!srv || !out) return fail(HMC_E_INVALID, "server and out must not be NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->st;
    out->active = (int64_t)srv->active.size();
    out->pending = (int64_t)srv->pending.size();
    return HMC_OK;
}

hmc_status hmc_server_destroy(hmc_server* srv) {
    if (!srv) return HMC_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    srv->worker.join();
    for (int k = 0; k < kStreams; ++k) (void)hipStreamDestroy(srv->streams[k]);
    (void)hipFree(srv->pool);
    (void)hipFree(srv->jobs_dev);
    (void)hipHostFree(srv->jobs_host);
    (void)hipFree(srv->lr16_dev);
    (void)hipHostFree(srv->lr16_host);
    for (auto& kv : srv->all) delete kv.second;
    delete srv->alloc;
    delete srv;
    return HMC_OK;
}

}  // extern "C"
