// Continuous-batching request server over the hot path (declared in topo_serve.h).
//
// One dispatcher thread turns queued requests into jobs and hands them to idle
// workers; each worker owns a HIP stream and a library context and runs its job with
// the ordinary entry points, so jobs of different workers overlap on the device.
// Admission keeps the resident meshes and bases plus the device workspace held by all
// workers within the budget.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "internal.hpp"
#include "topo_serve.h"

namespace topo {
namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct MeshRec {
    topo_mesh mesh;
    Grid g;
    uint8_t* mask = nullptr;
    double* f = nullptr;
};

struct BasisRec {
    int mesh_id = 0;
    void* phi = nullptr;
    int fp32 = 1;
    int kmax = 0;
};

struct Req {
    uint64_t ticket = 0;
    topo_request r{};
    std::vector<double> rho;  // host copy when the caller passed a host pointer
    double t_submit = 0.0;
};

struct Job {
    int kind = TOPO_REQ_HDM;
    std::vector<Req> reqs;
    int mesh_id = 0, basis_id = -1, prec = 0, max_refine = 0, kb = 0;
    size_t ws_need = 0;       // library workspace the job needs
    size_t staging_need = 0;  // worker staging buffer the job needs
};

struct Worker {
    int index = 0;
    topo_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    void* staging = nullptr;
    size_t staging_bytes = 0;
    std::thread th;
    std::condition_variable cv;
    bool has_job = false;
    bool busy = false;
    Job job;
    size_t held = 0;  // workspace + staging currently allocated (or reserved)
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace topo

using namespace topo;

struct topo_server {
    int device = 0;
    size_t budget = 0;
    int max_batch = 1;
    int cu = 256;
    std::string err;
    std::vector<MeshRec> meshes;
    std::vector<BasisRec> bases;
    std::mutex m;
    std::condition_variable cv_sched, cv_done;
    std::deque<Req> queue;
    std::unordered_set<uint64_t> pending;
    std::unordered_map<uint64_t, topo_result> done;
    uint64_t next_ticket = 1;
    std::vector<std::unique_ptr<Worker>> workers;
    std::thread sched;
    bool stop = false, stop_workers = false;
    size_t max_held = 0;
    int64_t submitted = 0, completed = 0, failed = 0, jobs = 0, rom_jobs = 0, hdm_jobs = 0, rom_reqs = 0,
            hdm_reqs = 0;
    size_t resident = 0;  // device bytes of the registered meshes and bases
    std::vector<double> lat[2];
};

namespace {

int srv_error(topo_server* s, int code, const char* fmt, ...) {
    if (s) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        s->err = buf;
    }
    return code;
}

// Workspace and staging a job of B requests needs on a worker.
void size_job(topo_server* S, Job& j, int B) {
    const MeshRec& mr = S->meshes[j.mesh_id];
    const Grid& g = mr.g;
    const bool mixed = j.prec == TOPO_MIXED;
    if (j.kind == TOPO_REQ_HDM) {
        // a mixed solve may redo fields in float64 (its workspace then grows to that size)
        j.ws_need = mixed ? std::max(ws_hdm_solve(g, true, B), ws_hdm_solve(g, false, B)) : ws_hdm_solve(g, false, B);
        j.staging_need = align_up((size_t)B * g.n_elems * 8) + align_up((size_t)B * g.n_dofs * 8);
    } else {
        const int kb = j.kb;
        const bool basis64 = !S->bases[j.basis_id].fp32;
        j.ws_need = std::max({ws_rom_build(g, kb, B, basis64, S->cu), ws_rom_solve(kb, 1),
                              ws_rom_estimate(g, kb, 1, j.max_refine)});
        j.staging_need = align_up((size_t)B * g.n_elems * 8) + align_up((size_t)B * kb * kb * 8) +
                         align_up((size_t)kb * kb * 8) + align_up((size_t)kb * 8) +
                         align_up((size_t)kb * 8) + 3 * 256;
    }
}

// Bytes a worker holds after running job j (the arena only grows, by Arena::grown).
size_t held_after(const Worker& w, const Job& j) {
    const size_t ws = w.ctx->ws_bytes >= j.ws_need ? w.ctx->ws_bytes : Arena::grown(j.ws_need);
    const size_t st = std::max(w.staging_bytes, j.staging_need);
    return ws + st;
}

// Detach the device memory of an idle worker (under the server lock); the caller frees
// it after releasing the lock (free_detached), so submit / wait never block on hipFree.
// An idle worker's stream has drained: every job ends with a synchronisation of it.
void release_worker_memory(Worker& w, std::vector<void*>& detached) {
    if (w.ctx->ws) {
        detached.push_back(w.ctx->ws);
        w.ctx->ws = nullptr;
        w.ctx->ws_bytes = 0;
    }
    if (w.staging) {
        detached.push_back(w.staging);
        w.staging = nullptr;
        w.staging_bytes = 0;
    }
    w.held = 0;
}

void free_detached(int device, std::vector<void*>& detached) {
    if (detached.empty()) return;
    (void)hipSetDevice(device);
    for (void* p : detached) (void)hipFree(p);
    detached.clear();
}

// Form the next job from the head of the queue (requests are not removed).
Job form_job(topo_server* S, std::vector<size_t>& idx) {
    Job j;
    idx.clear();
    const Req& head = S->queue.front();
    j.kind = head.r.kind;
    j.mesh_id = head.r.mesh_id;
    j.prec = head.r.prec;
    idx.push_back(0);
    if (j.kind == TOPO_REQ_HDM) {
        // HDM requests on the same mesh with the same precision, tolerance and limit
        // form one batched solve (every field's result is the one it gets alone)
        for (size_t i = 1; i < S->queue.size() && (int)idx.size() < S->max_batch; ++i) {
            const topo_request& r = S->queue[i].r;
            if (r.kind == TOPO_REQ_HDM && r.mesh_id == j.mesh_id && r.prec == j.prec && r.rtol == head.r.rtol &&
                (r.maxit > 0 ? r.maxit : 0) == (head.r.maxit > 0 ? head.r.maxit : 0))
                idx.push_back(i);
        }
    } else if (j.kind == TOPO_REQ_ROM) {
        j.basis_id = head.r.basis_id;
        j.max_refine = head.r.max_refine;
        j.kb = head.r.k;
        for (size_t i = 1; i < S->queue.size() && (int)idx.size() < S->max_batch; ++i) {
            const topo_request& r = S->queue[i].r;
            if (r.kind == TOPO_REQ_ROM && r.mesh_id == j.mesh_id && r.basis_id == j.basis_id &&
                r.prec == j.prec && r.max_refine == j.max_refine) {
                idx.push_back(i);
                j.kb = std::max(j.kb, r.k);
            }
        }
    }
    return j;
}

void finish(topo_server* S, const Req& q, const topo_result& res) {
    S->done[q.ticket] = res;
    S->pending.erase(q.ticket);
    ++S->completed;
    if (res.status != TOPO_OK) ++S->failed;
    else S->lat[q.r.kind == TOPO_REQ_ROM ? 1 : 0].push_back(res.t_done - res.t_submit);
}

void dispatcher(topo_server* S) {
    std::unique_lock<std::mutex> lk(S->m);
    std::vector<size_t> idx;
    while (true) {
        if (S->queue.empty()) {
            if (S->stop) break;
            S->cv_sched.wait(lk);
            continue;
        }
        Worker* w = nullptr;
        for (auto& wp : S->workers)
            if (!wp->busy) {
                w = wp.get();
                break;
            }
        if (!w) {
            S->cv_sched.wait(lk);
            continue;
        }
        Job job = form_job(S, idx);
        size_job(S, job, (int)idx.size());
        auto total_with = [&](Worker* target) {
            size_t t = S->resident;  // registered meshes and bases
            for (auto& wp : S->workers) t += (wp.get() == target) ? held_after(*wp, job) : wp->held;
            return t;
        };
        size_t total = total_with(w);
        if (total > S->budget) {
            // give back memory held by idle workers and retry
            std::vector<void*> detached;
            for (auto& wp : S->workers)
                if (!wp->busy && wp.get() != w) release_worker_memory(*wp, detached);
            total = total_with(w);
            if (total > S->budget) {
                release_worker_memory(*w, detached);
                total = total_with(w);
            }
            if (!detached.empty()) {
                lk.unlock();
                free_detached(S->device, detached);
                lk.lock();
                // the queue may have changed meanwhile: form the job again
                continue;
            }
        }
        bool any_busy = false;
        for (auto& wp : S->workers) any_busy |= wp->busy;
        if (total > S->budget) {
            if (any_busy) {
                S->cv_sched.wait(lk);  // a completing job frees its memory
                continue;
            }
            // cannot fit even alone
            const double t = now_s();
            for (size_t n = idx.size(); n-- > 0;) {
                Req q = std::move(S->queue[idx[n]]);
                S->queue.erase(S->queue.begin() + idx[n]);
                topo_result res{};
                res.status = TOPO_ENOMEM;
                res.kind = q.r.kind;
                res.batch = (int)idx.size();
                res.worker = -1;
                res.t_submit = q.t_submit;
                res.t_start = res.t_done = t;
                finish(S, q, res);
            }
            S->cv_done.notify_all();
            continue;
        }
        // admit: move the requests into the job (keep queue order for the rest)
        for (size_t n = 0; n < idx.size(); ++n) job.reqs.push_back(std::move(S->queue[idx[n]]));
        for (size_t n = idx.size(); n-- > 0;) S->queue.erase(S->queue.begin() + idx[n]);
        w->held = held_after(*w, job);
        S->max_held = std::max(S->max_held, total);
        ++S->jobs;
        if (job.kind == TOPO_REQ_ROM) {
            ++S->rom_jobs;
            S->rom_reqs += (int64_t)job.reqs.size();
        } else {
            ++S->hdm_jobs;
            S->hdm_reqs += (int64_t)job.reqs.size();
        }
        w->job = std::move(job);
        w->busy = true;
        w->has_job = true;
        w->cv.notify_one();
    }
}

// Runs outside the server lock.  Fills one result per request.
void run_job(topo_server* S, Worker& w, Job& job, std::vector<topo_result>& out) {
    const MeshRec& mr = S->meshes[job.mesh_id];
    const Grid& g = mr.g;
    const hipStream_t s = w.stream;
    const double t_start = now_s();
    const int B = (int)job.reqs.size();
    out.assign(B, topo_result{});
    for (int b = 0; b < B; ++b) {
        out[b].kind = job.kind;
        out[b].batch = B;
        out[b].worker = w.index;
        out[b].t_submit = job.reqs[b].t_submit;
        out[b].t_start = t_start;
    }
    auto fail_all = [&](int code) {
        const double t = now_s();
        for (auto& r : out) {
            r.status = code;
            r.t_done = t;
        }
    };
    (void)hipSetDevice(S->device);
    if (job.staging_need > w.staging_bytes) {
        if (w.staging) (void)hipFree(w.staging);
        w.staging = nullptr;
        w.staging_bytes = 0;
        if (hipMalloc(&w.staging, job.staging_need) != hipSuccess) {
            (void)hipGetLastError();
            return fail_all(TOPO_ENOMEM);
        }
        w.staging_bytes = job.staging_need;
    }
    // carve the staging buffer; every piece is checked against its size before any
    // device work, so a sizing mistake fails the job instead of writing out of bounds
    char* p = (char*)w.staging;
    char* const end = p + w.staging_bytes;
    bool overflow = false;
    auto carve = [&](size_t bytes) -> void* {
        if ((size_t)(end - p) < align_up(bytes)) {
            overflow = true;
            return nullptr;
        }
        void* q = p;
        p += align_up(bytes);
        return q;
    };
    const int kb = job.kb;
    double* rho_d = (double*)carve((size_t)B * g.n_elems * 8);
    double *u_d = nullptr, *khat = nullptr, *kblk = nullptr, *fhat = nullptr, *yhat = nullptr,
           *jk = nullptr, *rn = nullptr;
    if (job.kind == TOPO_REQ_HDM) {
        u_d = (double*)carve((size_t)B * g.n_dofs * 8);
    } else {
        khat = (double*)carve((size_t)B * kb * kb * 8);
        kblk = (double*)carve((size_t)kb * kb * 8);
        fhat = (double*)carve((size_t)kb * 8);
        yhat = (double*)carve((size_t)kb * 8);
        jk = (double*)carve(8);
        rn = (double*)carve(8);
    }
    if (overflow) {
        w.ctx->err = "internal: job staging larger than its reservation";
        return fail_all(TOPO_ENOMEM);
    }
    // densities: host copies or device pointers
    for (int b = 0; b < B; ++b) {
        const Req& q = job.reqs[b];
        const void* src = q.r.rho_on_device ? (const void*)q.r.rho : (const void*)q.rho.data();
        const hipMemcpyKind kind = q.r.rho_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        const hipError_t e = hipMemcpyAsync(rho_d + (size_t)b * g.n_elems, src, (size_t)g.n_elems * 8, kind, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            w.ctx->err = std::string("density upload: ") + hipGetErrorString(e);
            return fail_all(TOPO_EDEVICE);
        }
    }
    if (job.kind == TOPO_REQ_HDM) {
        const Req& q = job.reqs[0];
        std::vector<topo_info> info(B);
        const int maxit = q.r.maxit > 0 ? q.r.maxit : 1000000;
        const int rc = topo_hdm_solve_batch(w.ctx, &mr.mesh, rho_d, mr.mask, mr.f, u_d, B, q.r.rtol, maxit,
                                            q.r.prec, nullptr, info.data(), s);
        const double t = now_s();
        for (int b = 0; b < B; ++b) {
            // device errors fail the whole job; convergence outcomes are per field
            out[b].status = (rc == TOPO_OK || rc == TOPO_ENOCONV || rc == TOPO_ENOTSPD) ? info[b].status : rc;
            out[b].iters = info[b].iters;
            out[b].J = info[b].compliance_corr;
            out[b].resnorm = info[b].rel_resid;
            out[b].t_done = t;
        }
        return;
    }
    const BasisRec& br = S->bases[job.basis_id];
    int rc = topo_rom_build(w.ctx, &mr.mesh, br.phi, br.fp32, kb, br.kmax, mr.mask, mr.f, rho_d, B,
                            khat, fhat, job.prec, s);
    if (rc) return fail_all(rc);
    for (int b = 0; b < B; ++b) {
        const int k = job.reqs[b].r.k;
        const double* Kb = khat + (size_t)b * kb * kb;
        if (k != kb) {
            // leading k x k block of the batch operator
            const hipError_t e = hipMemcpy2DAsync(kblk, (size_t)k * 8, Kb, (size_t)kb * 8, (size_t)k * 8, k,
                                                  hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                w.ctx->err = std::string("leading block copy: ") + hipGetErrorString(e);
                out[b].status = TOPO_EDEVICE;
                out[b].t_done = now_s();
                continue;
            }
            Kb = kblk;
        }
        rc = topo_rom_solve(w.ctx, k, 1, Kb, fhat, yhat, jk, nullptr, s);
        if (rc == TOPO_OK)
            rc = topo_rom_estimate(w.ctx, &mr.mesh, br.phi, br.fp32, k, br.kmax, mr.mask, mr.f,
                                   rho_d + (size_t)b * g.n_elems, 1, Kb, yhat, jk, rn,
                                   job.max_refine, nullptr, s);
        double h[2] = {0.0, 0.0};
        if (rc == TOPO_OK) {
            hipError_t e = hipMemcpyAsync(&h[0], jk, 8, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipMemcpyAsync(&h[1], rn, 8, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                w.ctx->err = std::string("result read-back: ") + hipGetErrorString(e);
                rc = TOPO_EDEVICE;
            }
        }
        out[b].status = rc;
        out[b].J = h[0];
        out[b].resnorm = h[1];
        out[b].t_done = now_s();
    }
}

void worker_main(topo_server* S, Worker* w) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->m);
    std::vector<topo_result> res;
    while (true) {
        w->cv.wait(lk, [&] { return w->has_job || S->stop_workers; });
        if (!w->has_job) break;
        Job job = std::move(w->job);
        w->has_job = false;
        lk.unlock();
        run_job(S, *w, job, res);
        lk.lock();
        for (size_t b = 0; b < job.reqs.size(); ++b) {
            finish(S, job.reqs[b], res[b]);
            if (res[b].status != TOPO_OK)
                S->err = "worker " + std::to_string(w->index) + ": " + w->ctx->err;
        }
        w->held = w->ctx->ws_bytes + w->staging_bytes;
        S->max_held = std::max(S->max_held, [&] {
            size_t t = S->resident;
            for (auto& wp : S->workers) t += wp->held;
            return t;
        }());
        w->busy = false;
        S->cv_done.notify_all();
        S->cv_sched.notify_all();
    }
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const size_t i = std::min(v.size() - 1, (size_t)(q * (double)v.size()));
    return v[i];
}

}  // namespace

extern "C" {

int topo_server_create(topo_server** out, int32_t device, size_t hbm_budget_bytes, int32_t max_batch,
                       int32_t n_workers) {
    if (!out) return TOPO_EINVAL;
    *out = nullptr;
    if (max_batch < 1 || n_workers < 1 || n_workers > 16 || hbm_budget_bytes == 0) return TOPO_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return TOPO_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return TOPO_EDEVICE;
    auto* S = new topo_server();
    S->device = device;
    S->budget = hbm_budget_bytes;
    S->max_batch = max_batch;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) S->cu = prop.multiProcessorCount;
    for (int i = 0; i < n_workers; ++i) {
        auto w = std::make_unique<Worker>();
        w->index = i;
        // the server's admission keeps the workers within its own budget
        if (topo_ctx_create(&w->ctx, device, 0) != TOPO_OK ||
            hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess) {
            for (auto& x : S->workers) {
                topo_ctx_destroy(x->ctx);
                (void)hipStreamDestroy(x->stream);
            }
            if (w->ctx) topo_ctx_destroy(w->ctx);
            delete S;
            return TOPO_EDEVICE;
        }
        S->workers.push_back(std::move(w));
    }
    for (auto& w : S->workers) w->th = std::thread(worker_main, S, w.get());
    S->sched = std::thread(dispatcher, S);
    *out = S;
    return TOPO_OK;
}

int topo_server_destroy(topo_server* S) {
    if (!S) return TOPO_OK;
    {
        std::lock_guard<std::mutex> lk(S->m);
        S->stop = true;
    }
    S->cv_sched.notify_all();
    S->sched.join();  // returns once every queued request has been dispatched
    {
        std::unique_lock<std::mutex> lk(S->m);
        S->cv_done.wait(lk, [&] {
            for (auto& w : S->workers)
                if (w->busy || w->has_job) return false;
            return true;
        });
        S->stop_workers = true;
    }
    for (auto& w : S->workers) w->cv.notify_all();
    for (auto& w : S->workers) w->th.join();
    (void)hipSetDevice(S->device);
    for (auto& w : S->workers) {
        (void)hipStreamSynchronize(w->stream);
        if (w->staging) (void)hipFree(w->staging);
        topo_ctx_destroy(w->ctx);
        (void)hipStreamDestroy(w->stream);
    }
    for (auto& m : S->meshes) {
        (void)hipFree(m.mask);
        (void)hipFree(m.f);
    }
    for (auto& b : S->bases) (void)hipFree(b.phi);
    delete S;
    return TOPO_OK;
}

const char* topo_server_last_error(const topo_server* S) { return S ? S->err.c_str() : "no server"; }

int topo_server_register_mesh(topo_server* S, const topo_mesh* mesh, const uint8_t* mask,
                              const double* f, int32_t* mesh_id) {
    if (!S || !mesh_id || !mask || !f) return TOPO_EINVAL;
    int rc = validate_mesh(nullptr, mesh);
    if (rc) return srv_error(S, rc, "invalid mesh");
    MeshRec r;
    r.mesh = *mesh;
    r.g = make_grid(*mesh);
    const size_t N = (size_t)r.g.n_dofs;
    const size_t bytes = align_up(N) + align_up(N * 8);
    {
        std::lock_guard<std::mutex> lk(S->m);
        if (S->resident + bytes > S->budget)
            return srv_error(S, TOPO_ENOMEM, "mesh of %zu bytes exceeds the HBM budget (%zu resident of %zu)",
                             bytes, S->resident, S->budget);
        S->resident += bytes;  // reserved; given back if the upload fails
    }
    (void)hipSetDevice(S->device);
    if (hipMalloc(&r.mask, N) != hipSuccess || hipMalloc(&r.f, N * 8) != hipSuccess ||
        hipMemcpy(r.mask, mask, N, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(r.f, f, N * 8, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        if (r.mask) (void)hipFree(r.mask);
        if (r.f) (void)hipFree(r.f);
        std::lock_guard<std::mutex> lk(S->m);
        S->resident -= bytes;
        return srv_error(S, TOPO_ENOMEM, "mesh registration failed");
    }
    std::lock_guard<std::mutex> lk(S->m);
    S->meshes.push_back(r);
    *mesh_id = (int32_t)S->meshes.size() - 1;
    return TOPO_OK;
}

int topo_server_register_basis(topo_server* S, int32_t mesh_id, const void* phi, int32_t phi_fp32,
                               int32_t kmax, int32_t ldphi, int32_t* basis_id) {
    if (!S || !phi || !basis_id) return TOPO_EINVAL;
    Grid g;
    {
        std::lock_guard<std::mutex> lk(S->m);
        if (mesh_id < 0 || mesh_id >= (int)S->meshes.size()) return srv_error(S, TOPO_EINVAL, "bad mesh id");
        g = S->meshes[mesh_id].g;
    }
    if (kmax < 1 || ldphi < kmax || (long long)kmax > g.n_dofs) return srv_error(S, TOPO_EINVAL, "bad kmax / ldphi");
    BasisRec b;
    b.mesh_id = mesh_id;
    b.fp32 = phi_fp32 ? 1 : 0;
    b.kmax = kmax;
    const size_t es = b.fp32 ? 4 : 8;
    const size_t bytes = align_up((size_t)g.n_dofs * kmax * es);
    {
        std::lock_guard<std::mutex> lk(S->m);
        if (S->resident + bytes > S->budget)
            return srv_error(S, TOPO_ENOMEM, "basis of %zu bytes exceeds the HBM budget (%zu resident of %zu)",
                             bytes, S->resident, S->budget);
        S->resident += bytes;
    }
    (void)hipSetDevice(S->device);
    if (hipMalloc(&b.phi, (size_t)g.n_dofs * kmax * es) != hipSuccess ||
        hipMemcpy2D(b.phi, kmax * es, phi, (size_t)ldphi * es, kmax * es, (size_t)g.n_dofs,
                    hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        if (b.phi) (void)hipFree(b.phi);
        std::lock_guard<std::mutex> lk(S->m);
        S->resident -= bytes;
        return srv_error(S, TOPO_ENOMEM, "basis registration failed");
    }
    std::lock_guard<std::mutex> lk(S->m);
    S->bases.push_back(b);
    *basis_id = (int32_t)S->bases.size() - 1;
    return TOPO_OK;
}

int topo_server_submit(topo_server* S, const topo_request* req, uint64_t* ticket) {
    if (!S || !req || !ticket || !req->rho) return TOPO_EINVAL;
    Req q;
    q.r = *req;
    int n_elems = 0;
    {
        std::lock_guard<std::mutex> lk(S->m);
        if (req->mesh_id < 0 || req->mesh_id >= (int)S->meshes.size())
            return srv_error(S, TOPO_EINVAL, "bad mesh id");
        n_elems = S->meshes[req->mesh_id].g.n_elems;
        if (req->kind == TOPO_REQ_ROM) {
            if (req->basis_id < 0 || req->basis_id >= (int)S->bases.size())
                return srv_error(S, TOPO_EINVAL, "bad basis id");
            const BasisRec& b = S->bases[req->basis_id];
            if (b.mesh_id != req->mesh_id) return srv_error(S, TOPO_EINVAL, "basis belongs to another mesh");
            if (req->k < 1 || req->k > b.kmax) return srv_error(S, TOPO_EINVAL, "k out of range");
            if (req->max_refine < 0) return srv_error(S, TOPO_EINVAL, "max_refine < 0");
        } else if (req->kind == TOPO_REQ_HDM) {
            if (!(req->rtol > 0.0 && req->rtol < 1.0)) return srv_error(S, TOPO_EINVAL, "rtol must lie in (0,1)");
        } else {
            return srv_error(S, TOPO_EINVAL, "unknown request kind");
        }
        if (req->prec != TOPO_FP64 && req->prec != TOPO_MIXED) return srv_error(S, TOPO_EINVAL, "bad precision");
    }
    if (!req->rho_on_device) q.rho.assign(req->rho, req->rho + n_elems);
    q.t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->m);
        q.ticket = S->next_ticket++;
        *ticket = q.ticket;
        S->pending.insert(q.ticket);
        ++S->submitted;
        S->queue.push_back(std::move(q));
    }
    S->cv_sched.notify_all();
    return TOPO_OK;
}

int topo_server_wait(topo_server* S, uint64_t ticket, topo_result* res) {
    if (!S || !res) return TOPO_EINVAL;
    std::unique_lock<std::mutex> lk(S->m);
    if (!S->pending.count(ticket) && !S->done.count(ticket)) return srv_error(S, TOPO_EINVAL, "unknown ticket");
    S->cv_done.wait(lk, [&] { return S->done.count(ticket) > 0; });
    *res = S->done[ticket];
    S->done.erase(ticket);
    return res->status;
}

int topo_server_poll(topo_server* S, uint64_t ticket, topo_result* res) {
    if (!S || !res) return TOPO_EINVAL;
    std::lock_guard<std::mutex> lk(S->m);
    auto it = S->done.find(ticket);
    if (it == S->done.end()) return S->pending.count(ticket) ? TOPO_EAGAIN : srv_error(S, TOPO_EINVAL, "unknown ticket");
    *res = it->second;
    S->done.erase(it);
    return res->status;
}

int topo_server_stats(topo_server* S, topo_serve_stats* st) {
    if (!S || !st) return TOPO_EINVAL;
    std::lock_guard<std::mutex> lk(S->m);
    *st = topo_serve_stats{};
    st->submitted = S->submitted;
    st->completed = S->completed;
    st->failed = S->failed;
    st->jobs = S->jobs;
    st->rom_jobs = S->rom_jobs;
    st->hdm_jobs = S->hdm_jobs;
    st->mean_rom_batch = S->rom_jobs ? (double)S->rom_reqs / (double)S->rom_jobs : 0.0;
    st->mean_hdm_batch = S->hdm_jobs ? (double)S->hdm_reqs / (double)S->hdm_jobs : 0.0;
    st->resident_bytes = S->resident;
    st->budget_bytes = S->budget;
    size_t held = S->resident;
    for (auto& w : S->workers) held += w->held;
    st->held_bytes = held;
    st->max_held_bytes = S->max_held;
    for (int k = 0; k < 2; ++k) {
        st->p50_latency_s[k] = percentile(S->lat[k], 0.50);
        st->p99_latency_s[k] = percentile(S->lat[k], 0.99);
    }
    st->workers = (int32_t)S->workers.size();
    return TOPO_OK;
}

}  // extern "C"
