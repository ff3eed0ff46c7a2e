/*
 * topo_serve.h -- continuous-batching request server over the topo_rom.h hot path.
 *
 * A trust-region optimiser built on the method issues many ROM evaluations (model
 * values and error indicators of candidate designs; Sec. 4.3 and the numerical
 * experiments of Sec. 5, which need O(10^2 - 10^3) ROM evaluations per subproblem)
 * and a few full-order solves (one per major iteration).  The server accepts such
 * requests from any host thread while others are running:
 *
 *  - meshes (mask, load) and reduced bases are registered once and stay resident in
 *    device memory (library-owned copies);
 *  - each request carries its own density field (copied at submission);
 *  - a dispatcher thread forms jobs: HDM requests on the same (mesh, precision,
 *    tolerance, iteration limit) are fused into one batched solve (topo_hdm_solve_batch:
 *    every field's result is bitwise the one it gets alone); ROM requests on the
 *    same (mesh, basis, precision, refinement count) are fused into one batched
 *    reduced-operator build at the largest k of the batch, each request then using
 *    the leading k x k block (basis columns are prefixes, so K_hat_k is that block);
 *  - jobs run on a pool of worker threads, each with its own HIP stream and library
 *    context, so independent jobs overlap on the GPU;
 *  - the HBM budget given at creation covers the resident meshes and bases and the
 *    workers' device workspace: a registration that would take the resident set past
 *    it fails with TOPO_ENOMEM, and a job is admitted only when the workspace it needs,
 *    added to the resident set and to what the workers already hold, stays within it;
 *    a job that can never fit fails with TOPO_ENOMEM;
 *  - requests that arrive while jobs run are admitted as workers and memory free up.
 *
 * A request's result does not depend on the batch it ran in beyond floating-point
 * summation order of the shared build (same tolerance as the standalone call).
 */
#ifndef TOPO_SERVE_H
#define TOPO_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "topo_rom.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct topo_server topo_server;

#define TOPO_REQ_HDM 0  /* full-order solve: compliance (J) and true residual     */
#define TOPO_REQ_ROM 1  /* ROM evaluation: build + reduced solve + error indicator */

/* One request.  Host struct; rho is copied during topo_server_submit when it is a
 * host pointer; a device pointer (rho_on_device != 0) must stay valid until the
 * request completes. */
typedef struct topo_request {
    int32_t kind;          /* TOPO_REQ_HDM or TOPO_REQ_ROM                          */
    int32_t mesh_id;       /* from topo_server_register_mesh                        */
    int32_t basis_id;      /* ROM: from topo_server_register_basis                  */
    int32_t k;             /* ROM: leading basis columns used, 1 <= k <= kmax       */
    int32_t prec;          /* TOPO_FP64 or TOPO_MIXED                               */
    int32_t max_refine;    /* ROM: reduced refinement steps (topo_rom_estimate)     */
    int32_t maxit;         /* HDM: iteration limit (<= 0: library default)          */
    int32_t rho_on_device; /* 0: rho is a host pointer; 1: device pointer           */
    double rtol;           /* HDM: relative true-residual tolerance                  */
    const double* rho;     /* [n_elems] element densities                           */
} topo_request;

/* Outcome of one request.  Host struct.  Times are seconds of a steady clock. */
typedef struct topo_result {
    int32_t status;   /* TOPO_OK or a TOPO_E* code                                   */
    int32_t kind;
    int32_t iters;    /* HDM: inner PCG iterations                                   */
    int32_t batch;    /* number of requests in the job that served this one         */
    int32_t worker;   /* worker (stream) index                                       */
    int32_t pad;
    double J;         /* HDM: compliance (residual-corrected); ROM: J_k              */
    double resnorm;   /* HDM: final relative residual; ROM: ||f - K Phi y||          */
    double t_submit;  /* submission                                                  */
    double t_start;   /* job start on its worker                                     */
    double t_done;    /* results read back                                           */
} topo_result;

typedef struct topo_serve_stats {
    int64_t submitted, completed, failed;
    int64_t jobs, rom_jobs, hdm_jobs;
    double mean_rom_batch;      /* ROM requests per ROM job                          */
    double mean_hdm_batch;      /* HDM requests per HDM job                          */
    size_t budget_bytes;
    size_t resident_bytes;      /* registered meshes and bases                       */
    size_t held_bytes;          /* resident set + workspace held by the workers      */
    size_t max_held_bytes;      /* maximum over the server's life (<= budget)       */
    double p50_latency_s[2];    /* [HDM, ROM]: t_done - t_submit over completed     */
    double p99_latency_s[2];
    int32_t workers;
    int32_t pad;
} topo_serve_stats;

/* Create a server on `device` with `n_workers` worker streams (1..16), at most
 * `max_batch` requests per fused job (>= 1), and an HBM budget of `hbm_budget_bytes`
 * for the registered meshes and bases and the workers' device workspace. */
int topo_server_create(topo_server** out, int32_t device, size_t hbm_budget_bytes,
                       int32_t max_batch, int32_t n_workers);
/* Completes every queued request, stops the threads, frees all device memory. */
int topo_server_destroy(topo_server* srv);

/* Register a mesh with its Dirichlet mask (uint8 [N_u]) and load (f64 [N_u]), both
 * HOST arrays copied to the device.  *mesh_id receives the handle.  TOPO_ENOMEM when
 * its 9 N_u bytes would take the resident set past the budget. */
int topo_server_register_mesh(topo_server* srv, const topo_mesh* mesh, const uint8_t* mask,
                              const double* f, int32_t* mesh_id);
/* Register a basis for a registered mesh: HOST array Phi [N_u][ldphi] (float32 when
 * phi_fp32 != 0), columns 0..kmax-1 copied to the device.  TOPO_ENOMEM when its
 * N_u kmax (4 or 8) bytes would take the resident set past the budget. */
int topo_server_register_basis(topo_server* srv, int32_t mesh_id, const void* phi,
                               int32_t phi_fp32, int32_t kmax, int32_t ldphi,
                               int32_t* basis_id);

/* Queue a request (thread-safe, non-blocking).  *ticket identifies it.  Invalid
 * requests return TOPO_EINVAL immediately. */
int topo_server_submit(topo_server* srv, const topo_request* req, uint64_t* ticket);
/* Block until the request is done; fills *res (host) and forgets the ticket.
 * Returns the request's status (also in res->status), or TOPO_EINVAL for an
 * unknown ticket. */
int topo_server_wait(topo_server* srv, uint64_t ticket, topo_result* res);
/* Non-blocking: TOPO_EAGAIN while the request is pending, else as topo_server_wait. */
int topo_server_poll(topo_server* srv, uint64_t ticket, topo_result* res);
/* Counters and latency percentiles over all completed requests (host struct). */
int topo_server_stats(topo_server* srv, topo_serve_stats* stats);
/* Message of the last server-level error. */
const char* topo_server_last_error(const topo_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* TOPO_SERVE_H */
