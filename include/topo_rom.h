/*
 * topo_rom.h -- C ABI of the MI355X (gfx950) hot path of ROM-accelerated SIMP
 * minimum-compliance topology optimisation.
 *
 * Method: Yano, Huang & Zahr, "A globally convergent method to accelerate topology
 * optimization using on-the-fly model reduction".  The full-order model (HDM) is the
 * SIMP linear-elastic state equation K(rho) u = f on a structured grid of bilinear
 * (2D, Q4) or trilinear (3D, H8) elements (Sec. 2.1), its compliance f^T u (Sec. 2.3)
 * and the element sensitivity dc/drho_e = -alpha'(rho_e) u_e^T K_e u_e (Sec. 2.4 and
 * the adjoint appendix; compliance is self-adjoint).  The reduced-order model (ROM)
 * is the Galerkin projection K_hat = Phi^T K(rho) Phi, f_hat = Phi^T f, the reduced
 * solve K_hat y = f_hat and the residual norm ||f - K(rho) Phi y|| used as the error
 * indicator and trust-region constraint (Sec. 3.1, 3.3, 3.4 and Sec. 4.3).
 *
 * General conventions
 * -------------------
 *  - Every array argument is a DEVICE pointer owned by the caller (e.g. memory of a
 *    torch tensor), unless the comment says "host".  The library never frees or keeps
 *    caller pointers beyond the call.  Outputs are written only when TOPO_OK is
 *    returned (device outputs of a failed call are unspecified).
 *  - Structured grid: nel = (nx, ny[, nz]) elements of edge lengths h; node (i,j[,k])
 *    has index i + (nx+1)*(j + (ny+1)*k); element (ex,ey[,ez]) has index
 *    ex + nx*(ey + ny*ez).
 *  - DOF vectors are structure-of-arrays: component c of node n is entry
 *    c*n_nodes + n; N_u = dim * n_nodes.
 *  - mask: uint8 [N_u]; 1 marks a homogeneous Dirichlet DOF.  Those DOFs are
 *    eliminated (Sec. 2.1): entries of f and rows of Phi there are ignored (taken as
 *    zero), u = 0 and r = 0 there, and every norm / dot product runs over free DOFs.
 *  - Material law (Sec. 2.1): alpha(rho) = Emin + (E0 - Emin) rho^penal; the paper's
 *    law is the case E0 = 1, Emin = rho_l.
 *  - Basis Phi: row-major [N_u][ldphi] (k <= ldphi <= 1024), rows indexed like DOF
 *    vectors; the first k columns are used.  float32 when phi_fp32 != 0, float64
 *    otherwise.  Phi must have full column rank on the free DOFs (orthonormality is
 *    not required).
 *  - stream: a hipStream_t (NULL = the null stream).  Work is stream-ordered.  Calls
 *    that report a convergence or pivot outcome to the host (hdm_solve, rom_solve
 *    with status == NULL) synchronise that stream and return it synchronously; the
 *    others (rom_build, rom_estimate, hdm_gradient, ...) only enqueue work.
 *  - Threading: a context is used by one host thread at a time; distinct contexts
 *    may run concurrently on distinct streams.  The calls of one context share its
 *    device workspace, so when they go to different streams the caller orders them
 *    (for example by synchronising the first stream before the next call).
 *  - Errors: a negative TOPO_E* code; topo_last_error(ctx) gives a message.
 */
#ifndef TOPO_ROM_H
#define TOPO_ROM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TOPO_OK 0
#define TOPO_EINVAL (-1)   /* invalid argument (checked before any device work) */
#define TOPO_ENOMEM (-2)   /* device workspace allocation failed / over budget     */
#define TOPO_ENOCONV (-3)  /* iteration limit reached or stagnation                */
#define TOPO_ENOTSPD (-4)  /* non-positive pivot / CG breakdown: not SPD            */
#define TOPO_EDEVICE (-5)  /* HIP runtime error                                     */
#define TOPO_EAGAIN (-6)   /* serving: request cannot be admitted now               */

/* Precision of the hot loops. */
#define TOPO_FP64 0   /* everything in float64                                      */
#define TOPO_MIXED 1  /* float32 inner PCG (float64 correction and residual        */
                      /* replacement), float64 dots, norms, compliance, K_hat and     */
                      /* reduced Cholesky; float32 basis with float64 refinement      */

typedef struct topo_ctx topo_ctx;

/* Structured-grid problem description (Sec. 2.1).  Passed by host pointer. */
typedef struct topo_mesh {
    int32_t dim;      /* 2 (Q4) or 3 (H8)                                          */
    int32_t nel[3];   /* elements per axis; nel[2] ignored when dim == 2            */
    double h[3];      /* element edge lengths (> 0); h[2] ignored when dim == 2     */
    double E0;        /* solid stiffness (> Emin)                                   */
    double Emin;      /* void stiffness (>= 0)                                      */
    double nu;        /* Poisson ratio, -1 < nu < 0.5                               */
    double penal;     /* SIMP exponent p >= 1                                       */
    int32_t plane;    /* 2D only: 0 = plane stress, 1 = plane strain; unit thickness */
} topo_mesh;

/* Diagnostics of an HDM solve.  Host struct. */
typedef struct topo_info {
    int32_t iters;          /* inner PCG iterations summed over refinement steps      */
    int32_t refinements;    /* outer float64 residual / correction steps              */
    double rel_resid;       /* final true ||f - K u||_2 / ||f||_2 over free DOFs      */
    double compliance_raw;  /* f^T u                                                   */
    double compliance_corr; /* f^T u + u^T r = c* - ||u - u*||_K^2 (second order)    */
    int32_t fp64_fallback;  /* TOPO_MIXED only: 1 when a float32 correction failed to  */
                            /* reduce the true residual and the solve was redone in   */
                            /* float64 from u = 0 (iters counts both attempts)        */
    int32_t status;         /* outcome of this field: TOPO_OK, TOPO_ENOCONV or         */
                            /* TOPO_ENOTSPD (for batched solves, per field)            */
} topo_info;

/* ---- context ------------------------------------------------------------------ */

/* Create a context on HIP device `device`: element tables, device workspace.
 * hbm_budget_bytes bounds the device workspace the context may hold (0: no bound); a
 * call whose workspace would exceed it fails with TOPO_ENOMEM before any device work.
 * Ownership of *out passes to the caller; release with topo_ctx_destroy. */
int topo_ctx_create(topo_ctx** out, int32_t device, size_t hbm_budget_bytes);
int topo_ctx_destroy(topo_ctx* ctx);
/* Message of the last error raised on ctx (valid until the next call on ctx). */
const char* topo_last_error(const topo_ctx* ctx);
/* Static name of an error code. */
const char* topo_strerror(int32_t code);
/* Bytes of device workspace currently held by ctx (host scalar). */
size_t topo_ctx_workspace_bytes(const topo_ctx* ctx);

/* Instrumentation: bracket one run of 8 consecutive launches in `every` runs (0 = off)
 * of each hot kernel of ctx with HIP events on the stream it runs on (runs of 8: the
 * 3D PCG update's correction group). */
int topo_ctx_set_timing(topo_ctx* ctx, int32_t every);
/* Sampled launches and their summed device time in ms for one hot kernel: "apply",
 * "pcg_apply", "pcg_update", "residual", "rom_contract", "rom_reduce", "phit_v",
 * "phi_y", "chol", "chol_solve", "gradient", "pcg_step" (the one kernel per
 * iteration of the 2D float64 solve; "pcg_apply" / "pcg_update" are the two of the
 * other solves), "rom_apply" (the ROM build's transposed basis and K Phi products, per
 * field; "rom_contract" is then its matrix-core product, per field), and the number of
 * launches of that kernel issued since the last
 * reset while timing was on (graph replays included; may be NULL).  A launch of a
 * batched kernel covers every field of its batch.  Waits for pending samples (host
 * outputs); reset != 0 clears the kernel's counters afterwards. */
int topo_ctx_kernel_time(topo_ctx* ctx, const char* kernel, int64_t* samples,
                         double* total_ms, int64_t* launches, int32_t reset);

/* ---- element operator --------------------------------------------------------- */

/* Unit-density element stiffness K_e of the mesh's element (Sec. 2.1), exact for the
 * rectangular Q4 / H8 element.  Local DOF order: dim*a + c, tensor-order local node
 * a = ax + 2*ay (+ 4*az).  K0: HOST array of (dim*2^dim)^2 doubles, row-major. */
int topo_element_stiffness(const topo_mesh* mesh, double* K0);

/* Symmetry-blocked factor K_e = R^T R that the 3D apply and residual evaluate (in its
 * reduced-block form) (R: 5 rows for Q4, 18 for H8).  In the Walsh-Hadamard basis
 * N[m][c] = -sum_a (-1)^{popcount(m & a)} x[a][c] of an element vector x, K_e splits
 * into one block per reflection character n (entries (n ^ 2^c, c), c < dim).  Blocks
 * with one set bit drop their rigid translation entry; blocks with two set bits c < d
 * combine h[c] N[n^2^c][c] + h[d] N[n^2^d][d] (which annihilates the rotation in that
 * plane) followed by the remaining entry; blocks 0 and 7 keep all three entries.  F:
 * HOST array of 51 doubles: per block n (0 .. 2^dim - 1) six slots holding the upper-
 * triangular transposed Cholesky factor of the reduced block (L00 L01 L02 L11 L12 L22,
 * unused slots zero), then h[0..2] at 48..50.  TOPO_EINVAL for a mesh whose element
 * operator does not have that structure (not produced by valid meshes). */
int topo_element_factor(const topo_mesh* mesh, double* F);

/* ---- full-order model ----------------------------------------------------------- */

/* Matrix-free operator apply y_b = K(rho_b) x_b for B fields (Sec. 2.1,
 * K = sum_e alpha(rho_e) P_e K_e P_e^T), Dirichlet DOFs eliminated: y_f = K_ff x_f,
 * y = 0 on constrained DOFs, x ignored there.
 *   rho: [B][n_elems] float64;  x, y: [B][N_u], float64 when prec == TOPO_FP64,
 *   float32 when prec == TOPO_MIXED (the inner-loop apply). */
int topo_apply(topo_ctx* ctx, const topo_mesh* mesh, const double* rho,
               const uint8_t* mask, const void* x, void* y, int32_t B, int32_t prec,
               void* stream);

/* HDM state solve K_ff(rho) u_f = f_f (Sec. 2.1) by Jacobi-preconditioned CG on the
 * matrix-free operator, from u = 0, until the TRUE residual satisfies
 * ||f - K u||_2 <= rtol ||f||_2 (recomputed in float64).  TOPO_MIXED runs float32
 * inner CG solves on the float64 residual (iterative refinement).  Then compliance
 * f^T u (Sec. 2.3).
 *   rho [n_elems] f64, mask [N_u] u8, f [N_u] f64, u [N_u] f64 (output).
 *   compliance: HOST double, receives compliance_corr (may be NULL).
 *   info: HOST, may be NULL.  maxit bounds the total inner iterations.
 * Returns TOPO_ENOCONV when maxit is reached or refinement stagnates (u and info
 * then hold the last iterate), TOPO_ENOTSPD on a CG breakdown. */
int topo_hdm_solve(topo_ctx* ctx, const topo_mesh* mesh, const double* rho,
                   const uint8_t* mask, const double* f, double* u, double rtol,
                   int32_t maxit, int32_t prec, double* compliance, topo_info* info,
                   void* stream);

/* Batched HDM state solve: B density fields sharing the mesh, the Dirichlet mask and
 * the load (Sec. 2.1 state equation for each field; the method's trust-region
 * iterates and the benchmark's field batches), solved together with B fields per
 * kernel launch.  Same method, stopping rule and outputs per field as topo_hdm_solve;
 * every stopping, restart and residual-replacement decision is taken per field and
 * every reduction runs over the field's own data in a fixed order, so a field's u,
 * compliance and info are bitwise the same whatever batch it is solved in.
 *   rho [B][n_elems] f64, mask [N_u] u8, f [N_u] f64 (shared), u [B][N_u] f64 out.
 *   compliance: HOST [B] (may be NULL), receives each compliance_corr.
 *   info: HOST [B] (may be NULL); info[b].status is the field's outcome.  maxit bounds
 *   each field's inner iterations.
 * Returns TOPO_OK when every field converged, else the status of the first field that
 * did not (u and info then hold every field's last iterate and diagnostics). */
int topo_hdm_solve_batch(topo_ctx* ctx, const topo_mesh* mesh, const double* rho,
                         const uint8_t* mask, const double* f, double* u, int32_t B,
                         double rtol, int32_t maxit, int32_t prec, double* compliance,
                         topo_info* info, void* stream);

/* Element sensitivity of the compliance with respect to the filtered density,
 * dc[e] = -penal (E0 - Emin) rho_e^(penal-1) u_e^T K_e u_e (Sec. 2.4, compliance
 * remark: lambda* = u*, no adjoint solve), float64.
 *   rho [n_elems] f64, u [N_u] f64 (zero on Dirichlet DOFs), dc [n_elems] f64 out. */
int topo_hdm_gradient(topo_ctx* ctx, const topo_mesh* mesh, const double* rho,
                      const double* u, double* dc, void* stream);
/* The same for B fields: rho [B][n_elems], u [B][N_u], dc [B][n_elems] (float64). */
int topo_hdm_gradient_batch(topo_ctx* ctx, const topo_mesh* mesh, const double* rho,
                            const double* u, int32_t B, double* dc, void* stream);

/* ---- reduced-order model --------------------------------------------------------- */

/* Reduced operators of B density fields sharing one basis (Sec. 3.1, element-sum
 * form of K_hat; Sec. 3.4 cost analysis):
 *   Khat[b] = sum_e alpha(rho_be) (P_e^T Phi)^T K_e (P_e^T Phi)   [B][k][k] f64 out,
 *   fhat    = Phi^T f                                             [k] f64 out (may
 *             be NULL; it depends on the basis only).
 * Evaluated per field as W = K(rho_b) Phi, the k basis columns (masked rows zero) taken
 * as the vectors of one batched matrix-free apply in float64, then K_hat = Phi^T W as
 * one product over the N_u rows, accumulated in float64 on the matrix cores with
 * per-chunk partials summed in a fixed order.  The arithmetic is float64 in both
 * precisions (prec is validated but selects nothing here; a float32 basis is read as
 * its float32 values).  A field's K_hat does not depend on B.
 *   rho: [B][n_elems] f64.  Errors: TOPO_EINVAL (sizes, k beyond 1024 after padding to
 *   16, null pointers), TOPO_ENOMEM (workspace beyond the context budget),
 *   TOPO_EDEVICE. */
int topo_rom_build(topo_ctx* ctx, const topo_mesh* mesh, const void* phi,
                   int32_t phi_fp32, int32_t k, int32_t ldphi, const uint8_t* mask,
                   const double* f, const double* rho, int32_t B, double* Khat,
                   double* fhat, int32_t prec, void* stream);

/* Reduced solve (Sec. 3.1 and 3.4): float64 Cholesky of each K_hat[b], yhat[b] =
 * K_hat[b]^{-1} fhat, Jk[b] = fhat^T yhat[b] (the ROM compliance).
 *   Khat [B][k][k] f64 (symmetric; lower triangle read), fhat [k] f64,
 *   yhat [B][k] f64 out, Jk [B] f64 out.
 *   status: [B] int32 DEVICE out (0 ok, TOPO_ENOTSPD when a pivot is not positive),
 *   or NULL: then the call synchronises and returns TOPO_ENOTSPD if any failed. */
int topo_rom_solve(topo_ctx* ctx, int32_t k, int32_t B, const double* Khat,
                   const double* fhat, double* yhat, double* Jk, int32_t* status,
                   void* stream);

/* Allocation-free variant of topo_rom_solve, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results as topo_rom_solve, except that
 * status [B] int32 DEVICE out is required (the call never synchronises).  The
 * Cholesky factors go to a fixed device array of the library instead of the context's
 * workspace: B * k * k * 8 bytes must not exceed topo_rom_solve_noalloc_max_bytes()
 * (8 MiB; e.g. k = 200 with B <= 26), else TOPO_EINVAL before any device work.  No
 * device or host memory is allocated and the context's workspace is not touched.  Each
 * GPU holds one copy of that array until the process ends, shared by every call on
 * that GPU: calls that overlap on one GPU (other streams, other contexts, other host
 * threads) race on it, so the caller orders them.  It keeps the last call's factors;
 * nothing in it needs clearing (the factorisation writes every entry the solve reads).
 * Errors: TOPO_EINVAL (k, B < 1, null pointer, over the size limit), TOPO_EDEVICE. */
int topo_rom_solve_noalloc(topo_ctx* ctx, int32_t k, int32_t B, const double* Khat,
                           const double* fhat, double* yhat, double* Jk, int32_t* status,
                           void* stream);
/* Size in bytes of the fixed device array topo_rom_solve_noalloc uses (host scalar). */
size_t topo_rom_solve_noalloc_max_bytes(void);

/* Residual-based error indicator (Sec. 3.3 primal residual; Sec. 3.4 cost
 * analysis; Sec. 4.3 residual trust-region constraint):
 *   u_b = Phi yhat[b] (float64 accumulation), r_b = f - K(rho_b) u_b on free DOFs in
 *   float64, resnorm[b] = ||r_b||_2.
 * With max_refine > 0 the reduced coefficients are refined in float64, up to
 * max_refine times: yhat += K_hat^{-1} Phi^T r (a step is kept only while the
 * Galerkin residual ||Phi^T r|| of that field decreases, and only when K_hat[b]
 * factors), recovering float64 accuracy of a float32 K_hat; then
 * Jk[b] = f^T Phi yhat[b] and resnorm are those of the refined yhat.  Every decision is
 * taken on the device: the call does not synchronise the stream.
 *   yhat [B][k] f64 in/out, Jk [B] f64 out (may be NULL), resnorm [B] f64 out,
 *   Khat [B][k][k] f64 (only read when max_refine > 0),
 *   dJ [B][N_e] f64 out (may be NULL): the ROM sensitivity at the returned yhat, as
 *   topo_rom_gradient computes it, fused into the estimate (without refinement it is
 *   evaluated on the same u = Phi yhat as the residual, so no extra pass over Phi). */
int topo_rom_estimate(topo_ctx* ctx, const topo_mesh* mesh, const void* phi,
                      int32_t phi_fp32, int32_t k, int32_t ldphi, const uint8_t* mask,
                      const double* f, const double* rho, int32_t B, const double* Khat,
                      double* yhat, double* Jk, double* resnorm, int32_t max_refine,
                      double* dJ, void* stream);

/* Sensitivity of the ROM compliance J_k(rho) = f_hat^T K_hat(rho)^{-1} f_hat with
 * respect to the densities (Sec. 3.2: for the compliance the reduced adjoint equals the
 * reduced state; the element form is the sensitivity of Sec. 2.4 at u_k = Phi y_hat):
 *   dJ[b][e] = -alpha'(rho[b][e]) u_k,e^T K_e u_k,e,   u_k = Phi yhat[b]  (float64).
 * Phi, k, ldphi, mask as in topo_rom_build; rho [B][N_e] f64; yhat [B][k] f64 (the
 * coefficients rom_solve / rom_estimate returned for those densities); dJ [B][N_e] f64
 * out.  Only enqueues work.  Errors: TOPO_EINVAL (null pointer, B < 1, bad basis
 * shape), TOPO_ENOMEM (workspace), TOPO_EDEVICE. */
int topo_rom_gradient(topo_ctx* ctx, const topo_mesh* mesh, const void* phi,
                      int32_t phi_fp32, int32_t k, int32_t ldphi, const uint8_t* mask,
                      const double* rho, int32_t B, const double* yhat, double* dJ,
                      void* stream);

/* ---- Helmholtz density filter (Sec. 2.2) and the gradient through it (Sec. 2.4) ---- */

/* Flag of topo_filter_forward / topo_filter_adjoint: the nodal array (phi or mu, then
 * not NULL) holds an initial guess on entry. */
#define TOPO_FILTER_WARM 1

/* Filtered densities rho = rho*(psi) for B fields (Sec. 2.2): the nodal Helmholtz
 * problem H phi = b(psi) with H = sum_e (r^2 L_e + M_e) (bilinear / trilinear Laplacian
 * and mass matrices of the mesh's box element, homogeneous Neumann boundary, no node
 * constrained) and b_n = (|Omega_e| / nen) sum of psi_e over the elements around node n,
 * then rho_e = the mean of phi over the element's nen nodes.  r is the Helmholtz length
 * (the paper's r = 2 sqrt(3) R for a filter radius R; r = 0 gives the L2 projection).
 *   psi [B][N_e] f64 device, rho [B][N_e] f64 device out, phi [B][N_n] f64 device out
 *   (may be NULL; nodal values, node = i + (nx+1)(j + (ny+1)k)).
 * Solved by Jacobi-PCG in float64 to |b - H phi| <= rtol |b| per field (maxit
 * iterations at most), from phi = 0, or from the phi passed in with flags ==
 * TOPO_FILTER_WARM (a field whose guess already meets the tolerance takes no
 * iteration); *iters (host, may be NULL) gets the largest iteration count.
 * Synchronises (convergence checks).  Errors: TOPO_EINVAL (mesh, null pointer, B < 1,
 * r < 0, rtol outside (0, 1), maxit < 1), TOPO_ENOCONV, TOPO_ENOMEM, TOPO_EDEVICE. */
int topo_filter_forward(topo_ctx* ctx, const topo_mesh* mesh, double r, const double* psi,
                        int32_t B, double* rho, double* phi, double rtol, int32_t maxit,
                        int32_t flags, int32_t* iters, void* stream);

/* Gradient through the filter (Sec. 2.4 and the adjoint derivation of the appendix):
 * g = (d rho* / d psi)^T v for B fields, i.e. H mu = q(v) with q_n = (1 / nen) sum of v_e
 * over the elements around node n, then g_e = (|Omega_e| / nen) sum of mu over the
 * element's nodes.  (The appendix prints a minus sign in front of this product; its own
 * definitions give the plus sign used here, which finite differences confirm.)  With v =
 * dJ/drho this is dJ/dpsi.  v, g [B][N_e] f64 device; mu [B][N_n] (may be NULL); the rest
 * as topo_filter_forward.  Synchronises.  Same errors. */
int topo_filter_adjoint(topo_ctx* ctx, const topo_mesh* mesh, double r, const double* v,
                        int32_t B, double* g, double* mu, double rtol, int32_t maxit,
                        int32_t flags, int32_t* iters, void* stream);

/* ---- Reduced basis at a trust-region centre (Sec. 4.2) --------------------------- */

/* Largest snapshot window L the basis routines accept. */
#define TOPO_POD_MAX_WINDOW 48

/* Limited-memory snapshot window (Sec. 4.2, remark on keeping only the L most recent
 * trust-region centres).  The caller owns the window state:
 *   S [L][n] f64 device: slot i holds a snapshot at S + i*n;
 *   G [L][L] f64 device: G[i][j] = S_i . S_j for the valid slots 0..*count-1;
 *   *count (host, in/out): number of valid slots, 0 for an empty window;
 *   *next  (host, in/out): the slot of the oldest snapshot once the window is full (0
 *          while it fills).
 * Pushes the snapshot u [n] f64 device: while *count < L it goes to slot *count and the
 * window grows (rank-one update of G); once full it replaces slot *next, the oldest
 * (rank-two update: one snapshot in, one out), and *next advances modulo L.  One
 * streaming pass over the window computes the new row and column of G (deterministic
 * float64 sums) and stores u.  Only enqueues work; *count and *next are updated on
 * return.  Errors: TOPO_EINVAL (null pointer, n < 1, L outside [1,
 * TOPO_POD_MAX_WINDOW], inconsistent count/next), TOPO_ENOMEM, TOPO_EDEVICE. */
int topo_pod_push(topo_ctx* ctx, int64_t n, int32_t L, double* S, double* G, int32_t* count,
                  int32_t* next, const double* u, void* stream);

/* Reduced basis from the window and the snapshot at the new centre (Sec. 4.2, basis for
 * compliance output, where the adjoint snapshots equal the primal ones):
 *   Phi = GramSchmidt([POD_nk(U), u]),  n_k = min(count, nmax),
 * POD_nk(U) being the n_k leading left singular vectors of the window's snapshot matrix
 * U (count columns; their order in the window does not matter) and the Gram-Schmidt
 * step the classical one (u minus its projections on the POD columns, normalised).
 * Computed by the method of snapshots: eigen-decomposition of G (float64 Jacobi), POD
 * column j = U V_j / sigma_j.  POD directions with sigma_j <= rtol * sigma_0 are not
 * kept, and u adds no column when what is left of it has norm <= rtol * |u|.
 *   u [n] f64 device, may be NULL (POD of the window only);
 *   phi [n][ldphi] out, f32 (phi_fp32 != 0) or f64, row-major like every basis of this
 *        library; columns 0..*ncols-1 are written, the others are left untouched;
 *   *ncols (host out): columns written, the POD ones first then u's;
 *   *npod (host out, may be NULL): POD columns kept;
 *   sigma [count] f64 device out (may be NULL): singular values of U, descending.
 * The accuracy of a POD direction degrades with the square of sigma_0 / sigma_j (the
 * method of snapshots works with their squares), so rtol is meant to be >= about 1e-7.
 * Synchronises the stream (the column count is returned to the host).  Errors:
 * TOPO_EINVAL (null pointer, n < 1, L or count out of range, nmax < 0, rtol outside
 * [0, 1), nothing to build, ldphi smaller than min(count, nmax) + (u != NULL)),
 * TOPO_ENOMEM, TOPO_EDEVICE. */
int topo_pod_basis(topo_ctx* ctx, int64_t n, int32_t L, const double* S, const double* G,
                   int32_t count, const double* u, int32_t nmax, double rtol, void* phi,
                   int32_t phi_fp32, int32_t ldphi, int32_t* ncols, int32_t* npod,
                   double* sigma, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TOPO_ROM_H */
