// Full-order model on the device: matrix-free K(rho) apply, Jacobi-preconditioned CG
// with float64 iterative refinement, compliance and element sensitivity
// (Sec. 2.1 state equation, Sec. 2.3 compliance, Sec. 2.4 sensitivity).
//
// Global reductions never cross blocks inside a kernel: each kernel writes one
// partial per block, and the consumer kernel (the next one in the stream) sums the
// partials of its producer in a fixed order, redundantly in every block.  Kernel
// boundaries provide the coherence between the XCDs' L2 caches, so no fences or
// atomics are needed and every result is bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include <hip/hip_ext.h>

#include "graphs.hpp"
#include "march3.hpp"
#include "stencil.hpp"

namespace topo {

// ----------------------------------------------------------------------------------
// Per-solve tables: alpha_e in both precisions, 1 / sum_{e ∋ n} alpha_e per node.
// ----------------------------------------------------------------------------------
__global__ void k_alpha(int ne, const double* __restrict__ rho, double E0, double Emin,
                        double p, double* __restrict__ a64, float* __restrict__ a32) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t b = blockIdx.y;
    if (e >= (size_t)ne) return;
    const double a = simp_alpha(rho[b * ne + e], E0, Emin, p);
    if (a64) a64[b * ne + e] = a;
    if (a32) a32[b * ne + e] = (float)a;
}

__global__ void k_winv(Grid g, const double* __restrict__ a64, double* __restrict__ w64,
                       float* __restrict__ w32) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= g.n_nodes) return;
    int i, j, k;
    node_ijk(g, n, i, j, k);
    const double s = node_alpha_sum(g, i, j, k, a64);
    const double w = s > 0.0 ? 1.0 / s : 0.0;
    if (w64) w64[n] = w;
    if (w32) w32[n] = (float)w;
}

// ----------------------------------------------------------------------------------
// Public apply: y_b = K(rho_b) x_b, Dirichlet rows and columns eliminated.
// ----------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_apply2(Grid g, const T* __restrict__ alpha,
                                                   const T* __restrict__ K,
                                                   const uint8_t* __restrict__ mask,
                                                   const T* __restrict__ x, T* __restrict__ y) {
    const int n = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (n >= g.n_nodes) return;
    const size_t b = blockIdx.y;
    const T* xb = x + b * g.n_dofs;
    T* yb = y + b * g.n_dofs;
    const T* ab = alpha + b * g.n_elems;
    int i, j, k;
    node_ijk(g, n, i, j, k);
    FetchMasked<T> f{xb, mask, g.n_nodes};
    T out[2];
    node_apply2<T>(g, i, j, ab, K, f, out);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const size_t idx = (size_t)c * g.n_nodes + n;
        yb[idx] = mask[idx] ? T(0) : out[c];
    }
}

// Sources of the 3D march (march3.hpp): the values of node planes, fetched two slots
// per thread with every load issued unconditionally (an invalid node reads node 0 and
// is zeroed afterwards).
template <typename T>
struct SrcMasked {  // x with Dirichlet DOFs zeroed
    const T* __restrict__ x;
    const uint8_t* __restrict__ mask;
    int nn;
    T v[4][3];
    __device__ __forceinline__ void fetch(int slot, int node) {
        const int n = node >= 0 ? node : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T xv = x[c * nn + n];
            const uint8_t mk = mask[c * nn + n];
            v[slot][c] = (node < 0 || mk) ? T(0) : xv;
        }
    }
    __device__ __forceinline__ T value(int slot, int c) const { return v[slot][c]; }
};

template <typename T>
struct SrcPlain {
    const T* __restrict__ x;
    int nn;
    T v[4][3];
    __device__ __forceinline__ void fetch(int slot, int node) {
        const int n = node >= 0 ? node : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T xv = x[c * nn + n];
            v[slot][c] = node >= 0 ? xv : T(0);
        }
    }
    __device__ __forceinline__ T value(int slot, int c) const { return v[slot][c]; }
};

template <typename T>
struct SrcDirection {  // p_new = z + beta p_old
    const T* __restrict__ z;
    const T* __restrict__ p;
    T beta;
    int nn;
    T zv[4][3], pv[4][3];
    __device__ __forceinline__ void fetch(int slot, int node) {
        const int n = node >= 0 ? node : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T a = z[c * nn + n], b = p[c * nn + n];
            zv[slot][c] = node >= 0 ? a : T(0);
            pv[slot][c] = node >= 0 ? b : T(0);
        }
    }
    __device__ __forceinline__ T value(int slot, int c) const { return zv[slot][c] + beta * pv[slot][c]; }
};

// Fetch the two prologue planes k0 - 1 (slots 0, 1) and k0 (slots 2, 3).
template <typename Src>
__device__ __forceinline__ void march3_prologue(const Grid& g, const MarchBlock& m,
                                                const MarchSlots& sl, Src& src) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        src.fetch(r, march3_node(g, sl, r, m.k0 - 1));
        src.fetch(2 + r, march3_node(g, sl, r, m.k0));
    }
}

// 3D: one block per march column (blockIdx.x), one field per blockIdx.y.  M is the
// table of reduced element blocks (apply3_from_n).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_apply3(Grid g, const T* __restrict__ alpha,
                                                   const T* __restrict__ M,
                                                   const uint8_t* __restrict__ mask,
                                                   const T* __restrict__ x, T* __restrict__ y) {
    __shared__ MarchLds<T> L;
    const size_t b = blockIdx.y;
    const MarchBlock m = march3_block(g, xcd_block(blockIdx.x, gridDim.x));
    for (int i = threadIdx.x; i < kFacSize; i += blockDim.x) L.M[i] = M[i];
    const MarchSlots sl = march3_slots(g, m);
    SrcMasked<T> src{x + b * g.n_dofs, mask, g.n_nodes};
    march3_prologue(g, m, sl, src);
    T* yb = y + b * g.n_dofs;
    auto emit = [&](int n, const T (&out)[3], const T (&)[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t idx = (size_t)c * g.n_nodes + n;
            yb[idx] = mask[idx] ? T(0) : out[c];
        }
    };
    march3_run(g, m, sl, alpha + b * g.n_elems, L, src, emit);
}

// ----------------------------------------------------------------------------------
// Jacobi-PCG, two kernels per iteration:
//   k_pcg_apply (iteration it): beta = rz_it / rz_{it-1}; p_new = z + beta p_old fused
//                 into the stencil; q = K p_new; pq partials.  Also the stopping test
//                 on rr = ||r_it||^2.
//   k_pcg_update(iteration it): alpha = rz_it / pq; x += alpha p, r -= alpha q,
//                 z = D^{-1} r; rz / rr partials of the next iteration.
// Partials: part = [pq | rz(parity 0) | rz(parity 1) | rr(parity 0) | rr(parity 1)],
// ps doubles apart; the apply writes one pq partial per stencil block (napp), the
// initialisation and the update one rz / rr partial per node-linear block (nupd).
// Iteration it writes rz/rr into parity it & 1 and reads the current ones from parity
// (it + 1) & 1.  The PCG initialisation writes parity 1.  The apply of iteration it
// records its summed rz_it in the state by parity (rz[it & 1]): the update of the same
// iteration and the next apply read it there instead of summing its partials again.
// Block 0 alone writes the state record (done flag, iteration count, norms, rz).
// ----------------------------------------------------------------------------------
struct PcgState {
    double bb;    // reference ||r||^2 of the stopping test (set by the first apply, or by
                  // the host when a segment continues after a residual replacement)
    double rr;    // ||r||^2 at the last stopping test
    double tol2;  // the segment stops when rr <= tol2 * bb
    double rz[2]; // summed r.z of the last two applies, by iteration parity
    int done;     // 0 running, 1 converged, 2 iteration limit, 3 breakdown
    int iters;    // completed iterations (over all segments)
    int maxit;
    int pad;
};

__device__ __forceinline__ double* part_rz(double* p, int ps, int parity) { return p + (1 + parity) * ps; }
__device__ __forceinline__ double* part_rr(double* p, int ps, int parity) { return p + (3 + parity) * ps; }

// Block size of the node-linear PCG kernels and of the 2D apply: fewer, larger blocks
// leave fewer partial sums for the next kernel's prologue (measured at 241k DOF: 8 %
// shorter kernels than with 256 threads; 1024 threads were slower again).
constexpr int kPcgBlock = 512;

template <int DIM, typename T>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_init(Grid g, const T* __restrict__ b,
                                                     const T* __restrict__ winv, T ik0, T ik1,
                                                     T ik2, double* __restrict__ x, T* __restrict__ r,
                                                     T* __restrict__ z, T* __restrict__ p,
                                                     double* __restrict__ part, PcgState* st,
                                                     int ps, int maxit, double tol2) {
    __shared__ double lds[32];
    double v[2] = {0.0, 0.0};
    const T ik[3] = {ik0, ik1, ik2};
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < g.n_nodes; n += gridDim.x * blockDim.x) {
        const T w = winv[n];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const size_t i = (size_t)c * g.n_nodes + n;
            const T bi = b[i];
            const T zi = bi * w * ik[c];
            x[i] = 0.0;
            r[i] = bi;
            z[i] = zi;
            p[i] = T(0);
            v[0] += (double)bi * (double)zi;
            v[1] += (double)bi * (double)bi;
        }
    }
    block_reduce<2>(v, lds);
    if (threadIdx.x == 0) {
        part_rz(part, ps, 1)[blockIdx.x] = v[0];
        part_rr(part, ps, 1)[blockIdx.x] = v[1];
        if (blockIdx.x == 0) {
            st->done = 0;
            st->iters = 0;
            st->maxit = maxit;
            st->bb = 0.0;
            st->rr = 0.0;
            st->tol2 = tol2;
        }
    }
}

// Stopping test and CG coefficient of an apply, from the update partials (every block
// computes the same values).  Returns the done code; tb is beta.
template <typename T>
__device__ __forceinline__ int pcg_apply_scalars(double* part, PcgState* st, int ps, int nupd,
                                                 int parity, int first, T& tb, double* lds) {
    const int cur = (parity + 1) & 1;
    // rr and rz of the current residual (one pass); rz of the previous apply from the state
    const double* arrs[2] = {part_rr(part, ps, cur), part_rz(part, ps, cur)};
    double red[2];
    block_sum_arrays<2>(arrs, nupd, red, lds);
    const double rr = red[0];
    const double bb = first ? rr : st->bb;
    int code = 0;
    if (!isfinite(rr)) code = 3;
    else if (rr <= st->tol2 * bb) code = 1;
    else if (st->iters >= st->maxit) code = 2;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (first) st->bb = rr;
        st->rr = rr;
        if (code) st->done = code;
        else st->rz[parity] = red[1];
    }
    tb = first ? T(0) : (T)(red[1] / st->rz[cur]);
    return code;
}

// 2D: one node per thread (the launch covers every node).  The node's loads are issued
// before it waits on the scalar reduction.
template <typename T>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_apply2(Grid g, const T* __restrict__ alpha,
                                                       const T* __restrict__ K,
                                                       const uint8_t* __restrict__ mask,
                                                       const T* __restrict__ z,
                                                       const T* __restrict__ p_old,
                                                       T* __restrict__ p_new, T* __restrict__ q,
                                                       double* __restrict__ part, PcgState* st,
                                                       int ps, int nupd, int parity, int first) {
    if (st->done) return;
    __shared__ double lds[48];
    const int n = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const bool own = n < g.n_nodes;
    T zs[3][3][2], ps_[3][3][2], al[2][2];
    uint8_t mk[2];
    if (own) {
        int i, j, k;
        node_ijk(g, n, i, j, k);
        load_nbhd2(g, i, j, FetchPlain<T>{z, g.n_nodes}, zs);
        load_nbhd2(g, i, j, FetchPlain<T>{p_old, g.n_nodes}, ps_);
        load_alpha2(g, i, j, alpha, al);
#pragma unroll
        for (int c = 0; c < 2; ++c) mk[c] = mask[(size_t)c * g.n_nodes + n];
    }
    T tb;
    if (pcg_apply_scalars(part, st, ps, nupd, parity, first, tb, lds)) return;
    double v[1] = {0.0};
    if (own) {
        T out[2], pn[2];
        T xs[3][3][2];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int c = 0; c < 2; ++c) xs[dy][dx][c] = zs[dy][dx][c] + tb * ps_[dy][dx][c];
        pn[0] = xs[1][1][0];
        pn[1] = xs[1][1][1];
        apply_nbhd2(K, xs, al, out);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t idx = (size_t)c * g.n_nodes + n;
            const T qv = mk[c] ? T(0) : out[c];
            p_new[idx] = pn[c];
            q[idx] = qv;
            v[0] += (double)pn[c] * (double)qv;
        }
    }
    block_reduce<1>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// 3D: one block per march column.  The first two node planes of z and p_old are
// fetched before the scalar reduction; p_new = z + beta p_old is formed per node as
// the planes are staged, and the element march runs from LDS.  M is the table of
// reduced element blocks.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pcg_apply3(Grid g, const T* __restrict__ alpha,
                                                       const T* __restrict__ M,
                                                       const uint8_t* __restrict__ mask,
                                                       const T* __restrict__ z,
                                                       const T* __restrict__ p_old,
                                                       T* __restrict__ p_new, T* __restrict__ q,
                                                       double* __restrict__ part, PcgState* st,
                                                       int ps, int nrz, int parity, int first) {
    if (st->done) return;
    __shared__ MarchLds<T> L;
    __shared__ double lds[48];
    const MarchBlock m = march3_block(g, xcd_block(blockIdx.x, gridDim.x));
    for (int i = threadIdx.x; i < kFacSize; i += blockDim.x) L.M[i] = M[i];
    const MarchSlots sl = march3_slots(g, m);
    SrcDirection<T> src{z, p_old, T(0), g.n_nodes};
    march3_prologue(g, m, sl, src);
    T tb;
    if (pcg_apply_scalars(part, st, ps, nrz, parity, first, tb, lds)) return;
    src.beta = tb;
    double v[1] = {0.0};
    auto emit = [&](int n, const T (&out)[3], const T (&pn)[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t idx = (size_t)c * g.n_nodes + n;
            const T qv = mask[idx] ? T(0) : out[c];
            p_new[idx] = pn[c];
            q[idx] = qv;
            v[0] += (double)pn[c] * (double)qv;
        }
    };
    march3_run(g, m, sl, alpha, L, src, emit);
    block_reduce<1>(v, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// One node per thread (the launch covers every node); the node's loads are issued
// before the wait on the scalar reduction.
template <int DIM, typename T>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_update(Grid g, const T* __restrict__ winv,
                                                       T ik0, T ik1, T ik2, double* __restrict__ x,
                                                       T* __restrict__ r, T* __restrict__ z,
                                                       const T* __restrict__ p,
                                                       const T* __restrict__ q,
                                                       double* __restrict__ part, PcgState* st,
                                                       int ps, int npq, int parity) {
    if (st->done) return;
    __shared__ double lds[32];
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const bool own = n < g.n_nodes;
    double xv[DIM];
    T rv[DIM], pv[DIM], qv[DIM], w = T(0);
    if (own) {
        w = winv[n];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const size_t i = (size_t)c * g.n_nodes + n;
            xv[c] = x[i];
            rv[c] = r[i];
            pv[c] = p[i];
            qv[c] = q[i];
        }
    }
    const double pq = block_sum_array(part, npq, lds);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) st->done = 3;
        return;
    }
    const T a = (T)(st->rz[parity] / pq);
    const T ik[3] = {ik0, ik1, ik2};
    double v[2] = {0.0, 0.0};
    if (own) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const size_t i = (size_t)c * g.n_nodes + n;
            x[i] = xv[c] + (double)a * (double)pv[c];
            const T ri = rv[c] - a * qv[c];
            const T zi = ri * w * ik[c];
            r[i] = ri;
            z[i] = zi;
            v[0] += (double)ri * (double)zi;
            v[1] += (double)ri * (double)ri;
        }
    }
    block_reduce<2>(v, lds);
    if (threadIdx.x == 0) {
        part_rz(part, ps, parity)[blockIdx.x] = v[0];
        part_rr(part, ps, parity)[blockIdx.x] = v[1];
        if (blockIdx.x == 0) st->iters = st->iters + 1;
    }
}

// In-place fixed-order sum of the per-block partials of large launches: a[0] = sum of
// a[0..n), and likewise b when given (one block).  The consumer then reads 1 value
// instead of every block summing all partials again.  Skipped once the recursion is
// done: its producer did not run then, and summing again would count a[0] twice.
__global__ __launch_bounds__(1024) void k_partials_sum(double* __restrict__ a,
                                                       double* __restrict__ b, int n,
                                                       const int* done) {
    if (*done) return;
    __shared__ double lds[32];
    double v[2] = {0.0, 0.0};
    constexpr int U = 8;  // loads in flight per thread
    for (int i0 = threadIdx.x; i0 < n; i0 += U * blockDim.x) {
        double ta[U], tb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * blockDim.x;
            ta[u] = i < n ? a[i] : 0.0;
            tb[u] = (b && i < n) ? b[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v[0] += ta[u];
            v[1] += tb[u];
        }
    }
    block_reduce<2>(v, lds);
    if (threadIdx.x == 0) {
        a[0] = v[0];
        if (b) b[0] = v[1];
    }
}

// Residual replacement: the segment's correction has been added to u in float64 and
// the true residual r64 = f - K u recomputed; the recursion continues from
// r = scale * r64 (x restarts at 0, the search direction p is kept), so the Krylov
// progress of the earlier segments is not lost.  Writes the rz / rr partials of the
// replaced residual into parity `cur`, where the next apply reads them.
template <int DIM, typename T>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_replace(Grid g, const double* __restrict__ r64,
                                                        double scale, const T* __restrict__ winv,
                                                        T ik0, T ik1, T ik2, double* __restrict__ x,
                                                        T* __restrict__ r, T* __restrict__ z,
                                                        double* __restrict__ part, int ps, int cur) {
    __shared__ double lds[32];
    double v[2] = {0.0, 0.0};
    const T ik[3] = {ik0, ik1, ik2};
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < g.n_nodes; n += gridDim.x * blockDim.x) {
        const T w = winv[n];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const size_t i = (size_t)c * g.n_nodes + n;
            const T ri = (T)(scale * r64[i]);
            const T zi = ri * w * ik[c];
            x[i] = 0.0;
            r[i] = ri;
            z[i] = zi;
            v[0] += (double)ri * (double)zi;
            v[1] += (double)ri * (double)ri;
        }
    }
    block_reduce<2>(v, lds);
    if (threadIdx.x == 0) {
        part_rz(part, ps, cur)[blockIdx.x] = v[0];
        part_rr(part, ps, cur)[blockIdx.x] = v[1];
    }
}

// ----------------------------------------------------------------------------------
// 2D: Jacobi-PCG with one reduction phase per iteration (the Chronopoulos-Gear form of
// CG), one kernel per iteration.  With u = D^{-1} r, w = K u and s = K p:
//   beta_i = gamma_i / gamma_{i-1},  alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}),
//   p_i = u_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1},  x += alpha_i p_i,
//   r_{i+1} = r_i - alpha_i s_i,  u_{i+1} = D^{-1} r_{i+1},  w_{i+1} = K u_{i+1},
//   gamma_{i+1} = r_{i+1}.u_{i+1},  delta_{i+1} = w_{i+1}.u_{i+1}.
// The stencil needs u_{i+1} on the 3x3 neighbourhood of a node; a thread forms it
// there from r_i, w_i and s_{i-1} (elementwise), so a launch needs nothing from another
// block of the same launch, and its scalars come from the partials of the previous one.
// r, w and s are double-buffered: step i reads set i & 1 (r_i, w_i, s_{i-1}) and writes
// set (i + 1) & 1 (r_{i+1}, w_{i+1}, s_i); p and x are updated in place (own node only).
// Partials: part = [gamma(0) | gamma(1) | delta(0) | delta(1) | rr(0) | rr(1) | u.s | p.s],
// ps doubles apart, by the parity of the residual they belong to.  The state keeps
// gamma, alpha and the iteration count by parity: step i reads the slots of step i - 1
// and writes its own, so no block reads a value another block of its launch writes.
// ----------------------------------------------------------------------------------
struct Cg1State {
    double bb;        // reference ||r||^2 of the stopping test
    double rr;        // ||r||^2 at the last stopping test
    double tol2;      // the segment stops when rr <= tol2 * bb
    double gamma[2];  // gamma_i by parity of i
    double alpha[2];  // alpha_i by parity of i
    int done;         // 0 running, 1 converged, 2 iteration limit, 3 breakdown
    int maxit;
    int iters[2];     // step i writes iters[i & 1] = i + 1
};

enum { kCg1Step = 0, kCg1Fresh = 1, kCg1Continued = 2, kCg1Init = 3 };

__device__ __forceinline__ double* cg1_part(double* p, int ps, int k) { return p + (size_t)k * ps; }

// Node value of a per-node array on the 3x3 neighbourhood (zero outside the grid).
template <typename T>
__device__ __forceinline__ void load_node_nbhd2(const Grid& g, int i, int j, const T* __restrict__ a,
                                                T (&v)[3][3]) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int ii = i + dx - 1, jj = j + dy - 1;
            const bool ok = (ii >= 0) & (ii < g.nx1) & (jj >= 0) & (jj < g.ny1);
            v[dy][dx] = ok ? a[jj * g.nx1 + ii] : T(0);
        }
}

// One step (KIND kCg1Step / kCg1Fresh / kCg1Continued) at parity `parity`, or the
// initialisation (kCg1Init: r_0 = Rin = b, w_0 = K D^{-1} b, p = s = x = 0, written to
// set 0 with parity = 1).  A fresh step takes beta = 0; a continued step (after a
// residual replacement) takes the direction K-conjugate to the kept p, with the exact
// p^T K p, from the u.s / p.s partials of k_cg1_replace2.
template <typename T, int KIND>
__global__ __launch_bounds__(kPcgBlock) void k_cg1_step2(
    Grid g, const T* __restrict__ alpha, const T* __restrict__ K, const uint8_t* __restrict__ mask,
    const T* __restrict__ winv, T ik0, T ik1, const T* __restrict__ Rin, const T* __restrict__ Win,
    const T* __restrict__ Sin, T* __restrict__ Rout, T* __restrict__ Wout, T* __restrict__ Sout,
    T* __restrict__ P, double* __restrict__ x, double* __restrict__ part, Cg1State* st, int ps,
    int npart, int parity, int maxit, double tol2) {
    if (KIND != kCg1Init && st->done) return;
    __shared__ double lds[80];
    const int n = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const bool own = n < g.n_nodes;
    T rs[3][3][2], ws[3][3][2], ss[3][3][2], wv[3][3], al[2][2], pv[2];
    double xv[2];
    uint8_t mk[2];
    int i = 0, j = 0, k = 0;
    if (own) {  // every load is issued before the wait on the scalar reduction
        node_ijk(g, n, i, j, k);
        load_nbhd2(g, i, j, FetchPlain<T>{Rin, g.n_nodes}, rs);
        if constexpr (KIND != kCg1Init) {
            load_nbhd2(g, i, j, FetchPlain<T>{Win, g.n_nodes}, ws);
            load_nbhd2(g, i, j, FetchPlain<T>{Sin, g.n_nodes}, ss);
        }
        load_node_nbhd2(g, i, j, winv, wv);
        load_alpha2(g, i, j, alpha, al);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t idx = (size_t)c * g.n_nodes + n;
            mk[c] = mask[idx];
            if constexpr (KIND != kCg1Init) {
                pv[c] = P[idx];
                xv[c] = x[idx];
            }
        }
    }
    const int cur = parity, nxt = parity ^ 1;
    double be = 0.0, ah = 0.0;
    if constexpr (KIND == kCg1Init) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->done = 0;
            st->maxit = maxit;
            st->iters[0] = st->iters[1] = 0;
            st->bb = st->rr = 0.0;
            st->tol2 = tol2;
        }
    } else {
        double red[5];
        if constexpr (KIND == kCg1Continued) {
            const double* arrs[5] = {cg1_part(part, ps, cur), cg1_part(part, ps, 2 + cur),
                                     cg1_part(part, ps, 4 + cur), cg1_part(part, ps, 6),
                                     cg1_part(part, ps, 7)};
            block_sum_arrays<5>(arrs, npart, red, lds);
        } else {
            const double* arrs[3] = {cg1_part(part, ps, cur), cg1_part(part, ps, 2 + cur),
                                     cg1_part(part, ps, 4 + cur)};
            double r3[3];
            block_sum_arrays<3>(arrs, npart, r3, lds);
            red[0] = r3[0];
            red[1] = r3[1];
            red[2] = r3[2];
        }
        const double gam = red[0], dlt = red[1], rr = red[2];
        const double bb = KIND == kCg1Fresh ? rr : st->bb;
        int code = 0;
        if (!isfinite(rr)) code = 3;
        else if (rr <= st->tol2 * bb) code = 1;
        else if (st->iters[nxt] >= st->maxit) code = 2;
        if (!code) {
            if constexpr (KIND == kCg1Fresh) {
                ah = gam / dlt;
            } else if constexpr (KIND == kCg1Continued) {
                const double us = red[3], pss = red[4];
                if (pss > 0.0 && isfinite(pss)) {
                    be = -us / pss;
                    ah = gam / (dlt + be * us);
                } else {
                    ah = gam / dlt;
                }
            } else {
                be = gam / st->gamma[nxt];
                ah = gam / (dlt - be * gam / st->alpha[nxt]);
            }
            if (!(ah > 0.0) || !isfinite(ah) || !isfinite(be)) code = 3;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (KIND == kCg1Fresh) st->bb = rr;
            st->rr = rr;
            if (code) {
                st->done = code;
            } else {
                st->gamma[cur] = gam;
                st->alpha[cur] = ah;
                st->iters[cur] = st->iters[nxt] + 1;
            }
        }
        if (code) return;
    }
    double v[3] = {0.0, 0.0, 0.0};
    if (own) {
        const T tb = (T)be, ta = (T)ah;
        const T ik[2] = {ik0, ik1};
        T un[3][3][2], snew[2], rnew[2], unew[2];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    T si = T(0), rn = rs[dy][dx][c];
                    if constexpr (KIND != kCg1Init) {
                        si = ws[dy][dx][c] + tb * ss[dy][dx][c];
                        rn = rn - ta * si;
                    }
                    un[dy][dx][c] = rn * wv[dy][dx] * ik[c];
                    if (dy == 1 && dx == 1) {
                        snew[c] = si;
                        rnew[c] = rn;
                        unew[c] = un[1][1][c];
                    }
                }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t idx = (size_t)c * g.n_nodes + n;
            if constexpr (KIND == kCg1Init) {
                P[idx] = T(0);
                x[idx] = 0.0;
            } else {
                const T pn = rs[1][1][c] * wv[1][1] * ik[c] + tb * pv[c];  // u_i + beta p_{i-1}
                P[idx] = pn;
                x[idx] = xv[c] + (double)ta * (double)pn;
            }
            Sout[idx] = snew[c];
            Rout[idx] = rnew[c];
        }
        T out[2];
        apply_nbhd2(K, un, al, out);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t idx = (size_t)c * g.n_nodes + n;
            const T wn = mk[c] ? T(0) : out[c];
            Wout[idx] = wn;
            v[0] += (double)rnew[c] * (double)unew[c];
            v[1] += (double)wn * (double)unew[c];
            v[2] += (double)rnew[c] * (double)rnew[c];
        }
    }
    block_reduce<3>(v, lds);
    if (threadIdx.x == 0) {
        cg1_part(part, ps, nxt)[blockIdx.x] = v[0];
        cg1_part(part, ps, 2 + nxt)[blockIdx.x] = v[1];
        cg1_part(part, ps, 4 + nxt)[blockIdx.x] = v[2];
    }
}

// s = K p recomputed for the direction of the last step, into the set that step wrote.
// The recursion s_i = w_i + beta_i s_{i-1} carries each rounding of K u through about
// 1 / (1 - beta) iterations (beta ~ 0.98 here), which in float32 lets the recursive
// residual drift from the true one; refreshing s every kPcgChunk iterations bounds
// that sum.  Reads p (neighbourhood) only and writes s (own node).
template <typename T>
__global__ __launch_bounds__(kPcgBlock) void k_cg1_refresh2(Grid g, const T* __restrict__ alpha,
                                                         const T* __restrict__ K,
                                                         const uint8_t* __restrict__ mask,
                                                         const T* __restrict__ P, T* __restrict__ S,
                                                         const Cg1State* st) {
    if (st->done) return;
    const int n = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (n >= g.n_nodes) return;
    int i, j, k;
    node_ijk(g, n, i, j, k);
    T ps_[3][3][2], al[2][2], out[2];
    load_nbhd2(g, i, j, FetchPlain<T>{P, g.n_nodes}, ps_);
    load_alpha2(g, i, j, alpha, al);
    apply_nbhd2(K, ps_, al, out);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const size_t idx = (size_t)c * g.n_nodes + n;
        S[idx] = mask[idx] ? T(0) : out[c];
    }
}

// Residual replacement of the one-reduction recursion: r = scale * r64 (the float64 true
// residual), u = D^{-1} r, w = K u, and s = K p computed exactly for the kept direction
// p, written to set `cur` with x = 0; partials of gamma, delta, rr (parity cur) and of
// u.s, p.s, from which the continued step takes its conjugate direction.
template <typename T>
__global__ __launch_bounds__(kPcgBlock) void k_cg1_replace2(
    Grid g, const T* __restrict__ alpha, const T* __restrict__ K, const uint8_t* __restrict__ mask,
    const T* __restrict__ winv, T ik0, T ik1, const double* __restrict__ r64, double scale,
    const T* __restrict__ P, T* __restrict__ R, T* __restrict__ W, T* __restrict__ S,
    double* __restrict__ x, double* __restrict__ part, int ps, int cur) {
    __shared__ double lds[80];
    const int n = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (n < g.n_nodes) {
        int i, j, k;
        node_ijk(g, n, i, j, k);
        double rs[3][3][2];
        T ps_[3][3][2], wv[3][3], al[2][2];
        load_nbhd2(g, i, j, FetchPlain<double>{r64, g.n_nodes}, rs);
        load_nbhd2(g, i, j, FetchPlain<T>{P, g.n_nodes}, ps_);
        load_node_nbhd2(g, i, j, winv, wv);
        load_alpha2(g, i, j, alpha, al);
        const T ik[2] = {ik0, ik1};
        T un[3][3][2], rown[2], uown[2], pown[2];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const T rn = (T)(scale * rs[dy][dx][c]);
                    un[dy][dx][c] = rn * wv[dy][dx] * ik[c];
                    if (dy == 1 && dx == 1) {
                        rown[c] = rn;
                        uown[c] = un[1][1][c];
                        pown[c] = ps_[1][1][c];
                    }
                }
        T wo[2], so[2];
        apply_nbhd2(K, un, al, wo);
        apply_nbhd2(K, ps_, al, so);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t idx = (size_t)c * g.n_nodes + n;
            const bool fixed = mask[idx] != 0;
            const T wn = fixed ? T(0) : wo[c];
            const T sn = fixed ? T(0) : so[c];
            R[idx] = rown[c];
            W[idx] = wn;
            S[idx] = sn;
            x[idx] = 0.0;
            v[0] += (double)rown[c] * (double)uown[c];
            v[1] += (double)wn * (double)uown[c];
            v[2] += (double)rown[c] * (double)rown[c];
            v[3] += (double)uown[c] * (double)sn;
            v[4] += (double)pown[c] * (double)sn;
        }
    }
    block_reduce<5>(v, lds);
    if (threadIdx.x == 0) {
        cg1_part(part, ps, cur)[blockIdx.x] = v[0];
        cg1_part(part, ps, 2 + cur)[blockIdx.x] = v[1];
        cg1_part(part, ps, 4 + cur)[blockIdx.x] = v[2];
        cg1_part(part, ps, 6)[blockIdx.x] = v[3];
        cg1_part(part, ps, 7)[blockIdx.x] = v[4];
    }
}

// ----------------------------------------------------------------------------------
// float64 residual r = f - K u over free DOFs (u zero on Dirichlet DOFs), with
// per-block partials of ||r||^2, f^T u and u^T r for every field (blockIdx.y);
// k_residual_sum reduces them (one block per field) into out[4*b .. 4*b+2].
// ----------------------------------------------------------------------------------
// Residual, compliance and u^T r terms of one free DOF, accumulated into v.
__device__ __forceinline__ double residual_dof(const uint8_t* __restrict__ mask,
                                               const double* __restrict__ f,
                                               const double* __restrict__ ub, double* rb,
                                               size_t idx, double o, double (&v)[3]) {
    const bool fixed = mask[idx] != 0;
    const double fi = fixed ? 0.0 : f[idx];
    const double ui = ub[idx];
    const double ri = fixed ? 0.0 : fi - o;
    if (rb) rb[idx] = ri;
    v[0] += ri * ri;
    v[1] += fi * ui;
    v[2] += ui * ri;
    return ri;
}

__device__ __forceinline__ void residual_partials(double (&v)[3], double* __restrict__ part,
                                                  size_t b, double* lds) {
    block_reduce<3>(v, lds);
    const int nb = gridDim.x;
    double* pb = part + b * 3 * nb;
    if (threadIdx.x == 0) {
        pb[blockIdx.x] = v[0];
        pb[nb + blockIdx.x] = v[1];
        pb[2 * nb + blockIdx.x] = v[2];
    }
}

__global__ __launch_bounds__(kBlock) void k_residual2(Grid g, const double* __restrict__ alpha,
                                                      const double* __restrict__ K,
                                                      const uint8_t* __restrict__ mask,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ f,
                                                      double* __restrict__ r,
                                                      double* __restrict__ part) {
    __shared__ double lds[48];
    const size_t b = blockIdx.y;
    const int n = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const double* ub = u + b * g.n_dofs;
    double v[3] = {0.0, 0.0, 0.0};
    if (n < g.n_nodes) {
        int i, j, k;
        node_ijk(g, n, i, j, k);
        double o[2];
        node_apply2<double>(g, i, j, alpha + b * g.n_elems, K, FetchPlain<double>{ub, g.n_nodes}, o);
#pragma unroll
        for (int c = 0; c < 2; ++c)
            residual_dof(mask, f, ub, r ? r + b * g.n_dofs : nullptr, (size_t)c * g.n_nodes + n, o[c], v);
    }
    residual_partials(v, part, b, lds);
}

// 3D: one block per march column; M is the table of reduced element blocks.
__global__ __launch_bounds__(kBlock) void k_residual3(Grid g, const double* __restrict__ alpha,
                                                      const double* __restrict__ M,
                                                      const uint8_t* __restrict__ mask,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ f,
                                                      double* __restrict__ r,
                                                      double* __restrict__ part) {
    __shared__ MarchLds<double> L;
    __shared__ double lds[48];
    const size_t b = blockIdx.y;
    const double* ub = u + b * g.n_dofs;
    const MarchBlock m = march3_block(g, xcd_block(blockIdx.x, gridDim.x));
    for (int i = threadIdx.x; i < kFacSize; i += blockDim.x) L.M[i] = M[i];
    const MarchSlots sl = march3_slots(g, m);
    SrcPlain<double> src{ub, g.n_nodes};
    march3_prologue(g, m, sl, src);
    double v[3] = {0.0, 0.0, 0.0};
    double* rb = r ? r + b * g.n_dofs : nullptr;
    auto emit = [&](int n, const double (&o)[3], const double (&)[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) residual_dof(mask, f, ub, rb, (size_t)c * g.n_nodes + n, o[c], v);
    };
    march3_run(g, m, sl, alpha + b * g.n_elems, L, src, emit);
    residual_partials(v, part, b, lds);
}

__global__ __launch_bounds__(kBlock) void k_residual_sum(int nb, const double* __restrict__ part,
                                                         double* __restrict__ out) {
    __shared__ double lds[16];
    const int b = blockIdx.x;
    const double* pb = part + (size_t)b * 3 * nb;
    const double s0 = block_sum_array(pb, nb, lds);
    const double s1 = block_sum_array(pb + nb, nb, lds);
    const double s2 = block_sum_array(pb + 2 * nb, nb, lds);
    if (threadIdx.x == 0) {
        out[4 * b + 0] = s0;
        out[4 * b + 1] = s1;
        out[4 * b + 2] = s2;
    }
}

// rhs of a correction solve: b = s * r (cast to the inner precision)
template <typename T>
__global__ void k_scale_cast(long long n, const double* __restrict__ r, double s, T* __restrict__ b) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (T)(s * r[i]);
}

// u += s * d
template <typename T>
__global__ void k_correct(long long n, double* __restrict__ u, const T* __restrict__ d, double s) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] += s * (double)d[i];
}

// ----------------------------------------------------------------------------------
// Element sensitivity dc_e = -alpha'(rho_e) u_e^T K_e u_e   (float64), one field per
// blockIdx.y (rho [B][N_e], u [B][N_u], dc [B][N_e])
// ----------------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_gradient(Grid g, const double* __restrict__ rho,
                                                     const double* __restrict__ K,
                                                     const double* __restrict__ u, double E0,
                                                     double Emin, double p,
                                                     double* __restrict__ dc) {
    constexpr int NEN = 1 << DIM;
    constexpr int NE = DIM * NEN;
    const int e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (e >= g.n_elems) return;
    rho += (size_t)blockIdx.y * g.n_elems;
    u += (size_t)blockIdx.y * g.n_dofs;
    dc += (size_t)blockIdx.y * g.n_elems;
    const int ex = e % g.nx;
    const int t = e / g.nx;
    const int ey = t % g.ny;
    const int ez = t / g.ny;
    double ue[NE];
#pragma unroll
    for (int a = 0; a < NEN; ++a) {
        const int n = ((ez + (a >> 2)) * g.ny1 + (ey + ((a >> 1) & 1))) * g.nx1 + ex + (a & 1);
#pragma unroll
        for (int c = 0; c < DIM; ++c) ue[DIM * a + c] = u[(size_t)c * g.n_nodes + n];
    }
    // K_e annihilates rigid translations, so removing the element's mean displacement
    // leaves u_e^T K_e u_e unchanged and avoids cancellation on near-rigid elements.
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        double m = 0.0;
#pragma unroll
        for (int a = 0; a < NEN; ++a) m += ue[DIM * a + c];
        m *= 1.0 / NEN;
#pragma unroll
        for (int a = 0; a < NEN; ++a) ue[DIM * a + c] -= m;
    }
    double qf = 0.0;
#pragma unroll
    for (int i = 0; i < NE; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NE; ++j) s += K[i * NE + j] * ue[j];
        qf += ue[i] * s;
    }
    const double r = rho[e];
    double dp;  // d(rho^p)/d rho
    if (p == 3.0) dp = 3.0 * r * r;
    else if (p == 1.0) dp = 1.0;
    else if (p == 2.0) dp = 2.0 * r;
    else dp = p * pow(r, p - 1.0);
    dc[e] = -(E0 - Emin) * dp * qf;
}

// ----------------------------------------------------------------------------------
// Host drivers
// ----------------------------------------------------------------------------------
static int launch_tables(Ctx* ctx, const Grid& g, const topo_mesh& m, const double* rho,
                         int B, double* a64, float* a32, double* w64, float* w32,
                         hipStream_t s) {
    dim3 ga(grid_blocks(g.n_elems), B);
    hipLaunchKernelGGL(k_alpha, ga, dim3(kBlock), 0, s, g.n_elems, rho, m.E0, m.Emin, m.penal,
                       a64, a32);
    TOPO_CHECK_LAUNCH();
    if (w64 || w32) {
        hipLaunchKernelGGL(k_winv, dim3(grid_blocks(g.n_nodes)), dim3(kBlock), 0, s, g, a64, w64, w32);
        TOPO_CHECK_LAUNCH();
    }
    return TOPO_OK;
}

// Inner PCG solve K x = b in precision T to ||r||/||b|| <= tol (recursive residual).
template <int DIM, typename T>
struct PcgRun {
    const T* alpha;
    const T* K;
    const uint8_t* mask;
    const T* winv;
    T ik[3];
    T *b, *r, *z, *p0, *p1, *q;
    double* x;  // the segment's correction, accumulated in float64
    double* part;
    PcgState* st;
};


// Launch geometry of the PCG kernels: node-linear blocks for the init / update, stencil
// blocks for the apply, the stride of the partial arrays, and how many partials each
// consumer sums (1 when a launch has more blocks than kPcgMaxBlocks: its partials are
// then summed once by k_partials_sum).
struct PcgGeom {
    int nupd, napp, ps;
    int npq, nrz;  // partials read of the apply's pq and of the update's rz / rr
};

static PcgGeom pcg_geom(const Grid& g) {
    PcgGeom pg;
    pg.nupd = grid_blocks(g.n_nodes, kPcgBlock);
    pg.napp = g.dim == 2 ? grid_blocks(g.n_nodes, kPcgBlock) : stencil_blocks(g);
    pg.ps = std::max(pg.nupd, pg.napp);
    pg.npq = pg.napp > kPcgMaxBlocks ? 1 : pg.napp;
    pg.nrz = pg.nupd > kPcgMaxBlocks ? 1 : pg.nupd;
    return pg;
}


// Collapse the rz / rr partials of parity `par` written by a node-linear launch.
static void pcg_sum_rz(const PcgGeom& pg, double* part, int par, const PcgState* st, LaunchSink& L) {
    if (pg.nrz == 1 && pg.nupd > 1)
        L((const void*)k_partials_sum, dim3(1), dim3(1024), part + (1 + par) * (size_t)pg.ps,
          part + (3 + par) * (size_t)pg.ps, (int)pg.nupd, (const int*)&st->done);
}

// One PCG iteration (apply + update).
template <int DIM, typename T>
static void pcg_iteration(Ctx* ctx, const Grid& g, const PcgRun<DIM, T>& w, const PcgGeom& pg,
                          int parity, int first, LaunchSink& L, int timing) {
    const T* pold = parity ? w.p1 : w.p0;
    T* pnew = parity ? w.p0 : w.p1;
    const T* zc = w.z;
    {
        TimedLaunch tl(ctx, KID_PCG_APPLY, L.s, L.graph ? kTimeOff : timing, true);
        L.ev0 = tl.a;
        L.ev1 = tl.b;
        const void* fn = DIM == 2 ? (const void*)k_pcg_apply2<T> : (const void*)k_pcg_apply3<T>;
        L(fn, dim3(pg.napp), dim3(DIM == 2 ? kPcgBlock : kBlock), g, w.alpha, w.K, w.mask, zc, pold, pnew, w.q, w.part, w.st,
          (int)pg.ps, (int)pg.nrz, parity, first);
    }
    if (pg.npq == 1 && pg.napp > 1)
        L((const void*)k_partials_sum, dim3(1), dim3(1024), w.part, (double*)nullptr, (int)pg.napp,
          (const int*)&w.st->done);
    {
        TimedLaunch tl(ctx, KID_PCG_UPDATE, L.s, L.graph ? kTimeOff : timing, true);
        L.ev0 = tl.a;
        L.ev1 = tl.b;
        L((const void*)k_pcg_update<DIM, T>, dim3(pg.nupd), dim3(kPcgBlock), g, w.winv, w.ik[0], w.ik[1],
          w.ik[2], w.x, w.r, w.z, (const T*)pnew, (const T*)w.q, w.part, w.st, (int)pg.ps, (int)pg.npq,
          parity);
    }
    pcg_sum_rz(pg, w.part, parity, w.st, L);
}

constexpr int kPcgChunk = 16;  // iterations per graph replay (even)

// Graph of kPcgChunk iterations starting at parity 1 (so every replay continues the
// parity sequence).
template <int DIM, typename T>
static int pcg_graph(Ctx* ctx, const Grid& g, const PcgRun<DIM, T>& w, const PcgGeom& pg,
                     hipGraphExec_t* out) {
    std::vector<uintptr_t> key = {(uintptr_t)DIM, sizeof(T), (uintptr_t)pg.napp, (uintptr_t)kPcgChunk,
                                  (uintptr_t)g.nx, (uintptr_t)g.ny, (uintptr_t)g.nz,
                                  (uintptr_t)w.alpha, (uintptr_t)w.K, (uintptr_t)w.mask,
                                  (uintptr_t)w.winv, (uintptr_t)w.x, (uintptr_t)w.r, (uintptr_t)w.z,
                                  (uintptr_t)w.p0, (uintptr_t)w.p1, (uintptr_t)w.q, (uintptr_t)w.part,
                                  (uintptr_t)w.st};
    for (int c = 0; c < 3; ++c) key_push_double(key, (double)w.ik[c]);
    return cached_graph(ctx, key, [&](LaunchSink& L) {
        for (int c = 0; c < kPcgChunk; ++c) pcg_iteration<DIM, T>(ctx, g, w, pg, (1 + c) & 1, 0, L, kTimeOff);
    }, out);
}

// Runs iterations until the device state (type S, with a `done` field) reports done:
// graph replays of kPcgChunk iterations (exec), or without graphs direct launches in
// growing chunks; `direct(it, mode)` launches iteration it (parity it & 1).  issued: iterations
// launched so far (odd when exec is used).  The host checks the state one chunk behind.
template <typename S, typename Direct>
static int pcg_poll(Ctx* ctx, hipStream_t s, const S* st, hipGraphExec_t exec, long long issued,
                    long long cap, Direct direct, S* result) {
    void* pin = nullptr;
    int rc = pinned_host(ctx, 2 * sizeof(S), &pin);
    if (rc) return rc;
    S* hs = (S*)pin;
    hipEvent_t ev[2];
    TOPO_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    TOPO_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    bool pending[2] = {false, false};
    long long replays = 0;
    int chunk = 4;
    int slot = 0;
    while (true) {
        const int every = ctx->timing.every;
        if (exec && !(every > 0 && replays % every == 0)) {
            TOPO_HIP(hipGraphLaunch(exec, s));
            issued += kPcgChunk;
        } else if (exec) {
            // timing sample: two directly launched, timed iterations (keeps the parity)
            for (int c = 0; c < 2; ++c, ++issued) direct(issued, kTimeForced);
        } else {
            for (int c = 0; c < chunk; ++c, ++issued) direct(issued, kTimeSampled);
            if (chunk < 64) chunk *= 2;
        }
        ++replays;
        TOPO_CHECK_LAUNCH();
        TOPO_HIP(hipMemcpyAsync(&hs[slot], st, sizeof(S), hipMemcpyDeviceToHost, s));
        TOPO_HIP(hipEventRecord(ev[slot], s));
        pending[slot] = true;
        const int other = slot ^ 1;
        bool stop = false;
        if (pending[other]) {
            TOPO_HIP(hipEventSynchronize(ev[other]));
            pending[other] = false;
            stop = hs[other].done != 0;
        }
        if (stop || issued >= cap) break;
        slot = other;
    }
    TOPO_HIP(hipStreamSynchronize(s));
    TOPO_HIP(hipEventDestroy(ev[0]));
    TOPO_HIP(hipEventDestroy(ev[1]));
    TOPO_HIP(hipMemcpyAsync(&hs[0], st, sizeof(S), hipMemcpyDeviceToHost, s));
    TOPO_HIP(hipStreamSynchronize(s));
    *result = hs[0];
    return TOPO_OK;
}

// Runs PCG iterations until the device state reports done.  fresh: initialise from
// w.b (x = 0) with stopping tolerance tol and maxit, and run iteration 0 (which records
// ||b||^2); otherwise continue a segment whose state (done = 0, bb, tol2) the host has
// uploaded after a residual replacement, at iteration iters0.
template <int DIM, typename T>
static int pcg_run(Ctx* ctx, const Grid& g, PcgRun<DIM, T>& w, bool fresh, double tol, int maxit,
                   int iters0, hipStream_t s, PcgState* result) {
    const PcgGeom pg = pcg_geom(g);
    LaunchSink L;
    L.s = s;
    long long issued;
    if (fresh) {
        hipLaunchKernelGGL((k_pcg_init<DIM, T>), dim3(pg.nupd), dim3(kPcgBlock), 0, s, g, w.b, w.winv,
                           w.ik[0], w.ik[1], w.ik[2], w.x, w.r, w.z, w.p0, w.part, w.st, pg.ps,
                           maxit, tol * tol);
        TOPO_CHECK_LAUNCH();
        pcg_sum_rz(pg, w.part, 1, w.st, L);
        // iteration 0 (parity 0) records ||b||; the rest continue at parity 1
        pcg_iteration<DIM, T>(ctx, g, w, pg, 0, 1, L, kTimeSampled);
        issued = 1;
    } else {
        issued = iters0;
        if ((issued & 1) == 0) {  // graphs start at an odd iteration
            pcg_iteration<DIM, T>(ctx, g, w, pg, 0, 0, L, kTimeSampled);
            ++issued;
        }
    }
    TOPO_CHECK_LAUNCH();
    TOPO_HIP(L.err);
    hipGraphExec_t exec = nullptr;
    if (graphs_enabled()) {
        const int rc = pcg_graph<DIM, T>(ctx, g, w, pg, &exec);
        if (rc) return rc;
    }
    auto direct = [&](long long it, int mode) { pcg_iteration<DIM, T>(ctx, g, w, pg, (int)(it & 1), 0, L, mode); };
    const int rc = pcg_poll<PcgState>(ctx, s, w.st, exec, issued, (long long)maxit + 4096, direct, result);
    if (rc) return rc;
    TOPO_HIP(L.err);
    return TOPO_OK;
}

// ----------------------------------------------------------------------------------
// Host side of the 2D one-reduction recursion (k_cg1_step2).
// ----------------------------------------------------------------------------------
template <typename T>
struct Cg1Run {
    const T* alpha;
    const T* K;
    const uint8_t* mask;
    const T* winv;
    T ik[2];
    T* b;
    T *R[2], *W[2], *S[2];  // r, w = K D^{-1} r, s = K p by parity
    T* P;
    double* x;
    double* part;
    Cg1State* st;
    int nb, npart, ps;  // blocks, partials each block sums, partial stride
};

// Collapse the partials of parity par (and the u.s / p.s ones of a replacement) when the
// launch had more blocks than kPcgMaxBlocks.
template <typename T>
static void cg1_sum(const Cg1Run<T>& w, int par, bool extra, LaunchSink& L) {
    if (w.npart != 1 || w.nb <= 1) return;
    const int* done = &w.st->done;
    const size_t ps = (size_t)w.ps;
    L((const void*)k_partials_sum, dim3(1), dim3(1024), w.part + par * ps, w.part + (2 + par) * ps, w.nb, done);
    L((const void*)k_partials_sum, dim3(1), dim3(1024), w.part + (4 + par) * ps,
      extra ? w.part + 6 * ps : (double*)nullptr, w.nb, done);
    if (extra)
        L((const void*)k_partials_sum, dim3(1), dim3(1024), w.part + 7 * ps, (double*)nullptr, w.nb, done);
}

template <typename T>
static void cg1_step(Ctx* ctx, const Grid& g, const Cg1Run<T>& w, int parity, int kind, LaunchSink& L,
                     int timing, bool refresh = false) {
    const int nxt = parity ^ 1;
    {
        TimedLaunch tl(ctx, KID_PCG_STEP, L.s, L.graph ? kTimeOff : timing, true);
        L.ev0 = tl.a;
        L.ev1 = tl.b;
        const void* fn = kind == kCg1Fresh       ? (const void*)k_cg1_step2<T, kCg1Fresh>
                         : kind == kCg1Continued ? (const void*)k_cg1_step2<T, kCg1Continued>
                                                 : (const void*)k_cg1_step2<T, kCg1Step>;
        L(fn, dim3(w.nb), dim3(kPcgBlock), g, w.alpha, w.K, w.mask, w.winv, w.ik[0], w.ik[1],
          (const T*)w.R[parity], (const T*)w.W[parity], (const T*)w.S[parity], w.R[nxt], w.W[nxt],
          w.S[nxt], w.P, w.x, w.part, w.st, w.ps, w.npart, parity, 0, 0.0);
    }
    cg1_sum(w, nxt, false, L);
    if (refresh)
        L((const void*)k_cg1_refresh2<T>, dim3(w.nb), dim3(kPcgBlock), g, w.alpha, w.K, w.mask, (const T*)w.P,
          w.S[nxt], (const Cg1State*)w.st);
}

// The one-reduction counterpart of pcg_run: fresh (init from w.b, then a first step with
// beta = 0) or continued after k_cg1_replace2 has written set iters0 & 1.
template <typename T>
static int cg1_run(Ctx* ctx, const Grid& g, Cg1Run<T>& w, bool fresh, double tol, int maxit, int iters0,
                   hipStream_t s, Cg1State* result) {
    LaunchSink L;
    L.s = s;
    long long issued;
    if (fresh) {
        L((const void*)k_cg1_step2<T, kCg1Init>, dim3(w.nb), dim3(kPcgBlock), g, w.alpha, w.K, w.mask,
          w.winv, w.ik[0], w.ik[1], (const T*)w.b, (const T*)nullptr, (const T*)nullptr, w.R[0], w.W[0],
          w.S[0], w.P, w.x, w.part, w.st, w.ps, w.npart, 1, maxit, tol * tol);
        cg1_sum(w, 0, false, L);
        cg1_step(ctx, g, w, 0, kCg1Fresh, L, kTimeSampled);
        issued = 1;
    } else {
        cg1_step(ctx, g, w, iters0 & 1, kCg1Continued, L, kTimeSampled);
        issued = iters0 + 1;
        if ((issued & 1) == 0) {  // graphs start at an odd iteration
            cg1_step(ctx, g, w, 0, kCg1Step, L, kTimeSampled);
            ++issued;
        }
    }
    TOPO_CHECK_LAUNCH();
    TOPO_HIP(L.err);
    hipGraphExec_t exec = nullptr;
    if (graphs_enabled()) {
        std::vector<uintptr_t> key = {(uintptr_t)0xC61, sizeof(T), (uintptr_t)w.nb, (uintptr_t)w.npart,
                                      (uintptr_t)w.ps, (uintptr_t)kPcgChunk, (uintptr_t)g.nx, (uintptr_t)g.ny,
                                      (uintptr_t)w.alpha, (uintptr_t)w.K, (uintptr_t)w.mask, (uintptr_t)w.winv,
                                      (uintptr_t)w.R[0], (uintptr_t)w.R[1], (uintptr_t)w.W[0], (uintptr_t)w.W[1],
                                      (uintptr_t)w.S[0], (uintptr_t)w.S[1], (uintptr_t)w.P, (uintptr_t)w.x,
                                      (uintptr_t)w.part, (uintptr_t)w.st};
        for (int c = 0; c < 2; ++c) key_push_double(key, (double)w.ik[c]);
        const int rc = cached_graph(ctx, key, [&](LaunchSink& G) {
            for (int c = 0; c < kPcgChunk; ++c)
                cg1_step(ctx, g, w, (1 + c) & 1, kCg1Step, G, kTimeOff, c == kPcgChunk - 1);
        }, &exec);
        if (rc) return rc;
    }
    // iteration it refreshes s when it ends a chunk of kPcgChunk (as the graph's last step)
    auto direct = [&](long long it, int mode) {
        cg1_step(ctx, g, w, (int)(it & 1), kCg1Step, L, mode, (it % kPcgChunk) == 0);
    };
    const int rc = pcg_poll<Cg1State>(ctx, s, w.st, exec, issued, (long long)maxit + 4096, direct, result);
    if (rc) return rc;
    TOPO_HIP(L.err);
    return TOPO_OK;
}

// Largest ratio of true to recursive residual at the end of a segment for which the
// recursion is continued after the residual replacement (else it restarts).
static double replace_drift_max() {
    static double v = [] {
        const char* e = std::getenv("TOPO_REPLACE_DRIFT");
        return e ? std::atof(e) : 4.0;
    }();
    return v;
}

// Whether a 2D solve runs the one-reduction recursion (one kernel per iteration):
// float64 solves do; float32 solves keep the two-kernel recursion, whose recursively
// updated residual stays closer to the true one in float32 (the one-reduction form also
// updates s = K p recursively, and at 241k DOF needed 2.4x the iterations in float32).
// TOPO_PCG_ONE_REDUCTION=1 / 0 selects it for both precisions / for neither.
static bool one_reduction(bool fp64) {
    static const int mode = [] {
        const char* e = std::getenv("TOPO_PCG_ONE_REDUCTION");
        return e && e[0] ? std::atoi(e) : -1;
    }();
    return mode < 0 ? fp64 : mode != 0;
}

// Reduction of the residual a float32 segment aims for before its residual is replaced
// by the float64 one (small enough to keep the replacements rare, large enough that the
// float32 recursion has not drifted from the true residual).
static double mixed_segment_tol() {
    static double v = [] {
        const char* e = std::getenv("TOPO_MIXED_SEGMENT_TOL");
        double t = e ? std::atof(e) : 0.0;
        return t > 0.0 ? t : 1e-2;
    }();
    return v;
}

// K64: the dense element matrix in 2D, the reduced element blocks in 3D.
static int residual_launch(Ctx* ctx, const Grid& g0, const double* K64, const double* alpha64,
                           const uint8_t* mask, const double* u, const double* f, double* r, int B,
                           double* part, double* out, hipStream_t s) {
    // the residual march fits its own resident wave (never more blocks than a grid with
    // the default target, which sized the caller's partial arrays)
    Grid g = g0;
    if (g.dim == 3) g.mtarget = std::min(march3_target(ctx, (const void*)k_residual3), g0.mtarget > 0 ? g0.mtarget : 1024);
    const int nb = stencil_blocks(g);
    {
        TimedLaunch tl(ctx, KID_RESIDUAL, s);
        if (g.dim == 2)
            hipLaunchKernelGGL(k_residual2, dim3(nb, B), dim3(kBlock), 0, s, g, alpha64, K64, mask,
                               u, f, r, part);
        else
            hipLaunchKernelGGL(k_residual3, dim3(nb, B), dim3(kBlock), 0, s, g, alpha64, K64, mask,
                               u, f, r, part);
    }
    TOPO_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_residual_sum, dim3(B), dim3(kBlock), 0, s, nb, (const double*)part, out);
    TOPO_CHECK_LAUNCH();
    return TOPO_OK;
}

template <typename T>
struct HdmWs {
    double *a64, *w64, *r64, *part, *rpart, *rout, *x;
    T *b, *r, *z, *p0, *p1, *q;
    T *e0 = nullptr, *e1 = nullptr;  // 2D: the one-reduction recursion's two further vectors
    float *a32 = nullptr, *w32 = nullptr;
    PcgState* st;
    Cg1State* st1;
};

template <typename T>
static void hdm_takes(Arena& ar, const Grid& g, bool mixed, HdmWs<T>& w) {
    const long long N = g.n_dofs;
    const int nb = partial_stride(g);
    ar.take(&w.a64, g.n_elems);
    ar.take(&w.w64, g.n_nodes);
    if (mixed) {
        ar.take(&w.a32, g.n_elems);
        ar.take(&w.w32, g.n_nodes);
    }
    ar.take(&w.r64, N);
    ar.take(&w.part, 8 * (size_t)nb);  // 5 arrays in 3D, 8 in 2D
    ar.take(&w.rpart, 3 * (size_t)nb);
    ar.take(&w.rout, 4);
    ar.take(&w.st, 1);
    ar.take(&w.st1, 1);
    ar.take(&w.b, N);
    ar.take(&w.x, N);
    ar.take(&w.r, N);
    ar.take(&w.z, N);
    ar.take(&w.p0, N);
    ar.take(&w.p1, N);
    ar.take(&w.q, N);
    if (g.dim == 2) {
        ar.take(&w.e0, N);
        ar.take(&w.e1, N);
    }
}

size_t ws_hdm_solve(const Grid& g, bool mixed) {
    Arena ar;
    if (mixed) {
        HdmWs<float> w;
        hdm_takes(ar, g, true, w);
    } else {
        HdmWs<double> w;
        hdm_takes(ar, g, false, w);
    }
    return ar.total();
}

template <int DIM, typename T>
static int hdm_solve_impl(Ctx* ctx, const topo_mesh& m, const Grid& g0, const ElemTables* tb,
                          const double* rho, const uint8_t* mask, const double* f, double* u,
                          double rtol, int maxit, bool mixed, double* compliance,
                          topo_info* info, hipStream_t s, bool* stagnated) {
    Grid g = g0;
    if constexpr (DIM == 3) g.mtarget = march3_target(ctx, (const void*)k_pcg_apply3<T>);
    const long long N = g.n_dofs;
    if (stagnated) *stagnated = false;
    Arena ar;
    HdmWs<T> ws;
    hdm_takes(ar, g, mixed, ws);
    int rc = ar.commit(ctx, s);
    if (rc) return rc;
    double *a64 = ws.a64, *w64 = ws.w64, *r64 = ws.r64, *part = ws.part, *rpart = ws.rpart,
           *rout = ws.rout;
    T *b = ws.b, *r = ws.r, *z = ws.z, *p0 = ws.p0, *p1 = ws.p1, *q = ws.q;
    double* x = ws.x;
    float *a32 = ws.a32, *w32 = ws.w32;
    PcgState* st = ws.st;
    if (rc) return rc;
    rc = launch_tables(ctx, g, m, rho, 1, a64, a32, w64, w32, s);
    if (rc) return rc;
    const T* ta;
    const T* tw;
    if constexpr (sizeof(T) == 4) {
        ta = (const T*)a32;
        tw = (const T*)w32;
    } else {
        ta = (const T*)a64;
        tw = (const T*)w64;
    }
    PcgRun<DIM, T> w;
    w.alpha = ta;
    // 2D: the dense element matrix; 3D: the reduced blocks of the symmetry-blocked form
    if constexpr (DIM == 2) w.K = sizeof(T) == 4 ? (const T*)tb->K32 : (const T*)tb->K64;
    else w.K = sizeof(T) == 4 ? (const T*)tb->M32 : (const T*)tb->M64;
    w.mask = mask;
    w.winv = tw;
    for (int c = 0; c < 3; ++c) w.ik[c] = c < DIM ? (T)(1.0 / tb->diag[c]) : T(0);
    w.b = b;
    w.x = x;
    w.r = r;
    w.z = z;
    w.p0 = p0;
    w.p1 = p1;
    w.q = q;
    w.part = part;
    w.st = st;

    TOPO_HIP(hipMemsetAsync(u, 0, N * sizeof(double), s));
    // pinned host layout: [2 state poll slots | 4 residual sums | state upload]
    constexpr size_t kStateBytes = sizeof(PcgState) > sizeof(Cg1State) ? sizeof(PcgState) : sizeof(Cg1State);
    const size_t pin_res = 2 * kStateBytes;
    const size_t pin_up = pin_res + 4 * sizeof(double);
    void* pin = nullptr;
    rc = pinned_host(ctx, pin_up + kStateBytes, &pin);
    if (rc) return rc;
    auto residual = [&](double out[3]) -> int {
        int rc2 = residual_launch(ctx, g, g.dim == 2 ? tb->K64 : tb->M64, a64, mask, u, f, r64, 1, rpart, rout, s);
        if (rc2) return rc2;
        double* h = (double*)((char*)pin + pin_res);
        TOPO_HIP(hipMemcpyAsync(h, rout, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
        TOPO_HIP(hipStreamSynchronize(s));
        out[0] = h[0];
        out[1] = h[1];
        out[2] = h[2];
        return TOPO_OK;
    };
    double res[3];
    rc = residual(res);
    if (rc) return rc;
    // One Krylov recursion in precision T, cut into segments: each segment runs until
    // its recursive residual has dropped by tol_seg, then its correction is added to u
    // in float64, the true residual f - K u is recomputed in float64 and replaces the
    // recursive one, and the recursion continues with the same search direction.  The
    // inner system is scaled by 1 / ||f|| so that float32 values stay O(1).
    const double nf = std::sqrt(res[0]);
    const double scale = nf > 0.0 ? 1.0 / nf : 1.0;
    const double seg_min = mixed ? mixed_segment_tol() : 0.0;
    const PcgGeom pg = pcg_geom(g);
    const int bl = grid_blocks(N);
    const double drift_max = replace_drift_max();
    int total = 0, base = 0, segments = 0, status = TOPO_OK;
    bool fresh = true;
    double rr = res[0], rr_prev = INFINITY;
    // 2D: the one-reduction recursion (one kernel per iteration)
    const bool one_red = DIM == 2 && one_reduction(sizeof(T) == 8);
    Cg1Run<T> w1{};
    if (one_red) {
        w1.alpha = w.alpha;
        w1.K = w.K;
        w1.mask = mask;
        w1.winv = w.winv;
        w1.ik[0] = w.ik[0];
        w1.ik[1] = w.ik[1];
        w1.b = b;
        w1.R[0] = r;
        w1.R[1] = z;
        w1.W[0] = q;
        w1.W[1] = ws.e0;
        w1.S[0] = p0;
        w1.S[1] = p1;
        w1.P = ws.e1;
        w1.x = x;
        w1.part = part;
        w1.st = ws.st1;
        w1.nb = grid_blocks(g.n_nodes, kPcgBlock);
        w1.npart = w1.nb > kPcgMaxBlocks ? 1 : w1.nb;
        w1.ps = pg.ps;
    }
    struct {
        int done, iters;
        double rr, bb;
    } fin{};
    double last_rz[2] = {0.0, 0.0};  // 3D: r.z of the last two iterations of a segment
    // one segment of the recursion; its end state goes to fin
    auto run_segment = [&](bool fr, double tol, int mi, int it0) -> int {
        if (one_red) {
            Cg1State st1{};
            const int rc2 = cg1_run<T>(ctx, g, w1, fr, tol, mi, it0, s, &st1);
            if (rc2) return rc2;
            fin.done = st1.done;
            fin.iters = std::max(st1.iters[0], st1.iters[1]);
            fin.rr = st1.rr;
            fin.bb = st1.bb;
        } else {
            PcgState st0{};
            const int rc2 = pcg_run<DIM, T>(ctx, g, w, fr, tol, mi, it0, s, &st0);
            if (rc2) return rc2;
            fin.done = st0.done;
            fin.iters = st0.iters;
            fin.rr = st0.rr;
            fin.bb = st0.bb;
            last_rz[0] = st0.rz[0];
            last_rz[1] = st0.rz[1];
        }
        return TOPO_OK;
    };
    while (true) {
        const double rel = nf > 0.0 ? std::sqrt(rr) / nf : 0.0;
        if (rel <= rtol) break;
        if (total >= maxit || segments >= 400) {
            status = set_error(ctx, TOPO_ENOCONV, "no convergence: rel. residual %.3e after %d iterations",
                               rel, total);
            break;
        }
        if (segments > 0 && !(rr < 0.5 * rr_prev)) {
            status = set_error(ctx, TOPO_ENOCONV, "residual replacement stagnated at rel. residual %.3e", rel);
            if (stagnated) *stagnated = true;
            break;
        }
        double tol_seg = std::max(0.5 * rtol * nf / std::sqrt(rr), seg_min);
        tol_seg = std::min(std::max(tol_seg, 1e-15), 0.5);
        if (fresh) {
            hipLaunchKernelGGL((k_scale_cast<T>), dim3(bl), dim3(kBlock), 0, s, N, r64, scale, b);
            TOPO_CHECK_LAUNCH();
            base = total;
            rc = run_segment(true, tol_seg, maxit - base, 0);
        } else if (one_red) {
            Cg1State* up = (Cg1State*)((char*)pin + pin_up);
            *up = Cg1State{};
            up->bb = rr * scale * scale;
            up->rr = up->bb;
            up->tol2 = tol_seg * tol_seg;
            up->done = 0;
            up->maxit = maxit - base;
            up->iters[0] = up->iters[1] = fin.iters;
            TOPO_HIP(hipMemcpyAsync(w1.st, up, sizeof(Cg1State), hipMemcpyHostToDevice, s));
            const int cur = fin.iters & 1;
            hipLaunchKernelGGL((k_cg1_replace2<T>), dim3(w1.nb), dim3(kPcgBlock), 0, s, g, w1.alpha, w1.K,
                               mask, w1.winv, w1.ik[0], w1.ik[1], (const double*)r64, scale,
                               (const T*)w1.P, w1.R[cur], w1.W[cur], w1.S[cur], x, part, pg.ps, cur);
            TOPO_CHECK_LAUNCH();
            LaunchSink L;
            L.s = s;
            cg1_sum(w1, cur, true, L);
            TOPO_HIP(L.err);
            rc = run_segment(false, tol_seg, maxit - base, fin.iters);
        } else {
            // state first (done = 0), so that the partial sums below are not skipped
            PcgState* up = (PcgState*)((char*)pin + pin_up);
            *up = PcgState{};
            up->bb = rr * scale * scale;
            up->rr = up->bb;
            up->tol2 = tol_seg * tol_seg;
            up->done = 0;
            up->iters = fin.iters;
            up->maxit = maxit - base;
            // the replaced residual's apply takes beta against the last recursive rz
            up->rz[0] = last_rz[0];
            up->rz[1] = last_rz[1];
            TOPO_HIP(hipMemcpyAsync(st, up, sizeof(PcgState), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL((k_pcg_replace<DIM, T>), dim3(pg.nupd), dim3(kPcgBlock), 0, s, g,
                               (const double*)r64, scale, w.winv, w.ik[0], w.ik[1], w.ik[2], x, r, z,
                               part, pg.ps, (fin.iters + 1) & 1);
            TOPO_CHECK_LAUNCH();
            LaunchSink L;
            L.s = s;
            pcg_sum_rz(pg, part, (fin.iters + 1) & 1, st, L);
            TOPO_HIP(L.err);
            rc = run_segment(false, tol_seg, maxit - base, fin.iters);
        }
        if (rc) return rc;
        const int seg_iters = base + fin.iters - total;
        total = base + fin.iters;
        if (std::getenv("TOPO_DEBUG_PCG"))
            fprintf(stderr, "[pcg] segment %d (%s): %d its, done %d, recursive rel %.3e (tol %.1e), true rel before %.3e\n",
                    segments, fresh ? "fresh" : "continued", seg_iters, fin.done,
                    std::sqrt(fin.rr / std::max(fin.bb, 1e-300)), tol_seg, std::sqrt(rr) / nf);
        if (fin.done == 3 && seg_iters == 0) {
            status = set_error(ctx, TOPO_ENOTSPD, "CG breakdown: p^T K p <= 0");
            break;
        }
        hipLaunchKernelGGL((k_correct<double>), dim3(bl), dim3(kBlock), 0, s, N, u, (const double*)x,
                           nf > 0.0 ? nf : 1.0);
        TOPO_CHECK_LAUNCH();
        ++segments;
        rr_prev = rr;
        rc = residual(res);
        if (rc) return rc;
        rr = res[0];
        if (fin.done == 3 && !(rr < rr_prev)) {
            status = set_error(ctx, TOPO_ENOTSPD, "CG breakdown: p^T K p <= 0");
            break;
        }
        // continue the recursion only while it still tracks the true residual; a
        // segment whose true residual drifted far from the recursive one restarts
        const double drift = fin.rr > 0.0 ? std::sqrt(rr) * scale / std::sqrt(fin.rr) : INFINITY;
        fresh = !(drift <= drift_max) || fin.done != 1;
    }
    if (info) {
        info->iters = total;
        info->refinements = segments;
        info->rel_resid = nf > 0.0 ? std::sqrt(rr) / nf : 0.0;
        info->compliance_raw = res[1];
        info->compliance_corr = res[1] + res[2];
    }
    if (compliance) *compliance = res[1] + res[2];
    return status;
}

}  // namespace topo

using namespace topo;

extern "C" {

int topo_apply(topo_ctx* ctx, const topo_mesh* mesh, const double* rho, const uint8_t* mask,
               const void* x, void* y, int32_t B, int32_t prec, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    int rc = validate_mesh(ctx, mesh);
    if (rc) return rc;
    if (!rho || !mask || !x || !y) return set_error(ctx, TOPO_EINVAL, "null pointer argument");
    if (B < 1) return set_error(ctx, TOPO_EINVAL, "B must be >= 1");
    if (prec != TOPO_FP64 && prec != TOPO_MIXED) return set_error(ctx, TOPO_EINVAL, "bad precision");
    TOPO_HIP(hipSetDevice(ctx->device));
    Grid g = make_grid(*mesh);
    if (g.dim == 3)
        g.mtarget = march3_target(ctx, prec == TOPO_FP64 ? (const void*)k_apply3<double> : (const void*)k_apply3<float>);
    const ElemTables* tb = get_tables(ctx, *mesh);
    if (!tb) return set_error(ctx, TOPO_EDEVICE, "element table upload failed");
    hipStream_t s = (hipStream_t)stream;
    Arena ar;
    double* a64 = nullptr;
    float* a32 = nullptr;
    if (prec == TOPO_FP64) ar.take(&a64, (size_t)B * g.n_elems);
    else ar.take(&a32, (size_t)B * g.n_elems);
    rc = ar.commit(ctx, s);
    if (rc) return rc;
    rc = launch_tables(ctx, g, *mesh, rho, B, a64, a32, nullptr, nullptr, s);
    if (rc) return rc;
    dim3 grid(stencil_blocks(g), B);
    TimedLaunch tl(ctx, KID_APPLY, s);
    if (prec == TOPO_FP64) {
        if (g.dim == 2)
            hipLaunchKernelGGL((k_apply2<double>), grid, dim3(kBlock), 0, s, g, a64, tb->K64, mask,
                               (const double*)x, (double*)y);
        else
            hipLaunchKernelGGL((k_apply3<double>), grid, dim3(kBlock), 0, s, g, a64, tb->M64, mask,
                               (const double*)x, (double*)y);
    } else {
        if (g.dim == 2)
            hipLaunchKernelGGL((k_apply2<float>), grid, dim3(kBlock), 0, s, g, a32, tb->K32, mask,
                               (const float*)x, (float*)y);
        else
            hipLaunchKernelGGL((k_apply3<float>), grid, dim3(kBlock), 0, s, g, a32, tb->M32, mask,
                               (const float*)x, (float*)y);
    }
    TOPO_CHECK_LAUNCH();
    return TOPO_OK;
}

int topo_hdm_solve(topo_ctx* ctx, const topo_mesh* mesh, const double* rho, const uint8_t* mask,
                   const double* f, double* u, double rtol, int32_t maxit, int32_t prec,
                   double* compliance, topo_info* info, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    int rc = validate_mesh(ctx, mesh);
    if (rc) return rc;
    if (!rho || !mask || !f || !u) return set_error(ctx, TOPO_EINVAL, "null pointer argument");
    if (!(rtol > 0.0) || !(rtol < 1.0)) return set_error(ctx, TOPO_EINVAL, "rtol must lie in (0, 1)");
    if (maxit < 1) return set_error(ctx, TOPO_EINVAL, "maxit must be >= 1");
    if (prec != TOPO_FP64 && prec != TOPO_MIXED) return set_error(ctx, TOPO_EINVAL, "bad precision");
    TOPO_HIP(hipSetDevice(ctx->device));
    const Grid g = make_grid(*mesh);
    const ElemTables* tb = get_tables(ctx, *mesh);
    if (!tb) return set_error(ctx, TOPO_EDEVICE, "element table upload failed");
    hipStream_t s = (hipStream_t)stream;
    topo_info local{};
    topo_info* inf = info ? info : &local;
    *inf = topo_info{};
    if (prec == TOPO_FP64)
        return g.dim == 2 ? hdm_solve_impl<2, double>(ctx, *mesh, g, tb, rho, mask, f, u, rtol, maxit,
                                                      false, compliance, inf, s, nullptr)
                          : hdm_solve_impl<3, double>(ctx, *mesh, g, tb, rho, mask, f, u, rtol, maxit,
                                                      false, compliance, inf, s, nullptr);
    // mixed: float32 inner solves; if a float32 correction fails to reduce the true
    // residual (float32 rounding too coarse for this operator), redo the solve in float64
    bool stagnated = false;
    rc = g.dim == 2 ? hdm_solve_impl<2, float>(ctx, *mesh, g, tb, rho, mask, f, u, rtol, maxit, true,
                                               compliance, inf, s, &stagnated)
                    : hdm_solve_impl<3, float>(ctx, *mesh, g, tb, rho, mask, f, u, rtol, maxit, true,
                                               compliance, inf, s, &stagnated);
    if (rc != TOPO_ENOCONV || !stagnated) return rc;
    const topo_info first = *inf;
    const int left = maxit - first.iters;
    if (left < 1) return rc;
    rc = g.dim == 2 ? hdm_solve_impl<2, double>(ctx, *mesh, g, tb, rho, mask, f, u, rtol, left, false,
                                                compliance, inf, s, nullptr)
                    : hdm_solve_impl<3, double>(ctx, *mesh, g, tb, rho, mask, f, u, rtol, left, false,
                                                compliance, inf, s, nullptr);
    inf->iters += first.iters;
    inf->refinements += first.refinements;
    inf->fp64_fallback = 1;
    return rc;
}

int topo_hdm_gradient(topo_ctx* ctx, const topo_mesh* mesh, const double* rho, const double* u,
                      double* dc, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    int rc = validate_mesh(ctx, mesh);
    if (rc) return rc;
    if (!rho || !u || !dc) return set_error(ctx, TOPO_EINVAL, "null pointer argument");
    TOPO_HIP(hipSetDevice(ctx->device));
    const Grid g = make_grid(*mesh);
    const ElemTables* tb = get_tables(ctx, *mesh);
    if (!tb) return set_error(ctx, TOPO_EDEVICE, "element table upload failed");
    return gradient_launch(ctx, g, *mesh, tb, rho, u, 1, dc, (hipStream_t)stream);
}

}  // extern "C"

namespace topo {

int gradient_launch(Ctx* ctx, const Grid& g, const topo_mesh& m, const ElemTables* tb,
                    const double* rho, const double* u, int B, double* dc, hipStream_t s) {
    TimedLaunch tl(ctx, KID_GRADIENT, s);
    const dim3 grid(grid_blocks(g.n_elems), B);
    if (g.dim == 2)
        hipLaunchKernelGGL((k_gradient<2>), grid, dim3(kBlock), 0, s, g, rho, tb->K64, u, m.E0,
                           m.Emin, m.penal, dc);
    else
        hipLaunchKernelGGL((k_gradient<3>), grid, dim3(kBlock), 0, s, g, rho, tb->K64, u, m.E0,
                           m.Emin, m.penal, dc);
    TOPO_CHECK_LAUNCH();
    return TOPO_OK;
}

}  // namespace topo

// Entry points shared with the ROM translation unit.
namespace topo {

int residual_fp64(Ctx* ctx, const Grid& g, const ElemTables* tb, const double* alpha64,
                  const uint8_t* mask, const double* u, const double* f, double* r, int B,
                  double* part, double* out, hipStream_t s) {
    return residual_launch(ctx, g, g.dim == 2 ? tb->K64 : tb->M64, alpha64, mask, u, f, r, B, part, out, s);
}

int alpha_tables(Ctx* ctx, const Grid& g, const topo_mesh& m, const double* rho, int B,
                 double* a64, float* a32, hipStream_t s) {
    return launch_tables(ctx, g, m, rho, B, a64, a32, nullptr, nullptr, s);
}

}  // namespace topo
