// Full-order model on the device: matrix-free K(rho) apply, Jacobi-preconditioned CG
// with float64 iterative refinement, compliance and element sensitivity
// (Sec. 2.1 state equation, Sec. 2.3 compliance, Sec. 2.4 sensitivity), for B density
// fields per launch.
//
// Global reductions never cross blocks inside a kernel: each kernel writes one
// partial per block, and the consumer kernel (the next one in the stream) sums the
// partials of its producer in a fixed order, redundantly in every block.  Kernel
// boundaries provide the coherence between the XCDs' L2 caches, so no fences or
// atomics are needed and every result is bitwise reproducible.
//
// Batches: every launch of a solve covers B fields (one per blockIdx.y, or mapped with
// field_block); each field has its own vectors, partial arrays and recursion state,
// and every stopping, restart and replacement decision is taken per field, so a
// field's result is bitwise the same alone and in any batch.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include <hip/hip_ext.h>

#include "graphs.hpp"
#include "march3.hpp"
#include "stencil.hpp"

namespace topo {

// ----------------------------------------------------------------------------------
// Per-solve tables: alpha_e in both precisions, 1 / sum_{e ∋ n} alpha_e per node, for
// B fields (blockIdx.y).
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
    const size_t b = blockIdx.y;
    int i, j, k;
    node_ijk(g, n, i, j, k);
    const double s = node_alpha_sum(g, i, j, k, a64 + b * g.n_elems);
    const double w = s > 0.0 ? 1.0 / s : 0.0;
    if (w64) w64[b * g.n_nodes + n] = w;
    if (w32) w32[b * g.n_nodes + n] = (float)w;
}

// ----------------------------------------------------------------------------------
// Public apply: y_b = K(rho_b) x_b, Dirichlet rows and columns eliminated.  astride:
// elements between the alpha tables of consecutive vectors (N_e; 0 when every vector
// shares one density field, as the columns of the ROM contraction do); vstride: entries
// between consecutive vectors of x and y (N_u, or a padded pitch).  T: arithmetic type;
// TX, TY: the types x and y are stored in (T, or float32 x for float64 arithmetic).
// ----------------------------------------------------------------------------------
template <typename T, typename TX = T, typename TY = T>
__global__ __launch_bounds__(kBlock) void k_apply2(Grid g, const T* __restrict__ alpha, long long astride,
                                                   long long vstride, const T* __restrict__ K,
                                                   const uint8_t* __restrict__ mask,
                                                   const TX* __restrict__ x, TY* __restrict__ y) {
    const FieldBlock fb = field_block();
    const int n = fb.blk * blockDim.x + threadIdx.x;
    if (n >= g.n_nodes) return;
    const size_t b = fb.field;
    const TX* xb = x + b * vstride;
    TY* yb = y + b * vstride;
    const T* ab = alpha + b * astride;
    int i, j, k;
    node_ijk(g, n, i, j, k);
    FetchMasked<T, TX> f{xb, mask, g.n_nodes};
    T out[2];
    node_apply2<T>(g, i, j, ab, K, f, out);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const size_t idx = (size_t)c * g.n_nodes + n;
        yb[idx] = mask[idx] ? TY(0) : (TY)out[c];
    }
}

// Sources of the 3D march (march3.hpp): the values of node planes, fetched two slots
// per thread with every load issued unconditionally (an invalid node reads node 0 and
// is zeroed afterwards).
template <typename T, typename TX = T>
struct SrcMasked {  // x (stored as TX) with Dirichlet DOFs zeroed
    const TX* __restrict__ x;
    const uint8_t* __restrict__ mask;
    int nn;
    T v[4][3];
    __device__ __forceinline__ void fetch(int slot, int node) {
        const int n = node >= 0 ? node : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T xv = (T)x[c * nn + n];
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


// The Jacobi-preconditioned residual z = r / K_ii = (r (1 / sum alpha)) (1 / K_e,cc), rounded
// after each product, so that the update (for r.z) and the 3D apply (for p) form the
// same value.
__device__ __forceinline__ float jacobi_z(float r, float w, float ik) { return __fmul_rn(__fmul_rn(r, w), ik); }
__device__ __forceinline__ double jacobi_z(double r, double w, double ik) {
    return __dmul_rn(__dmul_rn(r, w), ik);
}

// The float32 3D apply forms z from r and 1 / sum alpha (the update then stores no z);
// the float64 one reads z, whose registers it could not hold beside r and 1 / sum alpha.
template <typename T>
struct ApplyFormsZ {
    static constexpr bool value = sizeof(T) == 4;
};

// Source of the element-once march: p_new = z + beta p_old at nodes of the grid, z read
// (float64) or formed from r and 1 / sum alpha of the node (float32).  I: index type.
template <typename T, typename I>
struct SrcDirection3 {
    using Index = I;
    const T* __restrict__ r;
    const T* __restrict__ winv;
    const T* __restrict__ p;
    T ik[3];
    T beta;
    unsigned nn;
    static constexpr bool FORM = ApplyFormsZ<T>::value;
    T rv[4][3], pv[4][3], wv[FORM ? 4 : 1];
    __device__ __forceinline__ void fetch(int slot, unsigned node) {
        if constexpr (FORM) wv[slot] = ld_at(winv, (I)node);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            rv[slot][c] = ld_at(r, (I)c * nn + node);  // r, or z when not FORM
            pv[slot][c] = ld_at(p, (I)c * nn + node);
        }
    }
    __device__ __forceinline__ T value(int slot, int c) const {
        if constexpr (FORM) return jacobi_z(rv[slot][c], wv[slot], ik[c]) + beta * pv[slot][c];
        else return rv[slot][c] + beta * pv[slot][c];
    }
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

// 3D: one block per march column and field.  M is the table of reduced element blocks
// (apply3_from_n).
template <typename T, typename TX = T, typename TY = T>
__global__ __launch_bounds__(kBlock) void k_apply3(Grid g, const T* __restrict__ alpha, long long astride,
                                                   long long vstride, const T* __restrict__ M,
                                                   const uint8_t* __restrict__ mask,
                                                   const TX* __restrict__ x, TY* __restrict__ y) {
    __shared__ MarchLds<T> L;
    const FieldBlock fb = field_block();
    const size_t b = fb.field;
    const MarchBlock m = march3_block(g, fb.blk);
    for (int i = threadIdx.x; i < kFacSize; i += blockDim.x) L.M[i] = M[i];
    const MarchSlots sl = march3_slots(g, m);
    SrcMasked<T, TX> src{x + b * vstride, mask, g.n_nodes};
    march3_prologue(g, m, sl, src);
    TY* yb = y + b * vstride;
    auto emit = [&](int n, const T (&out)[3], const T (&)[3]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t idx = (size_t)c * g.n_nodes + n;
            yb[idx] = mask[idx] ? TY(0) : (TY)out[c];
        }
    };
    march3_run(g, m, sl, alpha + b * astride, L, src, emit);
}

// ----------------------------------------------------------------------------------
// Jacobi-PCG, two kernels per iteration (3D solves, and 2D solves in float32):
//   k_pcg_apply (iteration it): beta = rz_it / rz_{it-1}; p_new = z + beta p_old fused
//                 into the stencil; q = K p_new; pq partials.  Also the stopping test
//                 on rr = ||r_it||^2.
//   k_pcg_update(iteration it): alpha = rz_it / pq; x += alpha p, r -= alpha q,
//                 z = D^{-1} r; rz / rr partials of the next iteration.
// Partials of a field: [pq | rz(parity 0) | rz(parity 1) | rr(parity 0) | rr(parity 1)],
// ps doubles apart; the apply writes one pq partial per stencil block (napp), the start
// and the update one rz / rr partial per node-linear block (nupd).  Iteration it of a
// field writes rz/rr into parity it & 1 and reads the current ones from parity
// (it + 1) & 1.  The apply of iteration it records its summed rz_it in the state by
// parity (rz[it & 1]): the update of the same iteration and the next apply read it
// there instead of summing its partials again.  The logical block 0 of a field alone
// writes its state record (done flag, iteration count, norms, rz).
//
// Parity: launches carry a launch parity lp (alternating); a field's iteration parity
// is lp ^ poff, poff being fixed by the host when the field's segment starts, so that
// fields at different iteration counts run in the same launches.
// ----------------------------------------------------------------------------------
struct PcgState {
    double bb;    // reference ||r||^2 of the stopping test (set by the first apply of a
                  // fresh segment, or by the host when a segment continues after a
                  // residual replacement)
    double rr;    // ||r||^2 at the last stopping test
    double tol2;  // the segment stops when rr <= tol2 * bb
    double rz[2]; // summed r.z of the last two applies, by iteration parity
    int done;     // 0 running, 1 converged, 2 iteration limit, 3 breakdown, 4 idle
    int iters;    // completed iterations of the recursion (since its last fresh start)
    int maxit;
    int poff;     // iteration parity = launch parity ^ poff
    int qoff;     // 3D: iteration phase (mod 8) = (launch index + qoff) mod 8
    int fresh;    // the recursion starts here: the first apply records bb, beta = 0
    int it0;      // iterations at the segment's start
    double alpha[8];  // alpha of the last updates of a correction group, by iteration
                      // phase (mod the group size)
};

// Steps the float64 correction x takes at once (a group), and with it the ring of search
// directions p_i (in slot i mod G) that the apply writes and the update reads: 2 in 2D
// (p0, p1), 8 in 3D (p0..p7).  x += sum of alpha_j p_{j+1} over the group's updates j, at
// the group's last update; the earlier ones only record alpha_j.
constexpr int kRing3 = 8;
template <int DIM>
struct XGroup {
    static constexpr int value = DIM == 3 ? kRing3 : 2;
};

template <typename T>
struct PRing {
    T* s[kRing3];
};

constexpr int kPcgParts = 8;  // partial arrays per field (5 used by the two-kernel
                              // recursion, 8 by the one-reduction recursion)

__device__ __forceinline__ double* part_rz(double* p, int ps, int parity) { return p + (1 + parity) * ps; }
__device__ __forceinline__ double* part_rr(double* p, int ps, int parity) { return p + (3 + parity) * ps; }

// Block size of the node-linear PCG kernels and of the 2D apply: fewer, larger blocks
// leave fewer partial sums for the next kernel's prologue (measured at 241k DOF: 8 %
// shorter kernels than with 256 threads; 1024 threads were slower again).
constexpr int kPcgBlock = 512;

// Start of a segment of a field's recursion (one node per thread, grid (nupd, B)):
// r = scale * r64 (the float64 true residual, scaled), z = D^{-1} r, x = 0, and the
// rz / rr partials into the parity the segment's first apply reads.  A fresh start
// also clears p (its first apply takes beta = 0); a continued one keeps the search
// direction, so the Krylov progress of the earlier segments is not lost.  Only fields
// with a nonzero scale fsc[b] start a segment; the others are left as they are.
template <int DIM, typename T>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_start(Grid g, const double* __restrict__ r64,
                                                      const double* __restrict__ fsc,
                                                      const T* __restrict__ winv, T ik0, T ik1,
                                                      T ik2, double* __restrict__ x, T* __restrict__ r,
                                                      T* __restrict__ z, T* __restrict__ p0,
                                                      double* __restrict__ part, const PcgState* st,
                                                      int ps) {
    const int f = blockIdx.y;
    const PcgState* sb = st + f;
    if (fsc[f] == 0.0) return;  // field not starting a segment now
    __shared__ double lds[32];
    const size_t fo = (size_t)f * g.n_dofs;
    r64 += fo;
    x += fo;
    r += fo;
    z += fo;
    p0 += fo;
    winv += (size_t)f * g.n_nodes;
    const double scale = fsc[f];
    const bool fresh = sb->fresh != 0;
    const int cur = (sb->iters + 1) & 1;
    double v[2] = {0.0, 0.0};
    const T ik[3] = {ik0, ik1, ik2};
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n < g.n_nodes) {
        const T w = winv[n];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const size_t i = (size_t)c * g.n_nodes + n;
            const T ri = (T)(scale * r64[i]);
            const T zi = jacobi_z(ri, w, ik[c]);
            x[i] = 0.0;
            r[i] = ri;
            if (DIM == 2 || !ApplyFormsZ<T>::value) z[i] = zi;  // else the 3D apply forms z
            if (fresh) p0[i] = T(0);
            v[0] += (double)ri * (double)zi;
            v[1] += (double)ri * (double)ri;
        }
    }
    block_reduce<2>(v, lds);
    if (threadIdx.x == 0) {
        double* pb = part + (size_t)f * kPcgParts * ps;
        part_rz(pb, ps, cur)[blockIdx.x] = v[0];
        part_rr(pb, ps, cur)[blockIdx.x] = v[1];
    }
}

// Stopping test and CG coefficient of an apply, from the update partials (every block
// of the field computes the same values).  Returns the done code; tb is beta.
template <typename T>
__device__ __forceinline__ int pcg_apply_scalars(const double* part, PcgState* st, int ps, int nupd,
                                                 int parity, bool lead, T& tb, double* lds) {
    const int cur = (parity + 1) & 1;
    const int first = st->fresh != 0 && st->iters == 0;
    // rr and rz of the current residual (one pass); rz of the previous apply from the state
    const double* arrs[2] = {part + (3 + cur) * ps, part + (1 + cur) * ps};
    double red[2];
    block_sum_arrays<2>(arrs, nupd, red, lds);
    const double rr = red[0];
    const double bb = first ? rr : st->bb;
    int code = 0;
    if (!isfinite(rr)) code = 3;
    else if (rr <= st->tol2 * bb) code = 1;
    else if (st->iters >= st->maxit) code = 2;
    if (lead && threadIdx.x == 0) {
        if (first) st->bb = rr;
        st->rr = rr;
        if (code) st->done = code;
        else st->rz[parity] = red[1];
    }
    tb = first ? T(0) : (T)(red[1] / st->rz[cur]);
    return code;
}

// 2D: one node per thread (the launch covers every node of every field).  The node's
// loads are issued before it waits on the scalar reduction.  I: index type of the
// neighbourhood loads (32-bit when the per-field arrays fit, narrow2).
template <typename T, typename I>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_apply2(Grid g, const T* __restrict__ alpha,
                                                       const T* __restrict__ K,
                                                       const uint8_t* __restrict__ mask,
                                                       const T* __restrict__ z, T* __restrict__ p0,
                                                       T* __restrict__ p1, T* __restrict__ q,
                                                       double* __restrict__ part, PcgState* st,
                                                       int ps, int nupd, int lp) {
    const FieldBlock fb = field_block();
    PcgState* sb = st + fb.field;
    if (sb->done) return;
    __shared__ double lds[48];
    const int parity = lp ^ sb->poff;
    const size_t fo = (size_t)fb.field * g.n_dofs;
    alpha += (size_t)fb.field * g.n_elems;
    z += fo;
    const T* p_old = (parity ? p1 : p0) + fo;
    T* p_new = (parity ? p0 : p1) + fo;
    q += fo;
    double* pb = part + (size_t)fb.field * kPcgParts * ps;
    const int n = fb.blk * blockDim.x + threadIdx.x;
    const bool own = n < g.n_nodes;
    T zs[3][3][2], ps_[3][3][2], al[2][2];
    uint8_t mk[2];
    if (own) {
        int i, j, k;
        node_ijk(g, n, i, j, k);
        load_nbhd2(g, i, j, FetchPlain<T, I>{z, g.n_nodes}, zs);
        load_nbhd2(g, i, j, FetchPlain<T, I>{p_old, g.n_nodes}, ps_);
        load_alpha2<T, I>(g, i, j, alpha, al);
#pragma unroll
        for (int c = 0; c < 2; ++c) mk[c] = mask[(size_t)c * g.n_nodes + n];
    }
    T tb;
    if (pcg_apply_scalars(pb, sb, ps, nupd, parity, fb.blk == 0, tb, lds)) return;
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
    if (threadIdx.x == 0) pb[fb.blk] = v[0];
}

// Emitter of the 3D PCG apply (once3_run): at each node slot of a plane the block
// writes p_new and its part of q when it is the node's primary block, else its part
// into the side section the node belongs to for this block.  The parts are not masked:
// p_new is zero at masked DOFs (so is r, hence z), so their products with p_new add
// nothing, and the update zeroes q there.  pq sums p_new . part over every part written.
template <typename T, typename I>
struct PcgEmit3 {
    const Grid& g;
    const OnceBlock& m;
    const MarchSlots& sl;
    const SideGeom& sg;
    const OnceLds<T>& L;
    T* __restrict__ p_new;
    T* __restrict__ q;
    T* __restrict__ side;
    using SInfo = typename std::conditional<sizeof(I) == 4, int, long long>::type;
    SInfo sinfo[2];  // side section of the slot on the planes below the chunk's top (bits
                     // 0-1, 0: primary) and its side index at plane 0 (bits 2-)
    double pq = 0.0;

    __device__ __forceinline__ PcgEmit3(const Grid& g_, const OnceBlock& m_, const MarchSlots& sl_,
                                        const SideGeom& sg_, const OnceLds<T>& L_, T* p_new_, T* q_, T* side_)
        : g(g_), m(m_), sl(sl_), sg(sg_), L(L_), p_new(p_new_), q(q_), side(side_) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int qs = threadIdx.x + r * kBlock;
            const int s = sl.base[r] >= 0 ? once3_section(g, m, qs, 0) : 0;  // no z bit below the top
            const int i = m.ex0 + qs % MPX, j = m.ey0 + qs / MPX;
            sinfo[r] = s | (s ? (SInfo)side_index(sg, s, i, j, 0) << 2 : 0);
        }
    }
    template <bool TOP>
    __device__ __forceinline__ void emit(int r, int k, int buf, const T (&y)[3]) {
        const int qs = threadIdx.x + r * kBlock;
        const int n = sl.base[r] + k * sl.pstride;
        // sections 1-3 advance by one x-y layer of the section per plane
        int s = (int)(sinfo[r] & 3);
        const SInfo sstr = s == 1 ? sg.nbx * sg.nny : s == 2 ? sg.nnx * sg.nby : sg.nbx * sg.nby;
        SInfo si = (sinfo[r] >> 2) + k * sstr;
        if (TOP && k < g.nz) {  // the chunk's top plane: the block above is primary
            s = once3_section(g, m, qs, k);
            si = (SInfo)side_index(sg, s, m.ex0 + qs % MPX, m.ey0 + qs / MPX, k);
        }
        T d = T(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T pn = L.plane[buf][c][qs];
            // separate stores (not one through a selected pointer) keep each base uniform
            if (s) {
                st_at(side, (I)si + (I)c * (I)sg.total, y[c]);
            } else {
                st_at(q, (I)n + (I)c * (I)g.n_nodes, y[c]);
                st_at(p_new, (I)n + (I)c * (I)g.n_nodes, pn);
            }
            d += pn * y[c];
        }
        pq += (double)d;
    }
};

// 3D: one block per element tile and field, each element evaluated once (once3_run).
// The first two node planes of z and p_old are fetched before the scalar reduction;
// p_new = z + beta p_old is formed per node as the planes are staged.  The block writes
// p_new and its part of q = K p_new at the nodes it is primary for, and its part at the
// other nodes of its tile into the side sections (side [B][3][total]); the update adds
// them.  The pq partial sums p_new . part over every part the block writes, which adds
// up to p_new . q over the blocks.  Mv: the reduced element blocks (apply3_from_n);
// I: index type of the per-field arrays (32-bit when their bytes fit).
template <typename T, typename I>
__global__ __launch_bounds__(kBlock, sizeof(T) == 4 ? 4 : 2) void k_pcg_apply3(Grid g, const T* __restrict__ alpha,
                                                       const FacTab<T> Mv,
                                                       const T* __restrict__ r /* z when float64 */,
                                                       const T* __restrict__ winv,
                                                       T ik0, T ik1, T ik2, const PRing<T> pr,
                                                       T* __restrict__ q,
                                                       T* __restrict__ side, const SideGeom sg,
                                                       double* __restrict__ part, PcgState* st, int ps,
                                                       int nrz, int lq) {
    const FieldBlock fb = field_block();
    PcgState* sb = st + fb.field;
    if (sb->done) return;
    __shared__ OnceLds<T> L;
    __shared__ double lds[48];
    const int phase = (lq + sb->qoff) & (kRing3 - 1);  // iteration mod 8: p_i in slot phase
    const int parity = phase & 1;
    const size_t fo = (size_t)fb.field * g.n_dofs;
    alpha += (size_t)fb.field * g.n_elems;
    r += fo;
    winv += (size_t)fb.field * g.n_nodes;
    const T* p_old = pr.s[phase] + fo;
    T* p_new = pr.s[(phase + 1) & (kRing3 - 1)] + fo;
    q += fo;
    side += (size_t)fb.field * 3 * sg.total;
    double* pb = part + (size_t)fb.field * kPcgParts * ps;
    const OnceBlock m = once3_block(g, fb.blk);
    const MarchSlots sl = once3_slots(g, m);
    SrcDirection3<T, I> src{r, winv, p_old, {ik0, ik1, ik2}, T(0), (unsigned)g.n_nodes};
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        src.fetch(r, once3_node(sl, r, m.ez0));
        src.fetch(2 + r, once3_node(sl, r, m.ez0 + 1));
    }
    PcgEmit3<T, I> E(g, m, sl, sg, L, p_new, q, side);
    T tb;
    if (pcg_apply_scalars(pb, sb, ps, nrz, parity, fb.blk == 0, tb, lds)) return;
    src.beta = tb;
    once3_run(g, m, sl, alpha, L, src, E, Mv.m);
    double v[1] = {E.pq};
    block_reduce<1>(v, lds);
    if (threadIdx.x == 0) pb[fb.blk] = v[0];
}

// One node per thread (grid (nupd, B)); the node's loads are issued before the wait on
// the scalar reduction.  3D: q is zeroed at masked DOFs here (the 3D apply writes
// unmasked parts), so that r stays zero there, from the node's mask bits (mask: [N_n],
// bit c for component c, k_node_mask); the 2D apply masks q itself (mask unused).
// I: index type of the per-field arrays (32-bit when their bytes fit, update_narrow);
// NPT: nodes per thread (grid (nupd of NPT kPcgBlock nodes, B)).
template <int DIM, typename T, bool FLUSH, typename I, int NPT>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_update(Grid g, const T* __restrict__ winv,
                                                       const uint8_t* __restrict__ mask,
                                                       T ik0, T ik1, T ik2, double* __restrict__ x,
                                                       T* __restrict__ r, T* __restrict__ z,
                                                       const PRing<T> pr,
                                                       const T* __restrict__ q,
                                                       const T* __restrict__ side, const SideGeom sg,
                                                       double* __restrict__ part, PcgState* st,
                                                       int ps, int npq, int lq) {
    constexpr int G = XGroup<DIM>::value;
    const int f = blockIdx.y;
    PcgState* sb = st + f;
    if (sb->done) return;
    __shared__ double lds[32];
    // iteration i mod G (3D: from the launch index mod 8; 2D: the parity)
    const int phase = G == kRing3 ? ((lq + sb->qoff) & (kRing3 - 1)) : ((lq ^ sb->poff) & 1);
    const int parity = phase & 1;
    const size_t fo = (size_t)f * g.n_dofs;
    winv += (size_t)f * g.n_nodes;
    x += fo;
    r += fo;
    if (z) z += fo;
    const T* p = pr.s[(phase + 1) & (G - 1)] + fo;  // the apply's p_new
    q += fo;
    double* pb = part + (size_t)f * kPcgParts * ps;
    // the correction x takes G steps at once, at the group's last update (the earlier ones
    // only record their alpha): the directions of the group's earlier updates are older
    // slots of the ring.  Segments start at launch 1 of a chunk and chunks hold a multiple
    // of G launches, so every field's groups end together, at the launches whose index
    // is a multiple of G: those run this kernel with FLUSH.  A thread takes NPT nodes,
    // kPcgBlock apart (NPT > 1 only without FLUSH: more loads in flight per thread).
    constexpr bool flush = FLUSH;
    static_assert(NPT == 1 || !FLUSH, "the correction update takes one node per thread");
    const int n0 = blockIdx.x * blockDim.x * NPT + threadIdx.x;
    double xv[NPT][DIM];
    T rv[NPT][DIM], pv[NPT][DIM], ppv[G - 1][DIM], qv[NPT][DIM], w[NPT];
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        const int n = n0 + u * kPcgBlock;
        w[u] = T(0);
        if (n >= g.n_nodes) continue;
        w[u] = ld_at(winv, (I)n);
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const I i = (I)c * (I)g.n_nodes + (I)n;
            if (flush) {
                xv[u][c] = ld_at(x, i);
#pragma unroll
                for (int j = 1; j < G; ++j) ppv[j - 1][c] = ld_at(pr.s[(phase + 1 - j) & (G - 1)] + fo, i);
            }
            rv[u][c] = ld_at((const T*)r, i);
            pv[u][c] = ld_at(p, i);
            qv[u][c] = ld_at(q, i);
        }
        if constexpr (DIM == 3) {
            const unsigned mk = ld_at(mask, (I)n);
            // q = the primary block's part + the parts of the blocks below the node, in
            // the order of their side sections
            const unsigned jk = sg.dnx.div((unsigned)n), kk = sg.dny.div(jk);
            const int i = n - (int)jk * g.nx1, j = (int)(jk - kk * (unsigned)g.ny1), k = (int)kk;
            const int ax = side_axes(g, sg, i, j, k);
            if (ax) {
                const T* sf = side + (size_t)f * 3 * sg.total;
                for (int sec = 1; sec < 8; ++sec)
                    if ((sec & ax) == sec) {
                        const I si = (I)side_index(sg, sec, i, j, k);
#pragma unroll
                        for (int c = 0; c < 3; ++c) qv[u][c] += ld_at(sf, (I)c * (I)sg.total + si);
                    }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if ((mk >> c) & 1u) qv[u][c] = T(0);
        }
    }
    const double pq = block_sum_array(pb, npq, lds);
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) sb->done = 3;
        return;
    }
    const T a = (T)(sb->rz[parity] / pq);
    double ao[G - 1];  // alpha of the group's earlier updates (j steps back)
#pragma unroll
    for (int j = 1; j < G; ++j) ao[j - 1] = flush ? sb->alpha[(phase - j) & (G - 1)] : 0.0;
    (void)ao;
    const T ik[3] = {ik0, ik1, ik2};
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int u = 0; u < NPT; ++u) {
        const int n = n0 + u * kPcgBlock;
        if (n >= g.n_nodes) continue;
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            const I i = (I)c * (I)g.n_nodes + (I)n;
            if (flush) {
                // pairs of steps summed from the oldest pair to the newest
                double s = G > 2 ? ao[G - 2] * (double)ppv[G - 2][c] + ao[G - 3] * (double)ppv[G - 3][c]
                                 : ao[0] * (double)ppv[0][c] + (double)a * (double)pv[u][c];
#pragma unroll
                for (int k = G / 2 - 2; k >= 1; --k)
                    s += ao[2 * k] * (double)ppv[2 * k][c] + ao[2 * k - 1] * (double)ppv[2 * k - 1][c];
                if constexpr (G > 2) s += ao[0] * (double)ppv[0][c] + (double)a * (double)pv[u][c];
                st_at(x, i, xv[u][c] + s);
            }
            const T ri = rv[u][c] - a * qv[u][c];
            const T zi = jacobi_z(ri, w[u], ik[c]);
            st_at(r, i, ri);
            if (DIM == 2 || !ApplyFormsZ<T>::value) st_at(z, i, zi);  // else the 3D apply forms z
            v[0] += (double)ri * (double)zi;
            v[1] += (double)ri * (double)ri;
        }
    }
    block_reduce<2>(v, lds);
    if (threadIdx.x == 0) {
        part_rz(pb, ps, parity)[blockIdx.x] = v[0];
        part_rr(pb, ps, parity)[blockIdx.x] = v[1];
        if (blockIdx.x == 0) {
            sb->alpha[phase] = (double)a;
            sb->iters = sb->iters + 1;
        }
    }
}

// In-place fixed-order sum of the per-block partials of large launches, one block per
// field: A[0] = sum of A[0..n), and likewise B when sb >= 0.  Array X sits at slot
// sx (+ the field's iteration parity when px, that parity being lp ^ poff ^ flip) of
// the field's partials.  The consumer then reads 1 value instead of every block summing
// all partials again.  Skipped once the field's recursion is done (its producer did
// not run then, and summing again would count A[0] twice), or, with a gate (the
// segment starts), for the fields whose gate entry is zero.
template <typename S>
__global__ __launch_bounds__(1024) void k_partials_sum(double* __restrict__ part, int ps, int n, int sa,
                                                       int pa, int sb, int pb, const S* st, int lp,
                                                       int flip, const double* gate) {
    const int f = blockIdx.x;
    if (gate ? gate[f] == 0.0 : st[f].done != 0) return;
    __shared__ double lds[32];
    const int par = lp ^ st[f].poff ^ flip;
    double* base = part + (size_t)f * kPcgParts * ps;
    double* a = base + (size_t)(sa + (pa ? par : 0)) * ps;
    double* b = sb >= 0 ? base + (size_t)(sb + (pb ? par : 0)) * ps : nullptr;
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
// Partials of a field: [gamma(0) | gamma(1) | delta(0) | delta(1) | rr(0) | rr(1) | u.s |
// p.s], ps doubles apart, by the parity of the residual they belong to.  The state keeps
// gamma, alpha and the iteration count by parity: step i reads the slots of step i - 1
// and writes its own, so no block reads a value another block of its launch writes.
// ----------------------------------------------------------------------------------
struct Cg1State {
    double bb;        // reference ||r||^2 of the stopping test
    double rr;        // ||r||^2 at the last stopping test
    double tol2;      // the segment stops when rr <= tol2 * bb
    double gamma[2];  // gamma_i by parity of i
    double alpha[2];  // alpha_i by parity of i
    int done;         // 0 running, 1 converged, 2 iteration limit, 3 breakdown, 4 idle
    int maxit;
    int iters[2];     // step i writes iters[i & 1] = i + 1
    int poff;         // iteration parity = launch parity ^ poff
    int kind0;        // kind of the segment's first step (kCg1Fresh / kCg1Continued)
    int it0;          // iteration count at the segment's start
    int pad;
};

enum { kCg1Step = 0, kCg1Fresh = 1, kCg1Continued = 2 };

__device__ __forceinline__ double* cg1_part(double* p, int ps, int k) { return p + (size_t)k * ps; }

// Node value of a per-node array on the 3x3 neighbourhood (zero outside the grid).
template <typename T, typename I = size_t>
__device__ __forceinline__ void load_node_nbhd2(const Grid& g, int i, int j, const T* __restrict__ a,
                                                T (&v)[3][3]) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int ii = i + dx - 1, jj = j + dy - 1;
            const bool ok = (ii >= 0) & (ii < g.nx1) & (jj >= 0) & (jj < g.ny1);
            v[dy][dx] = ok ? ld_at(a, (I)(jj * g.nx1 + ii)) : T(0);
        }
}

// One step of every running field.  The first step of a segment is fresh (beta = 0) or
// continued (after a residual replacement: the direction K-conjugate to the kept p,
// with the exact p^T K p, from the u.s / p.s partials of k_cg1_start2); the kind is
// read from the field's state.  I: index type of the neighbourhood loads (narrow2).
template <typename T, typename I>
__global__ __launch_bounds__(kPcgBlock) void k_cg1_step2(
    Grid g, const T* __restrict__ alpha, const T* __restrict__ K, const uint8_t* __restrict__ mask,
    const T* __restrict__ winv, T ik0, T ik1, T* __restrict__ R0, T* __restrict__ R1, T* __restrict__ W0,
    T* __restrict__ W1, T* __restrict__ S0, T* __restrict__ S1, T* __restrict__ P, double* __restrict__ x,
    double* __restrict__ part, Cg1State* st, int ps, int npart, int lp) {
    const FieldBlock fb = field_block();
    Cg1State* sb = st + fb.field;
    if (sb->done) return;
    __shared__ double lds[80];
    const int cur = lp ^ sb->poff, nxt = cur ^ 1;
    const int kind = sb->iters[nxt] == sb->it0 ? sb->kind0 : kCg1Step;
    const size_t fo = (size_t)fb.field * g.n_dofs;
    alpha += (size_t)fb.field * g.n_elems;
    winv += (size_t)fb.field * g.n_nodes;
    const T* Rin = (cur ? R1 : R0) + fo;
    const T* Win = (cur ? W1 : W0) + fo;
    const T* Sin = (cur ? S1 : S0) + fo;
    T* Rout = (nxt ? R1 : R0) + fo;
    T* Wout = (nxt ? W1 : W0) + fo;
    T* Sout = (nxt ? S1 : S0) + fo;
    P += fo;
    x += fo;
    double* pb = part + (size_t)fb.field * kPcgParts * ps;
    const int n = fb.blk * blockDim.x + threadIdx.x;
    const bool own = n < g.n_nodes;
    T rs[3][3][2], ws[3][3][2], ss[3][3][2], wv[3][3], al[2][2], pv[2];
    double xv[2];
    uint8_t mk[2];
    int i = 0, j = 0, k = 0;
    if (own) {  // every load is issued before the wait on the scalar reduction
        node_ijk(g, n, i, j, k);
        load_nbhd2(g, i, j, FetchPlain<T, I>{Rin, g.n_nodes}, rs);
        load_nbhd2(g, i, j, FetchPlain<T, I>{Win, g.n_nodes}, ws);
        load_nbhd2(g, i, j, FetchPlain<T, I>{Sin, g.n_nodes}, ss);
        load_node_nbhd2<T, I>(g, i, j, winv, wv);
        load_alpha2<T, I>(g, i, j, alpha, al);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t idx = (size_t)c * g.n_nodes + n;
            mk[c] = mask[idx];
            pv[c] = P[idx];
            xv[c] = x[idx];
        }
    }
    double be = 0.0, ah = 0.0;
    {
        double red[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (kind == kCg1Continued) {
            const double* arrs[5] = {cg1_part(pb, ps, cur), cg1_part(pb, ps, 2 + cur),
                                     cg1_part(pb, ps, 4 + cur), cg1_part(pb, ps, 6), cg1_part(pb, ps, 7)};
            block_sum_arrays<5>(arrs, npart, red, lds);
        } else {
            const double* arrs[3] = {cg1_part(pb, ps, cur), cg1_part(pb, ps, 2 + cur),
                                     cg1_part(pb, ps, 4 + cur)};
            double r3[3];
            block_sum_arrays<3>(arrs, npart, r3, lds);
            red[0] = r3[0];
            red[1] = r3[1];
            red[2] = r3[2];
        }
        const double gam = red[0], dlt = red[1], rr = red[2];
        const double bb = kind == kCg1Fresh ? rr : sb->bb;
        int code = 0;
        if (!isfinite(rr)) code = 3;
        else if (rr <= sb->tol2 * bb) code = 1;
        else if (sb->iters[nxt] >= sb->maxit) code = 2;
        if (!code) {
            if (kind == kCg1Fresh) {
                ah = gam / dlt;
            } else if (kind == kCg1Continued) {
                const double us = red[3], pss = red[4];
                if (pss > 0.0 && isfinite(pss)) {
                    be = -us / pss;
                    ah = gam / (dlt + be * us);
                } else {
                    ah = gam / dlt;
                }
            } else {
                be = gam / sb->gamma[nxt];
                ah = gam / (dlt - be * gam / sb->alpha[nxt]);
            }
            if (!(ah > 0.0) || !isfinite(ah) || !isfinite(be)) code = 3;
        }
        if (fb.blk == 0 && threadIdx.x == 0) {
            if (kind == kCg1Fresh) sb->bb = rr;
            sb->rr = rr;
            if (code) {
                sb->done = code;
            } else {
                sb->gamma[cur] = gam;
                sb->alpha[cur] = ah;
                sb->iters[cur] = sb->iters[nxt] + 1;
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
                    const T si = ws[dy][dx][c] + tb * ss[dy][dx][c];
                    const T rn = rs[dy][dx][c] - ta * si;
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
            const T pn = rs[1][1][c] * wv[1][1] * ik[c] + tb * pv[c];  // u_i + beta p_{i-1}
            P[idx] = pn;
            x[idx] = xv[c] + (double)ta * (double)pn;
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
        cg1_part(pb, ps, nxt)[fb.blk] = v[0];
        cg1_part(pb, ps, 2 + nxt)[fb.blk] = v[1];
        cg1_part(pb, ps, 4 + nxt)[fb.blk] = v[2];
    }
}

// s = K p recomputed for the direction of the step launched at parity lp, into the set
// that step wrote.  The recursion s_i = w_i + beta_i s_{i-1} carries each rounding of
// K u through about 1 / (1 - beta) iterations (beta ~ 0.98 here), which would let the
// recursive residual drift from the true one; refreshing s every kCg1Refresh iterations
// bounds that sum.  Reads p (neighbourhood) only and writes s (own node).
template <typename T>
__global__ __launch_bounds__(kPcgBlock) void k_cg1_refresh2(Grid g, const T* __restrict__ alpha,
                                                         const T* __restrict__ K,
                                                         const uint8_t* __restrict__ mask,
                                                         const T* __restrict__ P, T* __restrict__ S0,
                                                         T* __restrict__ S1, const Cg1State* st, int lp) {
    const FieldBlock fb = field_block();
    const Cg1State* sb = st + fb.field;
    if (sb->done) return;
    const int n = fb.blk * blockDim.x + threadIdx.x;
    if (n >= g.n_nodes) return;
    const int nxt = lp ^ sb->poff ^ 1;
    const size_t fo = (size_t)fb.field * g.n_dofs;
    P += fo;
    T* S = (nxt ? S1 : S0) + fo;
    alpha += (size_t)fb.field * g.n_elems;
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

// Start of a segment of the one-reduction recursion, written to set it0 & 1 with x = 0:
// r = scale * r64 (the float64 true residual, scaled), u = D^{-1} r, w = K u, and the
// partials of gamma, delta, rr.  A fresh start clears p and s (its first step takes
// beta = 0); a continued one computes s = K p exactly for the kept direction p and the
// partials of u.s, p.s, from which its first step takes the conjugate direction.
// Only fields with a nonzero scale fsc[b] start a segment.
template <typename T>
__global__ __launch_bounds__(kPcgBlock) void k_cg1_start2(
    Grid g, const T* __restrict__ alpha, const T* __restrict__ K, const uint8_t* __restrict__ mask,
    const T* __restrict__ winv, T ik0, T ik1, const double* __restrict__ r64, const double* __restrict__ fsc,
    T* __restrict__ P, T* __restrict__ R0, T* __restrict__ R1, T* __restrict__ W0, T* __restrict__ W1,
    T* __restrict__ S0, T* __restrict__ S1, double* __restrict__ x, double* __restrict__ part,
    const Cg1State* st, int ps) {
    const FieldBlock fb = field_block();
    const Cg1State* sb = st + fb.field;
    if (fsc[fb.field] == 0.0) return;  // field not starting a segment now
    __shared__ double lds[80];
    const int cur = sb->it0 & 1;
    const bool fresh = sb->kind0 == kCg1Fresh;
    const double scale = fsc[fb.field];
    const size_t fo = (size_t)fb.field * g.n_dofs;
    alpha += (size_t)fb.field * g.n_elems;
    winv += (size_t)fb.field * g.n_nodes;
    r64 += fo;
    P += fo;
    x += fo;
    T* R = (cur ? R1 : R0) + fo;
    T* W = (cur ? W1 : W0) + fo;
    T* S = (cur ? S1 : S0) + fo;
    double* pb = part + (size_t)fb.field * kPcgParts * ps;
    const int n = fb.blk * blockDim.x + threadIdx.x;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (n < g.n_nodes) {
        int i, j, k;
        node_ijk(g, n, i, j, k);
        double rs[3][3][2];
        T ps_[3][3][2], wv[3][3], al[2][2];
        load_nbhd2(g, i, j, FetchPlain<double>{r64, g.n_nodes}, rs);
        if (!fresh) load_nbhd2(g, i, j, FetchPlain<T>{P, g.n_nodes}, ps_);
        load_node_nbhd2(g, i, j, winv, wv);
        load_alpha2(g, i, j, alpha, al);
        const T ik[2] = {ik0, ik1};
        T un[3][3][2], rown[2], uown[2], pown[2] = {T(0), T(0)};
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
                        if (!fresh) pown[c] = ps_[1][1][c];
                    }
                }
        T wo[2], so[2] = {T(0), T(0)};
        apply_nbhd2(K, un, al, wo);
        if (!fresh) apply_nbhd2(K, ps_, al, so);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const size_t idx = (size_t)c * g.n_nodes + n;
            const bool fixed = mask[idx] != 0;
            const T wn = fixed ? T(0) : wo[c];
            const T sn = fixed ? T(0) : so[c];
            R[idx] = rown[c];
            W[idx] = wn;
            S[idx] = sn;
            if (fresh) P[idx] = T(0);
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
        cg1_part(pb, ps, cur)[fb.blk] = v[0];
        cg1_part(pb, ps, 2 + cur)[fb.blk] = v[1];
        cg1_part(pb, ps, 4 + cur)[fb.blk] = v[2];
        cg1_part(pb, ps, 6)[fb.blk] = v[3];
        cg1_part(pb, ps, 7)[fb.blk] = v[4];
    }
}

// u_b += s_b * d_b for the fields with s_b != 0 (grid (blocks, B), grid-stride)
template <typename T>
__global__ void k_correct(long long n, double* __restrict__ u, const T* __restrict__ d,
                          const double* __restrict__ s) {
    const int f = blockIdx.y;
    const double sf = s[f];
    if (sf == 0.0) return;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        u[(size_t)f * n + i] += sf * (double)d[(size_t)f * n + i];
}

// u += s * x for the two-kernel recursion, whose x lacks the last m = (iters - it0) mod G
// steps when the segment's updates ended inside a correction group (x takes G steps at a
// time): those steps are added here from the state (alpha by iteration phase) and the
// ring of directions (p_{j+1} of update j in slot (j + 1) mod G).
template <typename T, int G>
__global__ void k_correct_pcg(long long n, double* __restrict__ u, const double* __restrict__ x,
                              const PRing<T> pr, const PcgState* __restrict__ st, const double* __restrict__ s) {
    const int f = blockIdx.y;
    const double sf = s[f];
    if (sf == 0.0) return;
    const PcgState& S = st[f];
    const int m = (S.iters - S.it0) & (G - 1);
    double a[G - 1];
    const T* pl[G - 1];
#pragma unroll
    for (int j = 0; j < G - 1; ++j) {  // update iters - 1 - j and its direction
        a[j] = j < m ? S.alpha[(S.iters - 1 - j) & (G - 1)] : 0.0;
        pl[j] = pr.s[(S.iters - j) & (G - 1)] + (size_t)f * n;
    }
    x += (size_t)f * n;
    u += (size_t)f * n;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        double add = 0.0;
        for (int j = m - 1; j >= 0; --j) add += a[j] * (double)pl[j][i];
        u[i] += sf * (m ? x[i] + add : x[i]);
    }
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
// float64 residual r = f - K u over free DOFs (u zero on Dirichlet DOFs), with
// per-block partials of ||r||^2, f^T u and u^T r for every field (f shared by the
// fields); k_residual_sum reduces them (one block per field) into out[4*b .. 4*b+2].
// Fields with skip[b] != 0 (skip may be NULL) are left out.
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
                                                  const FieldBlock& fb, double* lds) {
    block_reduce<3>(v, lds);
    const int nb = gridDim.x;
    double* pb = part + (size_t)fb.field * 3 * nb;
    if (threadIdx.x == 0) {
        pb[fb.blk] = v[0];
        pb[nb + fb.blk] = v[1];
        pb[2 * nb + fb.blk] = v[2];
    }
}

__global__ __launch_bounds__(kBlock) void k_residual2(Grid g, const double* __restrict__ alpha,
                                                      const double* __restrict__ K,
                                                      const uint8_t* __restrict__ mask,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ f,
                                                      double* __restrict__ r,
                                                      double* __restrict__ part, const int* skip) {
    const FieldBlock fb = field_block();
    if (skip && skip[fb.field]) return;
    __shared__ double lds[48];
    const size_t b = fb.field;
    const int n = fb.blk * blockDim.x + threadIdx.x;
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
    residual_partials(v, part, fb, lds);
}

// 3D: one block per march column and field; M is the table of reduced element blocks.
__global__ __launch_bounds__(kBlock) void k_residual3(Grid g, const double* __restrict__ alpha,
                                                      const double* __restrict__ M,
                                                      const uint8_t* __restrict__ mask,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ f,
                                                      double* __restrict__ r,
                                                      double* __restrict__ part, const int* skip) {
    const FieldBlock fb = field_block();
    if (skip && skip[fb.field]) return;
    __shared__ MarchLds<double> L;
    __shared__ double lds[48];
    const size_t b = fb.field;
    const double* ub = u + b * g.n_dofs;
    const MarchBlock m = march3_block(g, fb.blk);
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
    residual_partials(v, part, fb, lds);
}

__global__ __launch_bounds__(kBlock) void k_residual_sum(int nb, const double* __restrict__ part,
                                                         double* __restrict__ out, const int* skip) {
    __shared__ double lds[16];
    const int b = blockIdx.x;
    if (skip && skip[b]) return;
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
        hipLaunchKernelGGL(k_winv, dim3(grid_blocks(g.n_nodes), B), dim3(kBlock), 0, s, g, a64, w64, w32);
        TOPO_CHECK_LAUNCH();
    }
    return TOPO_OK;
}

// Launch geometry of the PCG kernels: node-linear blocks for the start / update, stencil
// blocks for the apply, the stride of the partial arrays, and how many partials each
// consumer sums (1 when a launch has more blocks than kPcgMaxBlocks: its partials are
// then summed once by k_partials_sum).  The one-reduction step uses nupd / nrz.
// The plain 3D updates take this many nodes per thread: twice the loads in flight per
// wave (one node per thread left the plain update at 4.3 TB/s of measured traffic, the
// flush update, with four times the loads per thread, at 5.1 TB/s).
constexpr int kUpdateNpt = 2;

// The update of launch lq is the last of its correction group (FLUSH).
template <int DIM>
inline bool flush_of(int lq) {
    return (lq & (XGroup<DIM>::value - 1)) == 0;
}

struct PcgGeom {
    int nupd, napp, ps;
    int npq, nrz;  // partials read of the apply's pq and of the update's rz / rr
    int npt;         // nodes per thread of the plain 3D updates (kUpdateNpt or 1)
    int nupd_plain;  // their block count (and rz / rr partials)
};

static PcgGeom pcg_geom(const Grid& g) {
    PcgGeom pg;
    pg.nupd = grid_blocks(g.n_nodes, kPcgBlock);
    pg.napp = g.dim == 2 ? grid_blocks(g.n_nodes, kPcgBlock) : once3_blocks(g);
    pg.ps = std::max(pg.nupd, pg.napp);
    pg.npq = pg.napp > kPcgMaxBlocks ? 1 : pg.napp;
    pg.nrz = pg.nupd > kPcgMaxBlocks ? 1 : pg.nupd;
    // the plain 3D updates take kUpdateNpt nodes per thread when their partials go through
    // the summing kernel (which reads the count each launch wrote); otherwise the apply
    // reads nupd partials itself and every update writes that many
    pg.npt = g.dim == 3 && pg.nrz == 1 && pg.nupd > 1 ? kUpdateNpt : 1;
    pg.nupd_plain = grid_blocks(g.n_nodes, kPcgBlock * pg.npt);
    return pg;
}

// Device buffers of a batched solve.  The one-reduction recursion (2D float64) uses
// r, z as its residual sets, q, e0 as its w sets, p0, p1 as its s sets and e1 as p.
template <typename T>
struct PcgBufs {
    int B;
    const T* alpha;    // [B][N_e]
    const T* K;        // 2D: dense element matrix; 3D: reduced element blocks
    const uint8_t* mask;
    const uint8_t* mnode;  // 3D: mask bits per node
    const T* winv;     // [B][N_n]
    T ik[3];           // 1 / K_e[c][c]
    T *r, *z, *p0, *p1, *q, *e0, *e1;  // [B][N_u]
    T* pk[kRing3 - 2];  // 3D: the further slots of the ring of directions
    PRing<T> ring() const {
        PRing<T> r{};
        r.s[0] = p0;
        r.s[1] = p1;
        for (int k = 2; k < kRing3; ++k) r.s[k] = pk[k - 2];
        return r;
    }
    T* side;           // 3D: [B][3][side total] the apply's parts of shared nodes
    SideGeom sg;       // 3D: their sections (from the apply's launch geometry)
    FacTab<T> Mv;      // 3D: the reduced element blocks, passed by value
    bool narrow;       // 3D: the apply indexes its arrays with 32-bit offsets
    double* x;         // [B][N_u] the segment's correction, accumulated in float64
    double* part;      // [B][kPcgParts][ps]
    PcgState* st;      // [B]
    Cg1State* st1;     // [B]
    const double* r64; // [B][N_u] float64 true residual
    const double* fsc; // [B] scale of each field's inner system
};

// The float32 3D apply takes 32-bit indices when the bytes of every per-field array it
// reads or writes fit in 32 bits (below 4 GiB each); the float64 one 64-bit indices.
// The side sections hold under 4 N_n / 3 nodes for any chunk height (the z sections at
// most N_n, the x and y ones N_n / 32 and N_n / 8), so 2 N_n bounds them before the
// launch geometry is known.
template <typename T>
static bool apply3_narrow(const Grid& g) {
    const unsigned long long lim = 1ull << 32, nn = (unsigned long long)g.n_nodes;
    return sizeof(T) == 4 && 3ull * 2ull * nn * sizeof(T) < lim && (unsigned long long)g.n_elems * sizeof(T) < lim;
}

// The 2D stencil kernels take 32-bit neighbourhood indices when every per-field array
// they read fits in 4 GiB (DOF vectors up to float64, alpha per element).
static bool narrow2(const Grid& g) {
    const unsigned long long lim = 1ull << 32;
    return (unsigned long long)g.n_dofs * sizeof(double) < lim && (unsigned long long)g.n_elems * sizeof(double) < lim;
}

// The update takes 32-bit indices when each per-field array it touches fits in 4 GiB:
// the float64 correction x (the largest DOF array) and the side sections (2 N_n nodes
// bound them, as above).
template <typename T>
static bool update_narrow(const Grid& g) {
    const unsigned long long lim = 1ull << 32, nn = (unsigned long long)g.n_nodes;
    return (unsigned long long)g.n_dofs * sizeof(double) < lim && 3ull * 2ull * nn * sizeof(T) < lim;
}

// npt: nodes per thread of a plain (non-flush) update, 1 or kUpdateNpt.
template <int DIM, typename T>
static const void* pcg_update_fn(bool flush, bool narrow, int npt) {
    constexpr int W = kUpdateNpt;
    if (flush)
        return narrow ? (const void*)k_pcg_update<DIM, T, true, unsigned, 1>
                      : (const void*)k_pcg_update<DIM, T, true, size_t, 1>;
    if (npt == W)
        return narrow ? (const void*)k_pcg_update<DIM, T, false, unsigned, W>
                      : (const void*)k_pcg_update<DIM, T, false, size_t, W>;
    return narrow ? (const void*)k_pcg_update<DIM, T, false, unsigned, 1>
                  : (const void*)k_pcg_update<DIM, T, false, size_t, 1>;
}

template <typename T>
static const void* pcg_apply3_fn(bool narrow) {
    if constexpr (sizeof(T) == 4)
        if (narrow) return (const void*)k_pcg_apply3<T, unsigned>;
    return (const void*)k_pcg_apply3<T, size_t>;
}

// One iteration of the two-kernel recursion (apply + update) at launch index lq mod 8
// (launch parity lp = lq & 1).
template <int DIM, typename T>
static void pcg_iteration(Ctx* ctx, const Grid& g, const PcgBufs<T>& w, const PcgGeom& pg, int lq,
                          LaunchSink& L, int timing) {
    const int lp = lq & 1;
    {
        TimedLaunch tl(ctx, KID_PCG_APPLY, L.s, L.graph ? kTimeOff : timing, true);
        L.ev0 = tl.a;
        L.ev1 = tl.b;
        if constexpr (DIM == 2)
            L(narrow2(g) ? (const void*)k_pcg_apply2<T, unsigned> : (const void*)k_pcg_apply2<T, size_t>,
              dim3(pg.napp, w.B), dim3(kPcgBlock), g, w.alpha, w.K, w.mask,
              (const T*)w.z, w.p0, w.p1, w.q, w.part, w.st, pg.ps, pg.nrz, lp);
        else
            L(pcg_apply3_fn<T>(w.narrow), dim3(pg.napp, w.B), dim3(kBlock), g, w.alpha, w.Mv,
              (const T*)(ApplyFormsZ<T>::value ? w.r : w.z), w.winv, w.ik[0],
              w.ik[1], w.ik[2], w.ring(), w.q, w.side, w.sg, w.part, w.st, pg.ps, pg.nrz, lq);
    }
    if (pg.npq == 1 && pg.napp > 1)
        L((const void*)k_partials_sum<PcgState>, dim3(w.B), dim3(1024), w.part, pg.ps, pg.napp, 0, 0, -1, 0,
          (const PcgState*)w.st, lp, 0, (const double*)nullptr);
    {
        TimedLaunch tl(ctx, KID_PCG_UPDATE, L.s, L.graph ? kTimeOff : timing, true);
        L.ev0 = tl.a;
        L.ev1 = tl.b;
        const bool flush = flush_of<DIM>(lq);  // a group's last update
        L(pcg_update_fn<DIM, T>(flush, update_narrow<T>(g), flush ? 1 : pg.npt),
          dim3(flush ? pg.nupd : pg.nupd_plain, w.B), dim3(kPcgBlock), g, w.winv, DIM == 3 ? w.mnode : w.mask,
          w.ik[0], w.ik[1], w.ik[2], w.x, w.r, w.z,
          w.ring(), (const T*)w.q, (const T*)w.side, w.sg, w.part, w.st, pg.ps, pg.npq, lq);
    }
    if (pg.nrz == 1 && pg.nupd > 1)  // rz / rr of the update's own parity (its own block count)
        L((const void*)k_partials_sum<PcgState>, dim3(w.B), dim3(1024), w.part, pg.ps,
          flush_of<DIM>(lq) ? pg.nupd : pg.nupd_plain, 1, 1, 3, 1, (const PcgState*)w.st, lp, 0,
          (const double*)nullptr);
}

// One step of the one-reduction recursion at launch parity lp (then s = K p when refresh).
template <typename T>
static void cg1_step(Ctx* ctx, const Grid& g, const PcgBufs<T>& w, const PcgGeom& pg, int lp, LaunchSink& L,
                     int timing, bool refresh) {
    {
        TimedLaunch tl(ctx, KID_PCG_STEP, L.s, L.graph ? kTimeOff : timing, true);
        L.ev0 = tl.a;
        L.ev1 = tl.b;
        L(narrow2(g) ? (const void*)k_cg1_step2<T, unsigned> : (const void*)k_cg1_step2<T, size_t>,
          dim3(pg.nupd, w.B), dim3(kPcgBlock), g, w.alpha, w.K, w.mask, w.winv,
          w.ik[0], w.ik[1], w.r, w.z, w.q, w.e0, w.p0, w.p1, w.e1, w.x, w.part, w.st1, pg.ps, pg.nrz, lp);
    }
    if (pg.nrz == 1 && pg.nupd > 1) {  // the set the step wrote: its parity ^ 1
        L((const void*)k_partials_sum<Cg1State>, dim3(w.B), dim3(1024), w.part, pg.ps, pg.nupd, 0, 1, 2, 1,
          (const Cg1State*)w.st1, lp, 1, (const double*)nullptr);
        L((const void*)k_partials_sum<Cg1State>, dim3(w.B), dim3(1024), w.part, pg.ps, pg.nupd, 4, 1, -1, 0,
          (const Cg1State*)w.st1, lp, 1, (const double*)nullptr);
    }
    if (refresh)
        L((const void*)k_cg1_refresh2<T>, dim3(pg.nupd, w.B), dim3(kPcgBlock), g, w.alpha, w.K, w.mask,
          (const T*)w.e1, w.p0, w.p1, (const Cg1State*)w.st1, lp);
}

// ----------------------------------------------------------------------------------
// Segment control on the device.  A field's recursion runs in segments; when one ends
// (its state reports done), the end of the chunk (graph replay) in which it ended adds
// the segment's correction to u in float64, recomputes the true residual f - K u in
// float64, and either retires the field (converged, iteration limit, stagnation,
// breakdown) or starts its next segment: continued with the same search direction
// from the replaced residual, or restarted when the recursion had drifted from the true
// residual.  Every decision uses the field's own numbers only, and happens at a chunk
// boundary fixed by the field's own iteration count, so fields in one batch never wait
// for each other and a field's result does not depend on the batch.
// ----------------------------------------------------------------------------------
// Largest ratio of true to recursive residual at the end of a segment for which the
// recursion is continued after the residual replacement (else it restarts).
constexpr double kReplaceDriftMax = 4.0;
// Reduction of the residual a float32 segment aims for before its residual is replaced
// by the float64 one (small enough to keep the replacements rare, large enough that the
// float32 recursion has not drifted from the true residual; 3e-3 .. 1e-1 measured
// within 2 % of each other in iterations).
constexpr double kMixedSegmentTol = 1e-2;
constexpr int kMaxSegments = 400;

struct SegCtl {
    double nf;          // ||f_f|| (the inner system is scaled by 1 / nf)
    double scale;       // 1 / nf (1 when f = 0)
    double rr;          // ||f - K u||^2 of the current u
    double rr_prev;     // the same before the last segment
    double fin_rr;      // recursive (scaled) ||r||^2 at the end of the last segment
    double res[3];      // residual sums of the current u: ||r||^2, f^T u, u^T r
    double last_rz[2];  // r.z of the last two iterations of the last segment
    int live;           // 1 while the field is being solved
    int fresh;          // the next segment restarts the recursion
    int ending;         // the field's segment ended in the chunk just run
    int stagnated;      // retired because replacements stopped reducing the residual
    int total, base, segments, status, maxit, seg_iters, fin_done, fin_iters;
};

__device__ __forceinline__ int st_iters(const PcgState& s) { return s.iters; }
__device__ __forceinline__ int st_iters(const Cg1State& s) { return s.iters[0] > s.iters[1] ? s.iters[0] : s.iters[1]; }
__device__ __forceinline__ void st_rz(const PcgState& s, SegCtl& c) {
    c.last_rz[0] = s.rz[0];
    c.last_rz[1] = s.rz[1];
}
__device__ __forceinline__ void st_rz(const Cg1State&, SegCtl&) {}

// The state of the field's next segment (fresh: x = 0, beta = 0 at its first step;
// continued: same direction, the stopping test against the replaced residual).
__device__ __forceinline__ void seg_state(const SegCtl& c, double tol2, PcgState& p) {
    const int it0 = c.fresh ? 0 : c.fin_iters;
    p = PcgState{};
    p.bb = p.rr = c.fresh ? 0.0 : c.rr * c.scale * c.scale;
    p.tol2 = tol2;
    p.rz[0] = c.fresh ? 0.0 : c.last_rz[0];
    p.rz[1] = c.fresh ? 0.0 : c.last_rz[1];
    p.maxit = c.maxit - c.base;
    p.iters = it0;
    p.poff = (it0 & 1) ^ 1;  // the segment's first launch has launch parity 1
    p.qoff = (it0 - 1) & (kRing3 - 1);  // and launch index 1 mod 8
    p.fresh = c.fresh;
    p.it0 = it0;
}
__device__ __forceinline__ void seg_state(const SegCtl& c, double tol2, Cg1State& q) {
    const int it0 = c.fresh ? 0 : c.fin_iters;
    q = Cg1State{};
    q.bb = q.rr = c.fresh ? 0.0 : c.rr * c.scale * c.scale;
    q.tol2 = tol2;
    q.maxit = c.maxit - c.base;
    q.iters[0] = q.iters[1] = it0;
    q.poff = (it0 & 1) ^ 1;
    q.kind0 = c.fresh ? kCg1Fresh : kCg1Continued;
    q.it0 = it0;
}

// Stopping tests at the current u, then the next segment (fsc[b] = scale) or retirement.
template <typename S>
__device__ __forceinline__ void seg_next(SegCtl& c, S& st, double* fsc, int* live, int b, double rtol,
                                         double seg_min) {
    const double rel = c.nf > 0.0 ? sqrt(c.rr) / c.nf : 0.0;
    if (rel <= rtol) {
        c.live = 0;
    } else if (c.total >= c.maxit || c.segments >= kMaxSegments) {
        c.status = TOPO_ENOCONV;
        c.live = 0;
    } else if (c.segments > 0 && !(c.rr < 0.5 * c.rr_prev)) {
        c.status = TOPO_ENOCONV;
        c.stagnated = 1;
        c.live = 0;
    }
    if (!c.live) {
        st.done = 4;
        live[b] = 0;
        return;
    }
    double tol_seg = fmax(0.5 * rtol * c.nf / sqrt(c.rr), seg_min);
    tol_seg = fmin(fmax(tol_seg, 1e-15), 0.5);
    if (c.fresh) c.base = c.total;
    seg_state(c, tol_seg * tol_seg, st);
    fsc[b] = c.scale;
}

// After the initial residual (out[4b..4b+2]): every field to solve starts its first,
// fresh segment (or is done at once when u = 0 already meets the tolerance).
template <typename S>
__global__ void k_seg_init(int B, S* __restrict__ st, SegCtl* __restrict__ ctl, const double* __restrict__ out,
                           double* __restrict__ fsc, int* __restrict__ live, const int* __restrict__ solve,
                           const int* __restrict__ maxit, double rtol, double seg_min) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    SegCtl c{};
    fsc[b] = 0.0;
    live[b] = 0;
    if (!solve[b]) {
        st[b].done = 4;
        ctl[b] = c;
        return;
    }
    for (int q = 0; q < 3; ++q) c.res[q] = out[4 * b + q];
    c.nf = sqrt(c.res[0]);
    c.scale = c.nf > 0.0 ? 1.0 / c.nf : 1.0;
    c.rr = c.res[0];
    c.rr_prev = INFINITY;
    c.live = 1;
    c.fresh = 1;
    c.maxit = maxit[b];
    c.status = TOPO_OK;
    live[b] = 1;
    seg_next(c, st[b], fsc, live, b, rtol, seg_min);
    ctl[b] = c;
}

// End of a chunk, before the correction: the fields whose segment ended in it.  Their
// correction weight goes to corr[b] (0: none), the residual is recomputed for them only
// (skip[b] = 0); a breakdown without progress retires the field at once.
template <typename S>
__global__ void k_seg_mark(int B, S* __restrict__ st, SegCtl* __restrict__ ctl, int* __restrict__ skip,
                           double* __restrict__ corr, double* __restrict__ fsc, int* __restrict__ live) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    SegCtl& c = ctl[b];
    fsc[b] = 0.0;
    corr[b] = 0.0;
    skip[b] = 1;
    c.ending = 0;
    const int done = st[b].done;
    if (!c.live || done == 0) return;
    c.fin_done = done;
    c.fin_iters = st_iters(st[b]);
    c.fin_rr = st[b].rr;
    st_rz(st[b], c);
    c.seg_iters = c.base + c.fin_iters - c.total;
    c.total = c.base + c.fin_iters;
    if (done == 3 && c.seg_iters == 0) {
        c.status = TOPO_ENOTSPD;
        c.live = 0;
        live[b] = 0;
        st[b].done = 4;
        return;
    }
    c.ending = 1;
    skip[b] = 0;
    corr[b] = c.nf > 0.0 ? c.nf : 1.0;
    ++c.segments;
    c.rr_prev = c.rr;
}

// End of a chunk, after the corrected u's residual (out[4b..4b+2]): retire the field or
// start its next segment.
template <typename S>
__global__ void k_seg_control(int B, S* __restrict__ st, SegCtl* __restrict__ ctl, const double* __restrict__ out,
                              double* __restrict__ fsc, int* __restrict__ live, double rtol, double seg_min) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    SegCtl& c = ctl[b];
    if (!c.ending) return;
    c.ending = 0;
    for (int q = 0; q < 3; ++q) c.res[q] = out[4 * b + q];
    c.rr = c.res[0];
    if (c.fin_done == 3 && !(c.rr < c.rr_prev)) {
        c.status = TOPO_ENOTSPD;
        c.live = 0;
        live[b] = 0;
        st[b].done = 4;
        return;
    }
    // continue the recursion only while it still tracks the true residual; a segment
    // whose true residual drifted far from the recursive one restarts
    const double drift = c.fin_rr > 0.0 ? sqrt(c.rr) * c.scale / sqrt(c.fin_rr) : INFINITY;
    c.fresh = !(drift <= kReplaceDriftMax) || c.fin_done != 1;
    seg_next(c, st[b], fsc, live, b, rtol, seg_min);
}

// Mask bits per node: bit c set when DOF (node, c) is fixed (mask [3][N_n] -> [N_n]).
__global__ void k_node_mask(int n_nodes, const uint8_t* __restrict__ mask, uint8_t* __restrict__ bits) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_nodes) return;
    const size_t nn = (size_t)n_nodes;
    bits[n] = (uint8_t)((mask[n] ? 1u : 0u) | (mask[nn + n] ? 2u : 0u) | (mask[2 * nn + n] ? 4u : 0u));
}

// skip[b] = !solve[b]
__global__ void k_skip_from_solve(int B, const int* __restrict__ solve, int* __restrict__ skip) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) skip[b] = solve[b] ? 0 : 1;
}

// Iterations per graph replay: 16, or 64 when the batch is small (N_u B <= 4M DOF), where
// the chunk end (segment control, ~8 small kernels) would cost a third of a 16-iteration
// chunk.  Segments start at chunk ends, which are multiples of 16 launches either way,
// and the one-reduction recursion refreshes s every 16 launches, so a field's arithmetic
// does not depend on the chunk length (nor on the batch that chose it).
constexpr int kCg1Refresh = 16;
static int pcg_chunk_len(const Grid& g, int B) {
    return (long long)g.n_dofs * B <= (4LL << 20) ? 64 : 16;
}
static_assert(16 % kRing3 == 0 && 64 % kRing3 == 0, "chunks hold whole correction groups");

// Start of a segment for the fields with a nonzero scale fsc[b] (their states written
// by the segment controller): its partials for the first launch of the next chunk
// (launch parity 1).
template <int DIM, typename T>
static void phase_start(const Grid& g, const PcgBufs<T>& w, const PcgGeom& pg, bool one_red, LaunchSink& L) {
    if (one_red) {
        L((const void*)k_cg1_start2<T>, dim3(pg.nupd, w.B), dim3(kPcgBlock), g, w.alpha, w.K, w.mask, w.winv,
          w.ik[0], w.ik[1], w.r64, w.fsc, w.e1, w.r, w.z, w.q, w.e0, w.p0, w.p1, w.x, w.part,
          (const Cg1State*)w.st1, pg.ps);
        if (pg.nrz == 1 && pg.nupd > 1) {  // set it0 & 1, the first step's parity
            L((const void*)k_partials_sum<Cg1State>, dim3(w.B), dim3(1024), w.part, pg.ps, pg.nupd, 0, 1, 2, 1,
              (const Cg1State*)w.st1, 1, 0, w.fsc);
            L((const void*)k_partials_sum<Cg1State>, dim3(w.B), dim3(1024), w.part, pg.ps, pg.nupd, 4, 1, 6, 0,
              (const Cg1State*)w.st1, 1, 0, w.fsc);
            L((const void*)k_partials_sum<Cg1State>, dim3(w.B), dim3(1024), w.part, pg.ps, pg.nupd, 7, 0, -1, 0,
              (const Cg1State*)w.st1, 1, 0, w.fsc);
        }
    } else {
        L((const void*)k_pcg_start<DIM, T>, dim3(pg.nupd, w.B), dim3(kPcgBlock), g, w.r64, w.fsc, w.winv,
          w.ik[0], w.ik[1], w.ik[2], w.x, w.r, w.z, w.p0, w.part, (const PcgState*)w.st, pg.ps);
        if (pg.nrz == 1 && pg.nupd > 1)  // the parity the first apply reads: its own ^ 1
            L((const void*)k_partials_sum<PcgState>, dim3(w.B), dim3(1024), w.part, pg.ps, pg.nupd, 1, 1, 3, 1,
              (const PcgState*)w.st, 1, 1, w.fsc);
    }
}

// Iteration `it` of a chunk (its launch parity is it & 1; chunks start at it = 1).  The
// one-reduction recursion refreshes s after every iteration it with it % kCg1Refresh == 0.
template <int DIM, typename T>
static void phase_iteration(Ctx* ctx, const Grid& g, const PcgBufs<T>& w, const PcgGeom& pg, bool one_red,
                            long long it, LaunchSink& L, int timing) {
    if (one_red) cg1_step<T>(ctx, g, w, pg, (int)(it & 1), L, timing, it % kCg1Refresh == 0);
    else pcg_iteration<DIM, T>(ctx, g, w, pg, (int)(it & (kRing3 - 1)), L, timing);
}

// K64: the dense element matrix in 2D, the reduced element blocks in 3D.
static int residual_launch(Ctx* ctx, const Grid& g0, const double* K64, const double* alpha64,
                           const uint8_t* mask, const double* u, const double* f, double* r, int B,
                           double* part, double* out, const int* skip, hipStream_t s) {
    // the residual march fits its own resident wave (never more blocks than a grid with
    // the default target, which sized the caller's partial arrays)
    Grid g = g0;
    if (g.dim == 3) g.mtarget = std::min(march3_target(ctx, (const void*)k_residual3), g0.mtarget > 0 ? g0.mtarget : 1024);
    const int nb = stencil_blocks(g);
    {
        TimedLaunch tl(ctx, KID_RESIDUAL, s);
        if (g.dim == 2)
            hipLaunchKernelGGL(k_residual2, dim3(nb, B), dim3(kBlock), 0, s, g, alpha64, K64, mask,
                               u, f, r, part, skip);
        else
            hipLaunchKernelGGL(k_residual3, dim3(nb, B), dim3(kBlock), 0, s, g, alpha64, K64, mask,
                               u, f, r, part, skip);
    }
    TOPO_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_residual_sum, dim3(B), dim3(kBlock), 0, s, nb, (const double*)part, out, skip);
    TOPO_CHECK_LAUNCH();
    return TOPO_OK;
}

template <typename T>
struct HdmWs {
    double *a64 = nullptr, *w64 = nullptr, *r64 = nullptr, *part = nullptr, *rpart = nullptr,
           *rout = nullptr, *x = nullptr, *fsc = nullptr, *corr = nullptr;
    T *r = nullptr, *z = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
    T* pk[kRing3 - 2] = {};  // 3D: ring slots 2..7
    T *e0 = nullptr, *e1 = nullptr;  // 2D float64: the one-reduction recursion's two further vectors
    T* side = nullptr;               // 3D: the apply's parts of shared nodes
    uint8_t* mnode = nullptr;        // 3D: mask bits per node (k_node_mask)
    float *a32 = nullptr, *w32 = nullptr;
    int *skip = nullptr, *live = nullptr, *solve = nullptr, *maxit = nullptr;
    SegCtl* ctl = nullptr;
    PcgState* st = nullptr;
    Cg1State* st1 = nullptr;
};

template <typename T>
static void hdm_takes(Arena& ar, const Grid& g, bool mixed, int B, HdmWs<T>& w) {
    const size_t N = (size_t)B * g.n_dofs;
    const size_t ps = partial_stride(g);
    ar.take(&w.a64, (size_t)B * g.n_elems);
    ar.take(&w.w64, (size_t)B * g.n_nodes);
    if (mixed) {
        ar.take(&w.a32, (size_t)B * g.n_elems);
        ar.take(&w.w32, (size_t)B * g.n_nodes);
    }
    ar.take(&w.r64, N);
    ar.take(&w.part, (size_t)B * kPcgParts * ps);
    ar.take(&w.rpart, (size_t)B * 3 * ps);
    ar.take(&w.rout, (size_t)4 * B);
    ar.take(&w.fsc, (size_t)B);
    ar.take(&w.corr, (size_t)B);
    ar.take(&w.skip, (size_t)B);
    ar.take(&w.live, (size_t)B);
    ar.take(&w.solve, (size_t)B);
    ar.take(&w.maxit, (size_t)B);
    ar.take(&w.ctl, (size_t)B);
    ar.take(&w.st, (size_t)B);
    ar.take(&w.st1, (size_t)B);
    ar.take(&w.x, N);
    ar.take(&w.r, N);
    if (!(g.dim == 3 && ApplyFormsZ<T>::value)) ar.take(&w.z, N);  // the float 3D apply forms z
    ar.take(&w.p0, N);
    ar.take(&w.p1, N);
    if (g.dim == 3)  // the ring of kRing3 directions
        for (int k = 0; k < kRing3 - 2; ++k) ar.take(&w.pk[k], N);
    ar.take(&w.q, N);
    if (g.dim == 2 && !mixed) {
        ar.take(&w.e0, N);
        ar.take(&w.e1, N);
    }
    if (g.dim == 3) {
        ar.take(&w.side, (size_t)B * 3 * side_geom(g).total);
        ar.take(&w.mnode, (size_t)g.n_nodes);
    }
}

size_t ws_hdm_solve(const Grid& g, bool mixed, int B) {
    Arena ar;
    if (mixed) {
        HdmWs<float> w;
        hdm_takes(ar, g, true, B, w);
    } else {
        HdmWs<double> w;
        hdm_takes(ar, g, false, B, w);
    }
    return ar.total();
}


// Buffers of the segment controller.
struct SegBufs {
    SegCtl* ctl;    // [B]
    int* skip;      // [B] residual skipped for the field
    int* live;      // [B] the field is still being solved
    double* corr;   // [B] weight of the segment's correction in u (0: none)
    double* fsc;    // [B] scale of a segment starting now (0: none)
    int* solve;     // [B] fields to solve
    int* maxit;     // [B]
};

// The residual kernels of residual_launch, as launches of L (for chunk graphs).
static void residual_sink(LaunchSink& L, const Grid& g, const double* K64, const double* a64, const uint8_t* mask,
                          const double* u, const double* f, double* r, int B, double* part, double* out,
                          const int* skip) {
    const int nb = stencil_blocks(g);
    L(g.dim == 2 ? (const void*)k_residual2 : (const void*)k_residual3, dim3(nb, B), dim3(kBlock), g, a64, K64,
      mask, u, f, r, part, skip);
    L((const void*)k_residual_sum, dim3(B), dim3(kBlock), nb, (const double*)part, out, skip);
}

// End of a chunk: the fields whose segment ended get their correction, their residual
// and the controller's decision; the next segments start.
template <int DIM, typename T>
static void chunk_end(const Grid& g, const Grid& gres, const double* K64, const double* a64, const double* f,
                      double* u, double* rpart, double* rout, const PcgBufs<T>& w, const PcgGeom& pg, bool one_red,
                      const SegBufs& c, double rtol, double seg_min, LaunchSink& L) {
    const dim3 gb(grid_blocks(w.B, 64)), bb(64);
    const long long N = g.n_dofs;
    if (one_red)
        L((const void*)k_seg_mark<Cg1State>, gb, bb, w.B, w.st1, c.ctl, c.skip, c.corr, c.fsc, c.live);
    else
        L((const void*)k_seg_mark<PcgState>, gb, bb, w.B, w.st, c.ctl, c.skip, c.corr, c.fsc, c.live);
    if (one_red)
        L((const void*)k_correct<double>, dim3(std::min(grid_blocks(N), 1024), w.B), dim3(kBlock), N, u,
          (const double*)w.x, (const double*)c.corr);
    else
        L((const void*)k_correct_pcg<T, XGroup<DIM>::value>, dim3(std::min(grid_blocks(N), 1024), w.B),
          dim3(kBlock), N, u, (const double*)w.x, w.ring(), (const PcgState*)w.st, (const double*)c.corr);
    residual_sink(L, gres, K64, a64, w.mask, u, f, (double*)w.r64, w.B, rpart, rout, (const int*)c.skip);
    if (one_red)
        L((const void*)k_seg_control<Cg1State>, gb, bb, w.B, w.st1, c.ctl, (const double*)rout, c.fsc, c.live, rtol,
          seg_min);
    else
        L((const void*)k_seg_control<PcgState>, gb, bb, w.B, w.st, c.ctl, (const double*)rout, c.fsc, c.live, rtol,
          seg_min);
    phase_start<DIM, T>(g, w, pg, one_red, L);
}

// Batched HDM solve of the fields with solve[b] != 0 (the others are left untouched):
// one Krylov recursion per field in precision T, cut into segments (see the segment
// controller above), iterations replayed as graphs of one chunk each (pcg_chunk_len
// iterations and the chunk end); the host launches chunks and checks the fields' live
// flags one chunk behind.  The inner system of each field is scaled by 1 / ||f|| so
// that float32 values stay O(1).  2D float64 solves run the one-reduction recursion
// (one kernel per iteration).  Per-field outcomes go to status[b] (TOPO_OK,
// TOPO_ENOCONV, TOPO_ENOTSPD) and stagnated[b]; the return value is a device or
// allocation error only.
template <int DIM, typename T>
static int hdm_batch_impl(Ctx* ctx, const topo_mesh& m, const Grid& g0, const ElemTables* tb,
                          const double* rho, const uint8_t* mask, const double* f, double* u, int B,
                          double rtol, const int* maxit, const uint8_t* solve, bool mixed, topo_info* info,
                          int* status, uint8_t* stagnated, hipStream_t s) {
    Grid g = g0;
    // 3D: chunk heights sized for one resident wave of the apply per field, shared out
    // when more than 8 fields run in one launch: taller chunks then leave fewer side
    // entries and block prologues while the launch still spans several waves (16 fields
    // on 192x96x96: 14 layers, 504 blocks per field, 7.9 waves)
    if constexpr (DIM == 3)
        g.mtarget = std::max(1, march3_target(ctx, pcg_apply3_fn<T>(apply3_narrow<T>(g0))) / ((B + 7) / 8));
    Grid gres = g;  // the residual march fits its own resident wave (and the partial arrays)
    if constexpr (DIM == 3) gres.mtarget = std::min(march3_target(ctx, (const void*)k_residual3), g.mtarget);
    const long long N = g.n_dofs;
    const bool one_red = DIM == 2 && sizeof(T) == 8;
    const PcgGeom pg = pcg_geom(g);
    Arena ar;
    HdmWs<T> ws;
    hdm_takes(ar, g, mixed, B, ws);
    int rc = ar.commit(ctx, s);
    if (rc) return rc;
    SegBufs c{ws.ctl, ws.skip, ws.live, ws.corr, ws.fsc, ws.solve, ws.maxit};
    rc = launch_tables(ctx, g, m, rho, B, ws.a64, ws.a32, ws.w64, ws.w32, s);
    if (rc) return rc;
    PcgBufs<T> w{};
    w.B = B;
    if constexpr (sizeof(T) == 4) {
        w.alpha = (const T*)ws.a32;
        w.winv = (const T*)ws.w32;
    } else {
        w.alpha = (const T*)ws.a64;
        w.winv = (const T*)ws.w64;
    }
    // 2D: the dense element matrix; 3D: the reduced blocks of the symmetry-blocked form
    if constexpr (DIM == 2) w.K = sizeof(T) == 4 ? (const T*)tb->K32 : (const T*)tb->K64;
    else w.K = sizeof(T) == 4 ? (const T*)tb->M32 : (const T*)tb->M64;
    w.mask = mask;
    w.mnode = ws.mnode;
    for (int q = 0; q < 3; ++q) w.ik[q] = q < DIM ? (T)(1.0 / tb->diag[q]) : T(0);
    w.r = ws.r;
    w.z = ws.z;
    w.p0 = ws.p0;
    w.p1 = ws.p1;
    for (int k = 0; k < kRing3 - 2; ++k) w.pk[k] = ws.pk[k];
    w.q = ws.q;
    w.e0 = ws.e0;
    w.e1 = ws.e1;
    w.side = ws.side;
    if constexpr (DIM == 3) {
        w.sg = side_geom(g);
        w.Mv = sizeof(T) == 4 ? *(const FacTab<T>*)&tb->Mv32 : *(const FacTab<T>*)&tb->Mv64;
        w.narrow = apply3_narrow<T>(g);
    }
    w.x = ws.x;
    w.part = ws.part;
    w.st = ws.st;
    w.st1 = ws.st1;
    w.r64 = ws.r64;
    w.fsc = ws.fsc;
    const double* K64 = DIM == 2 ? tb->K64 : tb->M64;
    const double seg_min = mixed ? kMixedSegmentTol : 0.0;

    // pinned host layout: [2 live slots of B ints | B solve flags | B limits | B controls]
    const size_t off_solve = 2 * B * sizeof(int), off_maxit = off_solve + B * sizeof(int),
                 off_ctl = (off_maxit + B * sizeof(int) + 15) & ~size_t(15);
    void* pin = nullptr;
    rc = pinned_host(ctx, off_ctl + B * sizeof(SegCtl), &pin);
    if (rc) return rc;
    char* pc = (char*)pin;
    int* h_live = (int*)pc;
    int* h_solve = (int*)(pc + off_solve);
    int* h_maxit = (int*)(pc + off_maxit);
    SegCtl* h_ctl = (SegCtl*)(pc + off_ctl);
    long long cap = 0;
    for (int b = 0; b < B; ++b) {
        h_solve[b] = solve[b] ? 1 : 0;
        h_maxit[b] = maxit[b];
        if (solve[b]) {
            TOPO_HIP(hipMemsetAsync(u + (size_t)b * N, 0, N * sizeof(double), s));
            cap = std::max(cap, (long long)maxit[b]);
        }
    }
    cap += 4096;
    TOPO_HIP(hipMemcpyAsync(c.solve, h_solve, B * sizeof(int), hipMemcpyHostToDevice, s));
    TOPO_HIP(hipMemcpyAsync(c.maxit, h_maxit, B * sizeof(int), hipMemcpyHostToDevice, s));
    // the initial residual of the fields to solve, their first segments
    {
        LaunchSink L;
        L.s = s;
        hipLaunchKernelGGL(k_skip_from_solve, dim3(grid_blocks(B, 64)), dim3(64), 0, s, B, (const int*)c.solve,
                           c.skip);
        if (DIM == 3)
            hipLaunchKernelGGL(k_node_mask, dim3(grid_blocks(g.n_nodes)), dim3(kBlock), 0, s, (int)g.n_nodes, mask,
                               ws.mnode);
        residual_sink(L, gres, K64, ws.a64, mask, u, f, ws.r64, B, ws.rpart, ws.rout, (const int*)c.skip);
        if (one_red)
            L((const void*)k_seg_init<Cg1State>, dim3(grid_blocks(B, 64)), dim3(64), B, ws.st1, c.ctl,
              (const double*)ws.rout, c.fsc, c.live, (const int*)c.solve, (const int*)c.maxit, rtol, seg_min);
        else
            L((const void*)k_seg_init<PcgState>, dim3(grid_blocks(B, 64)), dim3(64), B, ws.st, c.ctl,
              (const double*)ws.rout, c.fsc, c.live, (const int*)c.solve, (const int*)c.maxit, rtol, seg_min);
        phase_start<DIM, T>(g, w, pg, one_red, L);
        TOPO_HIP(L.err);
        TOPO_CHECK_LAUNCH();
    }
    // mode: kTimeOff (graph construction), kTimeForced (a timing sample replacing a
    // replay: its first kTimeRun iterations timed, a whole correction group), kTimeSampled
    // (no graphs)
    const int chunk_len = pcg_chunk_len(g, B);
    auto chunk = [&](LaunchSink& L, int mode) {
        for (int q = 0; q < chunk_len; ++q) {
            const int tm = mode == kTimeForced ? (q < kTimeRun ? kTimeForced : kTimeOff) : mode;
            phase_iteration<DIM, T>(ctx, g, w, pg, one_red, 1 + q, L, tm);
        }
        chunk_end<DIM, T>(g, gres, K64, ws.a64, f, u, ws.rpart, ws.rout, w, pg, one_red, c, rtol, seg_min, L);
    };
    hipGraphExec_t exec = nullptr;
    if (graphs_enabled()) {
        std::vector<uintptr_t> key = {(uintptr_t)0xB7C7, (uintptr_t)DIM, sizeof(T), (uintptr_t)one_red,
                                      (uintptr_t)B, (uintptr_t)pg.napp, (uintptr_t)pg.nupd, (uintptr_t)chunk_len,
                                      (uintptr_t)g.nx, (uintptr_t)g.ny, (uintptr_t)g.nz, (uintptr_t)g.mtarget,
                                      (uintptr_t)gres.mtarget, (uintptr_t)w.alpha, (uintptr_t)w.K,
                                      (uintptr_t)w.mask, (uintptr_t)w.mnode, (uintptr_t)w.winv, (uintptr_t)w.x, (uintptr_t)w.r,
                                      (uintptr_t)w.z, (uintptr_t)w.p0, (uintptr_t)w.p1, (uintptr_t)w.q,
                                      (uintptr_t)w.e0, (uintptr_t)w.e1, (uintptr_t)w.side, (uintptr_t)w.part,
                                      (uintptr_t)w.st,
                                      (uintptr_t)w.st1, (uintptr_t)ws.a64, (uintptr_t)ws.r64, (uintptr_t)ws.rpart,
                                      (uintptr_t)ws.rout, (uintptr_t)u, (uintptr_t)f, (uintptr_t)c.ctl,
                                      (uintptr_t)c.skip, (uintptr_t)c.live, (uintptr_t)c.corr, (uintptr_t)c.fsc};
        for (int q = 0; q < 3; ++q) key_push_double(key, (double)w.ik[q]);
        for (int k = 0; k < kRing3 - 2; ++k) key.push_back((uintptr_t)w.pk[k]);
        key_push_double(key, rtol);
        key_push_double(key, seg_min);
        rc = cached_graph(ctx, key, [&](LaunchSink& G) { chunk(G, kTimeOff); }, &exec, s);
        if (rc) return rc;
    }
    // chunks until every field has retired; the host reads the live flags one chunk
    // behind.  A timing sample replaces one replay by direct launches (two timed).
    hipEvent_t ev[2];
    TOPO_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    TOPO_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    bool pending[2] = {false, false};
    long long issued = 0, replays = 0;
    int slot = 0;
    LaunchSink L;
    L.s = s;
    const int kids[2] = {one_red ? KID_PCG_STEP : KID_PCG_APPLY, one_red ? -1 : KID_PCG_UPDATE};
    while (true) {
        const int every = ctx->timing.every;
        if (exec && !(every > 0 && replays % every == 0)) {
            const hipError_t e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) {
                rc = set_error(ctx, TOPO_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
                break;
            }
        } else {
            chunk(L, exec ? kTimeForced : kTimeSampled);
            if (L.err != hipSuccess) {
                rc = set_error(ctx, TOPO_EDEVICE, "PCG chunk launch: %s", hipGetErrorString(L.err));
                break;
            }
        }
        issued += chunk_len;
        ++replays;
        if (every > 0)
            for (int kid : kids)
                if (kid >= 0) ctx->timing.launched[kid] += chunk_len;
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(h_live + (size_t)slot * B, c.live, B * sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(ev[slot], s);
        if (e != hipSuccess) {
            rc = set_error(ctx, TOPO_EDEVICE, "PCG chunk: %s", hipGetErrorString(e));
            break;
        }
        pending[slot] = true;
        const int other = slot ^ 1;
        bool stop = false;
        if (pending[other]) {
            e = hipEventSynchronize(ev[other]);
            if (e != hipSuccess) {
                rc = set_error(ctx, TOPO_EDEVICE, "PCG chunk: %s", hipGetErrorString(e));
                break;
            }
            pending[other] = false;
            stop = true;
            for (int b = 0; b < B; ++b) stop &= h_live[(size_t)other * B + b] == 0;
        }
        if (stop || issued >= cap) break;
        slot = other;
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (rc) return rc;
    TOPO_HIP(hipMemcpyAsync(h_ctl, c.ctl, B * sizeof(SegCtl), hipMemcpyDeviceToHost, s));
    TOPO_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < B; ++b) {
        if (!solve[b]) continue;
        SegCtl& fd = h_ctl[b];
        if (fd.live) {  // the iteration cap of the chunk loop (every field has a limit below it)
            fd.status = TOPO_ENOCONV;
            fd.live = 0;
        }
        topo_info& in = info[b];
        in.iters = fd.total;
        in.refinements = fd.segments;
        in.rel_resid = fd.nf > 0.0 ? std::sqrt(fd.rr) / fd.nf : 0.0;
        in.compliance_raw = fd.res[1];
        in.compliance_corr = fd.res[1] + fd.res[2];
        in.status = fd.status;
        if (stagnated) stagnated[b] = fd.stagnated ? 1 : 0;
        if (fd.status == TOPO_ENOCONV && !fd.stagnated)
            set_error(ctx, TOPO_ENOCONV, "no convergence: rel. residual %.3e after %d iterations (field %d)",
                      in.rel_resid, fd.total, b);
        else if (fd.status == TOPO_ENOCONV)
            set_error(ctx, TOPO_ENOCONV, "residual replacement stagnated at rel. residual %.3e (field %d)",
                      in.rel_resid, b);
        else if (fd.status == TOPO_ENOTSPD)
            set_error(ctx, TOPO_ENOTSPD, "CG breakdown: p^T K p <= 0 (field %d)", b);
        status[b] = fd.status;
    }
    return TOPO_OK;
}

// Batched solve with the mixed-precision fallback: a field whose float32 corrections
// stop reducing the true residual (float32 rounding too coarse for its operator) is
// redone in float64 from zero with the iterations it has left.
template <int DIM>
static int hdm_solve_batch(Ctx* ctx, const topo_mesh& m, const Grid& g, const ElemTables* tb, const double* rho,
                           const uint8_t* mask, const double* f, double* u, int B, double rtol, int maxit,
                           bool mixed, topo_info* info, hipStream_t s) {
    std::vector<int> mi(B, maxit), status(B, TOPO_OK);
    std::vector<uint8_t> solve(B, 1), stag(B, 0);
    for (int b = 0; b < B; ++b) info[b] = topo_info{};
    if (!mixed)
        return hdm_batch_impl<DIM, double>(ctx, m, g, tb, rho, mask, f, u, B, rtol, mi.data(), solve.data(),
                                           false, info, status.data(), nullptr, s);
    int rc = hdm_batch_impl<DIM, float>(ctx, m, g, tb, rho, mask, f, u, B, rtol, mi.data(), solve.data(), true,
                                        info, status.data(), stag.data(), s);
    if (rc) return rc;
    bool any = false;
    std::vector<topo_info> first(info, info + B);
    for (int b = 0; b < B; ++b) {
        solve[b] = stag[b] && maxit - first[b].iters >= 1;
        mi[b] = maxit - first[b].iters;
        any |= solve[b] != 0;
    }
    if (!any) return TOPO_OK;
    rc = hdm_batch_impl<DIM, double>(ctx, m, g, tb, rho, mask, f, u, B, rtol, mi.data(), solve.data(), false,
                                     info, status.data(), nullptr, s);
    if (rc) return rc;
    for (int b = 0; b < B; ++b)
        if (solve[b]) {
            info[b].iters += first[b].iters;
            info[b].refinements += first[b].refinements;
            info[b].fp64_fallback = 1;
        }
    return TOPO_OK;
}

}  // namespace topo

using namespace topo;

namespace topo {

// W = K(rho) X for ncols vectors X = [ncols][ld] (ld >= N_u) sharing one density field
// (alpha: its table, [N_e]), Dirichlet rows and columns eliminated: the columns of the
// ROM contraction K_hat = X^T K X.  X stored as TX (float32 or float64), arithmetic and W
// in float64.  Entries ld - N_u past each vector are not written.
template <typename TX>
int apply_columns(Ctx* ctx, const Grid& g0, const ElemTables* tb, const double* alpha, const uint8_t* mask,
                  const TX* x, double* y, int ncols, long long ld, hipStream_t s) {
    Grid g = g0;
    if (g.dim == 3) g.mtarget = march3_target(ctx, (const void*)k_apply3<double, TX, double>);
    const dim3 grid(stencil_blocks(g), ncols);
    if (g.dim == 2)
        hipLaunchKernelGGL((k_apply2<double, TX, double>), grid, dim3(kBlock), 0, s, g, alpha, 0LL, ld, tb->K64,
                           mask, x, y);
    else
        hipLaunchKernelGGL((k_apply3<double, TX, double>), grid, dim3(kBlock), 0, s, g, alpha, 0LL, ld, tb->M64,
                           mask, x, y);
    TOPO_CHECK_LAUNCH();
    return TOPO_OK;
}
template int apply_columns<float>(Ctx*, const Grid&, const ElemTables*, const double*, const uint8_t*,
                                  const float*, double*, int, long long, hipStream_t);
template int apply_columns<double>(Ctx*, const Grid&, const ElemTables*, const double*, const uint8_t*,
                                   const double*, double*, int, long long, hipStream_t);

}  // namespace topo

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
            hipLaunchKernelGGL((k_apply2<double>), grid, dim3(kBlock), 0, s, g, a64, (long long)g.n_elems,
                               (long long)g.n_dofs, tb->K64, mask, (const double*)x, (double*)y);
        else
            hipLaunchKernelGGL((k_apply3<double>), grid, dim3(kBlock), 0, s, g, a64, (long long)g.n_elems,
                               (long long)g.n_dofs, tb->M64, mask, (const double*)x, (double*)y);
    } else {
        if (g.dim == 2)
            hipLaunchKernelGGL((k_apply2<float>), grid, dim3(kBlock), 0, s, g, a32, (long long)g.n_elems,
                               (long long)g.n_dofs, tb->K32, mask, (const float*)x, (float*)y);
        else
            hipLaunchKernelGGL((k_apply3<float>), grid, dim3(kBlock), 0, s, g, a32, (long long)g.n_elems,
                               (long long)g.n_dofs, tb->M32, mask, (const float*)x, (float*)y);
    }
    TOPO_CHECK_LAUNCH();
    return TOPO_OK;
}

int topo_hdm_solve_batch(topo_ctx* ctx, const topo_mesh* mesh, const double* rho, const uint8_t* mask,
                         const double* f, double* u, int32_t B, double rtol, int32_t maxit, int32_t prec,
                         double* compliance, topo_info* info, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    int rc = validate_mesh(ctx, mesh);
    if (rc) return rc;
    if (!rho || !mask || !f || !u) return set_error(ctx, TOPO_EINVAL, "null pointer argument");
    if (B < 1) return set_error(ctx, TOPO_EINVAL, "B must be >= 1");
    if (!(rtol > 0.0) || !(rtol < 1.0)) return set_error(ctx, TOPO_EINVAL, "rtol must lie in (0, 1)");
    if (maxit < 1) return set_error(ctx, TOPO_EINVAL, "maxit must be >= 1");
    if (prec != TOPO_FP64 && prec != TOPO_MIXED) return set_error(ctx, TOPO_EINVAL, "bad precision");
    TOPO_HIP(hipSetDevice(ctx->device));
    const Grid g = make_grid(*mesh);
    const ElemTables* tb = get_tables(ctx, *mesh);
    if (!tb) return set_error(ctx, TOPO_EDEVICE, "element table upload failed");
    hipStream_t s = (hipStream_t)stream;
    std::vector<topo_info> local;
    topo_info* inf = info;
    if (!inf) {
        local.resize(B);
        inf = local.data();
    }
    const bool mixed = prec == TOPO_MIXED;
    rc = g.dim == 2 ? hdm_solve_batch<2>(ctx, *mesh, g, tb, rho, mask, f, u, B, rtol, maxit, mixed, inf, s)
                    : hdm_solve_batch<3>(ctx, *mesh, g, tb, rho, mask, f, u, B, rtol, maxit, mixed, inf, s);
    if (rc) return rc;
    int first_bad = -1;
    for (int b = 0; b < B; ++b) {
        if (compliance) compliance[b] = inf[b].compliance_corr;
        if (inf[b].status != TOPO_OK && first_bad < 0) first_bad = b;
    }
    if (first_bad < 0) return TOPO_OK;
    const int code = inf[first_bad].status;
    if (B > 1) {
        const std::string msg = ctx->err;
        set_error(ctx, code, "field %d: %s", first_bad, msg.c_str());
    }
    return code;
}

int topo_hdm_solve(topo_ctx* ctx, const topo_mesh* mesh, const double* rho, const uint8_t* mask,
                   const double* f, double* u, double rtol, int32_t maxit, int32_t prec,
                   double* compliance, topo_info* info, void* stream) {
    return topo_hdm_solve_batch(ctx, mesh, rho, mask, f, u, 1, rtol, maxit, prec, compliance, info, stream);
}

int topo_hdm_gradient_batch(topo_ctx* ctx, const topo_mesh* mesh, const double* rho, const double* u,
                            int32_t B, double* dc, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    int rc = validate_mesh(ctx, mesh);
    if (rc) return rc;
    if (!rho || !u || !dc) return set_error(ctx, TOPO_EINVAL, "null pointer argument");
    if (B < 1) return set_error(ctx, TOPO_EINVAL, "B must be >= 1");
    TOPO_HIP(hipSetDevice(ctx->device));
    const Grid g = make_grid(*mesh);
    const ElemTables* tb = get_tables(ctx, *mesh);
    if (!tb) return set_error(ctx, TOPO_EDEVICE, "element table upload failed");
    return gradient_launch(ctx, g, *mesh, tb, rho, u, B, dc, (hipStream_t)stream);
}

int topo_hdm_gradient(topo_ctx* ctx, const topo_mesh* mesh, const double* rho, const double* u,
                      double* dc, void* stream) {
    return topo_hdm_gradient_batch(ctx, mesh, rho, u, 1, dc, stream);
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

// Entry points shared with the ROM translation unit.
int residual_fp64(Ctx* ctx, const Grid& g, const ElemTables* tb, const double* alpha64,
                  const uint8_t* mask, const double* u, const double* f, double* r, int B,
                  double* part, double* out, hipStream_t s) {
    return residual_launch(ctx, g, g.dim == 2 ? tb->K64 : tb->M64, alpha64, mask, u, f, r, B, part, out,
                           nullptr, s);
}

int alpha_tables(Ctx* ctx, const Grid& g, const topo_mesh& m, const double* rho, int B,
                 double* a64, float* a32, hipStream_t s) {
    return launch_tables(ctx, g, m, rho, B, a64, a32, nullptr, nullptr, s);
}

}  // namespace topo
