// 2D node-centric matrix-free application of K(rho) = sum_e alpha_e P_e K_e P_e^T
// (Sec. 2.1) on a structured grid.  One thread owns one node and gathers the
// contributions of the 4 elements around it: for each element it needs only the 2
// rows of K_e that belong to its node, so every element row is evaluated exactly once
// over the whole grid and no scatter / atomic is needed.  The 3x3 neighbour values
// are loaded once into registers; consecutive threads own consecutive nodes along x,
// so every load is coalesced and the reuse across neighbours is served by the L1/L2
// caches.  K_e is read through uniform (scalar) loads.  (3D uses the element-centric
// march of march3.hpp.)
#pragma once

#include "internal.hpp"

namespace topo {

// Input fetchers: value of component c at node n (n is always in range).  I: index type
// of the per-field array (32-bit when its bytes fit: the load then takes the uniform base
// and one 32-bit offset instead of a 64-bit address per neighbour).
template <typename T, typename I = size_t>
struct FetchPlain {
    const T* __restrict__ x;
    int nn;
    __device__ __forceinline__ T operator()(int n, int c) const { return ld_at(x, (I)c * (I)nn + (I)n); }
};

template <typename T, typename TX = T>
struct FetchMasked {  // x (stored as TX) in the arithmetic type T, Dirichlet DOFs zeroed
    const TX* __restrict__ x;
    const uint8_t* __restrict__ mask;
    int nn;
    __device__ __forceinline__ T operator()(int n, int c) const {
        const size_t i = (size_t)c * nn + n;
        return mask[i] ? T(0) : (T)x[i];
    }
};

// 2D building blocks, split so that a caller can issue every load before it waits on
// anything else: the 3x3 neighbourhood of node (i,j) (zero outside the grid) and the
// alpha of the 2x2 elements around it (zero outside the grid).
template <typename T, typename Fetch>
__device__ __forceinline__ void load_nbhd2(const Grid& g, int i, int j, const Fetch& fetch,
                                           T (&xs)[3][3][2]) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int ii = i + dx - 1, jj = j + dy - 1;
            const bool ok = (ii >= 0) & (ii < g.nx1) & (jj >= 0) & (jj < g.ny1);
            const int n = jj * g.nx1 + ii;
            xs[dy][dx][0] = ok ? fetch(n, 0) : T(0);
            xs[dy][dx][1] = ok ? fetch(n, 1) : T(0);
        }
}

template <typename T, typename I = size_t>
__device__ __forceinline__ void load_alpha2(const Grid& g, int i, int j, const T* __restrict__ alpha,
                                            T (&al)[2][2]) {
#pragma unroll
    for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) {
            const int exx = i - 1 + ex, eyy = j - 1 + ey;
            const bool ok = (exx >= 0) & (exx < g.nx) & (eyy >= 0) & (eyy < g.ny);
            al[ey][ex] = ok ? ld_at(alpha, (I)(eyy * g.nx + exx)) : T(0);
        }
}

// out[c] = (K(rho) x)(node, c) from its loaded neighbourhood and element alphas.
template <typename T>
__device__ __forceinline__ void apply_nbhd2(const T* __restrict__ K, T (&xs)[3][3][2],
                                            const T (&al)[2][2], T (&out)[2]) {
    // K_e rows sum to zero per component (rigid translations), so each element vector
    // may be taken relative to this node's value: exact, and free of cancellation when
    // x is smooth.  Out-of-grid entries only meet alpha = 0.
    {
        const T c0 = xs[1][1][0], c1 = xs[1][1][1];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                xs[dy][dx][0] -= c0;
                xs[dy][dx][1] -= c1;
            }
    }
    out[0] = out[1] = T(0);
#pragma unroll
    for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) {
            const int a = (1 - ex) + 2 * (1 - ey);  // local index of this node in e
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const T* row = K + (2 * a + c) * 8;
                T s = T(0);
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int bx = b & 1, by = b >> 1;
                    s += row[2 * b] * xs[ey + by][ex + bx][0];
                    s += row[2 * b + 1] * xs[ey + by][ex + bx][1];
                }
                out[c] += al[ey][ex] * s;
            }
        }
}

// out[c] = (K(rho) x)(node (i,j,k), c) with x given by `fetch` (zero outside the grid)
// and alpha_e read from `alpha` (zero outside the grid).
template <typename T, typename Fetch>
__device__ __forceinline__ void node_apply2(const Grid& g, int i, int j,
                                            const T* __restrict__ alpha,
                                            const T* __restrict__ K, const Fetch& fetch,
                                            T (&out)[2]) {
    T xs[3][3][2];
    T al[2][2];
    load_nbhd2(g, i, j, fetch, xs);
    load_alpha2(g, i, j, alpha, al);
    apply_nbhd2(K, xs, al, out);
}

// Sum of alpha_e over the elements around a node (the Jacobi diagonal of K is
// K_e[c][c] times this sum on the structured grid: every local node of a rectangular
// element has the same diagonal entry per component).
template <typename T>
__device__ __forceinline__ T node_alpha_sum(const Grid& g, int i, int j, int k,
                                            const T* __restrict__ alpha) {
    T s = T(0);
    for (int ez = 0; ez < (g.dim == 3 ? 2 : 1); ++ez)
        for (int ey = 0; ey < 2; ++ey)
            for (int ex = 0; ex < 2; ++ex) {
                const int exx = i - 1 + ex, eyy = j - 1 + ey;
                const int ezz = g.dim == 3 ? k - 1 + ez : 0;
                if (exx >= 0 && exx < g.nx && eyy >= 0 && eyy < g.ny && ezz >= 0 && ezz < g.nz)
                    s += alpha[(ezz * g.ny + eyy) * g.nx + exx];
            }
    return s;
}

__device__ __forceinline__ void node_ijk(const Grid& g, int n, int& i, int& j, int& k) {
    const unsigned t = g.dnx1.div((unsigned)n), kk = g.dny1.div(t);
    i = n - (int)t * g.nx1;
    j = (int)(t - kk * (unsigned)g.ny1);
    k = (int)kk;
}

}  // namespace topo
