// Node-centric matrix-free application of K(rho) = sum_e alpha_e P_e K_e P_e^T
// (Sec. 2.1) on a structured grid.  One thread owns one node and gathers the
// contributions of the 2^dim elements around it: for each element it needs only the
// dim rows of K_e that belong to its node, so every element row is evaluated exactly
// once over the whole grid and no scatter / atomic is needed.  The 3^dim neighbour
// values are loaded once into registers; consecutive threads own consecutive nodes
// along x, so every load is coalesced and the 3x reuse across neighbours is served
// by the L1/L2 caches.  K_e is read through uniform (scalar) loads.
#pragma once

#include "internal.hpp"

namespace topo {

// Input fetchers: value of component c at node n (n is always in range).
template <typename T>
struct FetchPlain {
    const T* __restrict__ x;
    int nn;
    __device__ __forceinline__ T operator()(int n, int c) const { return x[(size_t)c * nn + n]; }
};

template <typename T>
struct FetchMasked {
    const T* __restrict__ x;
    const uint8_t* __restrict__ mask;
    int nn;
    __device__ __forceinline__ T operator()(int n, int c) const {
        const size_t i = (size_t)c * nn + n;
        return mask[i] ? T(0) : x[i];
    }
};

// p_new = z + beta * p_old (the CG direction update fused into the apply).
template <typename T>
struct FetchDirection {
    const T* __restrict__ z;
    const T* __restrict__ p;
    T beta;
    int nn;
    __device__ __forceinline__ T operator()(int n, int c) const {
        const size_t i = (size_t)c * nn + n;
        return z[i] + beta * p[i];
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

template <typename T>
__device__ __forceinline__ void load_alpha2(const Grid& g, int i, int j, const T* __restrict__ alpha,
                                            T (&al)[2][2]) {
#pragma unroll
    for (int ey = 0; ey < 2; ++ey)
#pragma unroll
        for (int ex = 0; ex < 2; ++ex) {
            const int exx = i - 1 + ex, eyy = j - 1 + ey;
            const bool ok = (exx >= 0) & (exx < g.nx) & (eyy >= 0) & (eyy < g.ny);
            al[ey][ex] = ok ? alpha[eyy * g.nx + exx] : T(0);
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

template <typename T, typename Fetch>
__device__ __forceinline__ void node_apply3(const Grid& g, int i, int j, int k,
                                            const T* __restrict__ alpha,
                                            const T* __restrict__ K, const Fetch& fetch,
                                            T (&out)[3]) {
    T xs[3][3][3][3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int ii = i + dx - 1, jj = j + dy - 1, kk = k + dz - 1;
                const bool ok = (ii >= 0) & (ii < g.nx1) & (jj >= 0) & (jj < g.ny1) &
                                (kk >= 0) & (kk < g.nz1);
                const int n = (kk * g.ny1 + jj) * g.nx1 + ii;
#pragma unroll
                for (int c = 0; c < 3; ++c) xs[dz][dy][dx][c] = ok ? fetch(n, c) : T(0);
            }
    // element vectors relative to this node's value (see node_apply2)
    {
        const T c0 = xs[1][1][1][0], c1 = xs[1][1][1][1], c2 = xs[1][1][1][2];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    xs[dz][dy][dx][0] -= c0;
                    xs[dz][dy][dx][1] -= c1;
                    xs[dz][dy][dx][2] -= c2;
                }
    }
    out[0] = out[1] = out[2] = T(0);
#pragma unroll
    for (int ez = 0; ez < 2; ++ez)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
            for (int ex = 0; ex < 2; ++ex) {
                const int exx = i - 1 + ex, eyy = j - 1 + ey, ezz = k - 1 + ez;
                const bool ok = (exx >= 0) & (exx < g.nx) & (eyy >= 0) & (eyy < g.ny) &
                                (ezz >= 0) & (ezz < g.nz);
                const T al = ok ? alpha[(ezz * g.ny + eyy) * g.nx + exx] : T(0);
                const int a = (1 - ex) + 2 * (1 - ey) + 4 * (1 - ez);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T* row = K + (3 * a + c) * 24;
                    T s = T(0);
#pragma unroll
                    for (int b = 0; b < 8; ++b) {
                        const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
#pragma unroll
                        for (int d = 0; d < 3; ++d)
                            s += row[3 * b + d] * xs[ez + bz][ey + by][ex + bx][d];
                    }
                    out[c] += al * s;
                }
            }
}

// ----------------------------------------------------------------------------------
// 3D, LDS-tiled: a block of 256 threads owns a 16 x 4 x 4 tile of nodes.  The tile and
// its one-node halo (18 x 6 x 6 nodes, 3 components) and the 17 x 5 x 5 element alphas
// around it are staged in LDS once, so each input value is read from memory ~2.5 times
// instead of 27 times; every thread then evaluates exactly the same arithmetic as
// node_apply3 from LDS.
// ----------------------------------------------------------------------------------
constexpr int H3X = T3X + 2, H3Y = T3Y + 2, H3Z = T3Z + 2;
constexpr int H3N = H3X * H3Y * H3Z;                    // halo nodes per tile
// LDS row stride of the halo: for float, 16 (mod 32) words, so that the two y-rows of
// nodes a half-wave reads fall on disjoint banks; double keeps the dense stride (the
// larger tile would cost occupancy)
template <typename T> struct Tile3Stride { static constexpr int X = sizeof(T) == 4 ? 48 : H3X; };
template <typename T>
__host__ __device__ constexpr int tile3_slot(int q) {
    return q + (q / H3X) * (Tile3Stride<T>::X - H3X);
}
constexpr int E3X = T3X + 1, E3Y = T3Y + 1, E3Z = T3Z + 1;
constexpr int E3N = E3X * E3Y * E3Z;                    // element alphas per tile

template <typename T>
struct Tile3Lds {
    static constexpr int SX = Tile3Stride<T>::X;
    T x[3][SX * H3Y * H3Z];
    T al[E3N];
};

// origin of tile t and this thread's node inside it
__device__ __forceinline__ void tile3_origin(const Grid& g, int t, int& i0, int& j0, int& k0) {
    const int ntx = (g.nx1 + T3X - 1) / T3X, nty = (g.ny1 + T3Y - 1) / T3Y;
    i0 = (t % ntx) * T3X;
    j0 = ((t / ntx) % nty) * T3Y;
    k0 = (t / (ntx * nty)) * T3Z;
}

// Stage the element alphas of the tile (zero outside the grid).
template <typename T>
__device__ __forceinline__ void tile3_load_alpha(const Grid& g, int i0, int j0, int k0,
                                                 const T* __restrict__ alpha, Tile3Lds<T>& L) {
    for (int q = threadIdx.x; q < E3N; q += blockDim.x) {
        const int ex = q % E3X, ey = (q / E3X) % E3Y, ez = q / (E3X * E3Y);
        const int exx = i0 - 1 + ex, eyy = j0 - 1 + ey, ezz = k0 - 1 + ez;
        const bool ok = (exx >= 0) & (exx < g.nx) & (eyy >= 0) & (eyy < g.ny) & (ezz >= 0) & (ezz < g.nz);
        L.al[q] = ok ? alpha[((size_t)ezz * g.ny + eyy) * g.nx + exx] : T(0);
    }
}

// Halo position q of the tile -> global node (or -1 outside the grid).
__device__ __forceinline__ int tile3_halo_node(const Grid& g, int i0, int j0, int k0, int q) {
    const int hx = q % H3X, hy = (q / H3X) % H3Y, hz = q / (H3X * H3Y);
    const int ii = i0 - 1 + hx, jj = j0 - 1 + hy, kk = k0 - 1 + hz;
    const bool ok = (ii >= 0) & (ii < g.nx1) & (jj >= 0) & (jj < g.ny1) & (kk >= 0) & (kk < g.nz1);
    return ok ? (kk * g.ny1 + jj) * g.nx1 + ii : -1;
}

// This thread's node inside the tile.
__device__ __forceinline__ void tile3_thread(int& tx, int& ty, int& tz) {
    tx = threadIdx.x % T3X;
    ty = (threadIdx.x / T3X) % T3Y;
    tz = threadIdx.x / (T3X * T3Y);
}

// Stage the halo values given by `fetch` (zero outside the grid).
template <typename T, typename Fetch>
__device__ __forceinline__ void tile3_stage(const Grid& g, int i0, int j0, int k0,
                                            const Fetch& fetch, Tile3Lds<T>& L) {
    for (int q = threadIdx.x; q < H3N; q += blockDim.x) {
        const int n = tile3_halo_node(g, i0, j0, k0, q);
#pragma unroll
        for (int c = 0; c < 3; ++c) L.x[c][tile3_slot<T>(q)] = n >= 0 ? fetch(n, c) : T(0);
    }
}

// out[c] for this thread's node from the staged tile (same arithmetic as node_apply3).
template <typename T>
__device__ __forceinline__ void tile3_compute(const Tile3Lds<T>& L, const T* __restrict__ K,
                                              int tx, int ty, int tz, T (&out)[3]) {
    T xs[3][3][3][3];
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int q = ((tz + dz) * H3Y + (ty + dy)) * Tile3Lds<T>::SX + (tx + dx);
#pragma unroll
                for (int c = 0; c < 3; ++c) xs[dz][dy][dx][c] = L.x[c][q];
            }
    {
        const T c0 = xs[1][1][1][0], c1 = xs[1][1][1][1], c2 = xs[1][1][1][2];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz)
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    xs[dz][dy][dx][0] -= c0;
                    xs[dz][dy][dx][1] -= c1;
                    xs[dz][dy][dx][2] -= c2;
                }
    }
    out[0] = out[1] = out[2] = T(0);
#pragma unroll
    for (int ez = 0; ez < 2; ++ez)
#pragma unroll
        for (int ey = 0; ey < 2; ++ey)
#pragma unroll
            for (int ex = 0; ex < 2; ++ex) {
                const T al = L.al[((tz + ez) * E3Y + (ty + ey)) * E3X + (tx + ex)];
                const int a = (1 - ex) + 2 * (1 - ey) + 4 * (1 - ez);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T* row = K + (3 * a + c) * 24;
                    T s = T(0);
#pragma unroll
                    for (int b = 0; b < 8; ++b) {
                        const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
#pragma unroll
                        for (int d = 0; d < 3; ++d)
                            s += row[3 * b + d] * xs[ez + bz][ey + by][ex + bx][d];
                    }
                    out[c] += al * s;
                }
            }
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
    i = n % g.nx1;
    const int t = n / g.nx1;
    j = t % g.ny1;
    k = t / g.ny1;
}

}  // namespace topo
