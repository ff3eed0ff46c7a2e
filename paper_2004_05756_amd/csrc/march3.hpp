// Element-centric 3D apply, marching along z (Sec. 2.1: K(rho) x = sum_e alpha_e
// P_e K_e P_e^T x).  A block owns a column of 31 x 7 node columns (one 32 x 8 tile of
// element columns, one element per thread, the extra row and column being the
// neighbours the owned nodes also touch) over KZ node planes.  For each element layer
// it stages the next node plane (33 x 9 nodes) in LDS, every thread evaluates its
// element with the symmetry-blocked factor (about 210 operations instead of the 576
// multiply-adds of the dense element rows), and each owned node sums the four corner
// contributions of the layer below and the four of the layer above in a fixed order
// (deterministic, no atomics).
#pragma once

#include "elemfac.hpp"

namespace topo {

constexpr int MPX = MEX + 1, MPY = MEY + 1;         // staged node plane
constexpr int MPN = MPX * MPY;                      // 297 nodes
static_assert(MEX * MEY == kBlock, "one thread per element column");

struct MarchBlock {
    int i0, j0, k0, k1;  // owned nodes: [i0, i0+31) x [j0, j0+7) x [k0, k1)
};

__device__ __forceinline__ MarchBlock march3_block(const Grid& g, int b) {
    const int tx = march3_tiles_x(g), ty = march3_tiles_y(g), kz = march3_kz(g);
    MarchBlock m;
    m.i0 = (b % tx) * MOX;
    m.j0 = ((b / tx) % ty) * MOY;
    m.k0 = (b / (tx * ty)) * kz;
    m.k1 = min(m.k0 + kz, g.nz1);
    return m;
}

template <typename T>
struct MarchLds {
    T plane[2][3][MPN];   // node planes, double-buffered
    T xch[3][4][kBlock];  // corner sums of the current node plane [c][corner][thread]
    T F[kFacSize];
};

// Node of plane slot q at node plane k, or -1 outside the grid.
__device__ __forceinline__ int march3_node(const Grid& g, const MarchBlock& m, int q, int k) {
    const int px = q % MPX, py = q / MPX;
    const int i = m.i0 - 1 + px, j = m.j0 - 1 + py;
    const bool ok = (i >= 0) & (i < g.nx1) & (j >= 0) & (j < g.ny1) & (k >= 0) & (k < g.nz1);
    return ok ? (k * g.ny1 + j) * g.nx1 + i : -1;
}

// The march.  Src (per plane slot, this thread's two slots):
//   fetch(int slot_index, int node)  issue the loads of node (node may be -1: zero)
//   value(int slot_index, int c)     the fetched value
// Emit (owned nodes, in node-plane order):
//   emit(int node, const T (&y)[3], const T (&xn)[3])  y = (K x)(node), xn = x(node)
// The caller has fetched planes k0-1 (set 0) and k0 (set 1) and calls with them.
template <typename T, typename Src, typename Emit>
__device__ __forceinline__ void march3_run(const Grid& g, const MarchBlock& m,
                                           const T* __restrict__ alpha, MarchLds<T>& L,
                                           Src& src, Emit& emit) {
    const int tid = threadIdx.x;
    const int tx = tid % MEX, ty = tid / MEX;
    const int ex = m.i0 - 1 + tx, ey = m.j0 - 1 + ty;
    const bool exy = (ex >= 0) & (ex < g.nx) & (ey >= 0) & (ey < g.ny);
    // commit the two prologue planes (src sets 0, 1) to LDS buffers 0, 1
#pragma unroll
    for (int set = 0; set < 2; ++set)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int q = tid + r * kBlock;
            if (q < MPN)
#pragma unroll
                for (int c = 0; c < 3; ++c) L.plane[set][c][q] = src.value(2 * set + r, c);
        }
    const int K = m.k1 - m.k0;
    T top[4][3];
#pragma unroll
    for (int v = 0; v < 4; ++v) top[v][0] = top[v][1] = top[v][2] = T(0);
    T al_next = T(0);
    {
        const int ez = m.k0 - 1;
        if (exy && ez >= 0 && ez < g.nz) al_next = alpha[((size_t)ez * g.ny + ey) * g.nx + ex];
    }
    for (int s = 0; s <= K; ++s) {
        const int ez = m.k0 - 1 + s;  // element layer between node planes ez and ez + 1
        const int bot = s & 1, topb = (s + 1) & 1;
        if (s >= 1) {
            // plane ez + 1, fetched during the previous step, into buffer topb
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int q = tid + r * kBlock;
                if (q < MPN)
#pragma unroll
                    for (int c = 0; c < 3; ++c) L.plane[topb][c][q] = src.value(r, c);
            }
        }
        __syncthreads();
        // loads for the next step: node plane ez + 2 and the next layer's alpha
        const T al = al_next;
        if (s < K) {
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int q = tid + r * kBlock;
                src.fetch(r, q < MPN ? march3_node(g, m, q, ez + 2) : -1);
            }
            const int ezn = ez + 1;
            al_next = (exy && ezn < g.nz) ? alpha[((size_t)ezn * g.ny + ey) * g.nx + ex] : T(0);
        }
        // this thread's element: nodes a = ax + 2 ay + 4 az
        T A[8][3], Y[8][3];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int q = (ty + ((a >> 1) & 1)) * MPX + tx + (a & 1);
            const int buf = (a >> 2) ? topb : bot;
#pragma unroll
            for (int c = 0; c < 3; ++c) A[a][c] = L.plane[buf][c][q];
        }
        elem_apply3(A, L.F, al, Y);
        // node plane ez: corner sums of the layer below (top) and this layer (bottom)
        T xn[3];
        if (s >= 1) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int c = 0; c < 3; ++c) L.xch[c][v][tid] = top[v][c] + Y[v][c];
#pragma unroll
            for (int c = 0; c < 3; ++c) xn[c] = L.plane[bot][c][ty * MPX + tx];
        }
        __syncthreads();
        if (s >= 1 && tx >= 1 && ty >= 1) {
            const int i = m.i0 - 1 + tx, j = m.j0 - 1 + ty;
            if (i < g.nx1 && j < g.ny1) {
                T y[3];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    y[c] = (L.xch[c][3][tid - MEX - 1] + L.xch[c][2][tid - MEX]) +
                           (L.xch[c][1][tid - 1] + L.xch[c][0][tid]);
                emit((ez * g.ny1 + j) * g.nx1 + i, y, xn);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int c = 0; c < 3; ++c) top[v][c] = Y[v + 4][c];
    }
}

}  // namespace topo
