// Element-centric 3D apply, marching along z (Sec. 2.1: K(rho) x = sum_e alpha_e
// P_e K_e P_e^T x).  A block owns a column of 31 x 7 node columns (one 32 x 8 tile of
// element columns, one element per thread, the extra row and column being the
// neighbours the owned nodes also touch) over KZ node planes.  For each element layer
// it stages the next node plane (33 x 9 nodes) in LDS, every thread evaluates its
// element in the symmetry-blocked form (edge differences, one symmetric product per
// reflection block, the Walsh-Hadamard transform back: under 200 operations instead of
// the 576 multiply-adds of the dense element rows), and each owned node sums the four corner
// contributions of the layer below and the four of the layer above in a fixed order
// (deterministic, no atomics).
#pragma once

#include <type_traits>

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
    T M[kFacSize];  // reduced blocks of the element operator (apply3_from_n)
};

// Plane slots of this thread (q = tid and tid + kBlock): the node index at plane 0
// (or -1 when the column lies outside the grid); plane k adds k * (nx1 * ny1).
struct MarchSlots {
    int base[2];
    int pstride;
};

__device__ __forceinline__ MarchSlots march3_slots(const Grid& g, const MarchBlock& m) {
    MarchSlots sl;
    sl.pstride = g.nx1 * g.ny1;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int q = threadIdx.x + r * kBlock;
        const int px = q % MPX, py = q / MPX;
        const int i = m.i0 - 1 + px, j = m.j0 - 1 + py;
        const bool ok = (q < MPN) & (i >= 0) & (i < g.nx1) & (j >= 0) & (j < g.ny1);
        sl.base[r] = ok ? j * g.nx1 + i : -1;
    }
    return sl;
}

// Node of slot r at node plane k, or -1.
__device__ __forceinline__ int march3_node(const Grid& g, const MarchSlots& sl, int r, int k) {
    return (sl.base[r] >= 0 && k >= 0 && k < g.nz1) ? sl.base[r] + k * sl.pstride : -1;
}

// Per face (the 4 nodes f = fx + 2 fy of one z level of an element) and component:
// the sum and the y-alternating difference of its two x-edge differences, and the sum
// of its two y-edge differences.  Shared by the element below and the one above.
template <typename T>
struct FaceSums {
    T X[3], Xs[3], Y[3];
};

template <typename T>
__device__ __forceinline__ void face_sums(const T (&a)[4][3], FaceSums<T>& f) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T dx0 = a[1][c] - a[0][c], dx1 = a[3][c] - a[2][c];
        const T dy0 = a[2][c] - a[0][c], dy1 = a[3][c] - a[1][c];
        f.X[c] = dx0 + dx1;
        f.Xs[c] = dx0 - dx1;
        f.Y[c] = dy0 + dy1;
    }
}

// N = neg_wht3 of the element from its bottom (b) and top (t) faces.
template <typename T>
__device__ __forceinline__ void neg_wht3_faces(const T (&ab)[4][3], const T (&at)[4][3],
                                               const FaceSums<T>& fb, const FaceSums<T>& ft,
                                               T (&N)[8][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        N[0][c] = T(0);
        N[1][c] = fb.X[c] + ft.X[c];
        N[3][c] = fb.Xs[c] + ft.Xs[c];
        N[5][c] = fb.X[c] - ft.X[c];
        N[7][c] = fb.Xs[c] - ft.Xs[c];
        N[2][c] = fb.Y[c] + ft.Y[c];
        N[6][c] = fb.Y[c] - ft.Y[c];
        N[4][c] = ((at[0][c] - ab[0][c]) + (at[1][c] - ab[1][c])) +
                  ((at[2][c] - ab[2][c]) + (at[3][c] - ab[3][c]));
    }
}

// The march.  Src (this thread's two plane slots):
//   fetch(int slot_index, int node)  issue the loads of node (node may be -1: zero)
//   value(int slot_index, int c)     the fetched value
// Emit (owned nodes, in node-plane order):
//   emit(int node, const T (&y)[3], const T (&xn)[3])  y = (K x)(node), xn = x(node)
// The caller has fetched planes k0-1 (slots 0, 1) and k0 (slots 2, 3).
template <typename T, typename Src, typename Emit>
__device__ __forceinline__ void march3_run(const Grid& g, const MarchBlock& m,
                                           const MarchSlots& sl, const T* __restrict__ alpha,
                                           MarchLds<T>& L, Src& src, Emit& emit) {
    const int tid = threadIdx.x;
    const int tx = tid % MEX, ty = tid / MEX;
    const int ex = m.i0 - 1 + tx, ey = m.j0 - 1 + ty;
    const bool exy = (ex >= 0) & (ex < g.nx) & (ey >= 0) & (ey < g.ny);
    const int abase = exy ? ey * g.nx + ex : 0;
    const int astride = g.nx * g.ny;
    // commit the two prologue planes to LDS buffers 0, 1
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
    auto alpha_at = [&](int ez) -> T {
        const bool ok = exy && ez >= 0 && ez < g.nz;
        const T a = alpha[ok ? (size_t)ez * astride + abase : 0];
        return ok ? a : T(0);
    };
    T al_next = alpha_at(m.k0 - 1);
    T ab[4][3];        // bottom face of the current element (carried from the step before)
    FaceSums<T> fb;
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
            for (int r = 0; r < 2; ++r) src.fetch(r, march3_node(g, sl, r, ez + 2));
            al_next = alpha_at(ez + 1);
        }
        if (s == 0) {
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int q = (ty + (f >> 1)) * MPX + tx + (f & 1);
#pragma unroll
                for (int c = 0; c < 3; ++c) ab[f][c] = L.plane[bot][c][q];
            }
            face_sums(ab, fb);
        }
        T at[4][3];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int q = (ty + (f >> 1)) * MPX + tx + (f & 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) at[f][c] = L.plane[topb][c][q];
        }
        FaceSums<T> ft;
        face_sums(at, ft);
        T N[8][3], Y[8][3];
        neg_wht3_faces(ab, at, fb, ft, N);
        apply3_from_n(N, L.M, al, Y);
        // node plane ez: corner sums of the layer below (top) and this layer (bottom)
        if (s >= 1) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int c = 0; c < 3; ++c) L.xch[c][v][tid] = top[v][c] + Y[v][c];
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
                emit((ez * g.ny1 + j) * g.nx1 + i, y, ab[0]);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                top[v][c] = Y[v + 4][c];
                ab[v][c] = at[v][c];
            }
        fb = ft;
    }
}

}  // namespace topo

namespace topo {

// ----------------------------------------------------------------------------------
// Element-once march.  The block's tile is elements [ex0, ex0+32) x [ey0, ey0+8) over
// element layers [ez0, ez1); its node planes are the 33 x 9 nodes [ex0, ex0+32] x
// [ey0, ey0+8].  Each element layer is evaluated once, every node of the plane below it
// is emitted with the corner sums of the (up to) four tile elements of the layer below
// and the four of the layer above, and the top plane of the chunk is emitted with the
// last layer's corners alone.  The corner exchange has a zero border (34 x 10 slots per
// corner and component) so that a node of the tile's edge reads the missing elements as
// zeros without a test.
// ----------------------------------------------------------------------------------
constexpr int OXX = MEX + 2;              // padded exchange row
constexpr int OXN = OXX * (MEY + 2);      // 340 slots

template <typename T>
struct OnceLds {
    T plane[3][3][MPN];   // node planes, triple-buffered (plane k in buffer (k - ez0) % 3)
    T xch[3][4][OXN];     // corner sums [c][corner][padded element slot]
};

struct OnceBlock {
    int ex0, ey0, ez0, ez1;
};

__device__ __forceinline__ OnceBlock once3_block(const Grid& g, int b) {
    const int tx = once3_tiles_x(g), ty = once3_tiles_y(g), kz = once3_kz(g);
    OnceBlock m;
    m.ex0 = (b % tx) * MEX;
    m.ey0 = ((b / tx) % ty) * MEY;
    m.ez0 = (b / (tx * ty)) * kz;
    m.ez1 = min(m.ez0 + kz, g.nz);
    return m;
}

// Plane slots q = tid, tid + kBlock of the tile's node plane (px = q % 33, py = q / 33).
__device__ __forceinline__ MarchSlots once3_slots(const Grid& g, const OnceBlock& m) {
    MarchSlots sl;
    sl.pstride = g.nx1 * g.ny1;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int q = threadIdx.x + r * kBlock;
        const int i = m.ex0 + q % MPX, j = m.ey0 + q / MPX;
        const bool ok = (q < MPN) & (i < g.nx1) & (j < g.ny1);
        sl.base[r] = ok ? j * g.nx1 + i : -1;
    }
    return sl;
}

// Side section of node slot q at node plane k for this block: 0 when the block is the
// node's primary, else the bits of the high faces the node lies on.
__device__ __forceinline__ int once3_section(const Grid& g, const OnceBlock& m, int q, int k) {
    const int px = q % MPX, py = q / MPX;
    return (px == MEX && m.ex0 + MEX < g.nx ? 1 : 0) | (py == MEY && m.ey0 + MEY < g.ny ? 2 : 0) |
           (k == m.ez1 && k < g.nz ? 4 : 0);
}

// Node of slot r at node plane k for the element-once march, clamped to a node of the
// grid: a slot outside the grid (ragged tile) reads some node's finite values, which
// reach only the elements outside the mesh, whose alpha is zero.
__device__ __forceinline__ unsigned once3_node(const MarchSlots& sl, int r, int k) {
    return (unsigned)((sl.base[r] >= 0 ? sl.base[r] : 0) + k * sl.pstride);
}

// The march.  Src:
//   Index                           index type of its arrays and of alpha
//   fetch(int slot, unsigned node)  issue the loads of node
//   value(int slot, int c)          the fetched value
// the caller has fetched planes ez0 (slots 0, 1) and ez0 + 1 (slots 2, 3).  Emit:
//   emit<TOP>(int r, int k, int buf, const T (&y)[3])  y = this block's part of (K x)
//                  at the node of slot r at plane k, whose values x are in L.plane[buf]
//                  (a plane buffer is written again only two layers later, after a
//                  barrier every emitter of that plane has passed); TOP: k is the
//                  chunk's top plane
// Mt: the reduced element blocks (apply3_from_n).  Barriers per element layer: after the
// plane is staged and after the corner exchange.
template <typename T, typename Src, typename Emit>
__device__ __forceinline__ void once3_run(const Grid& g, const OnceBlock& m, const MarchSlots& sl,
                                          const T* __restrict__ alpha, OnceLds<T>& L, Src& src,
                                          Emit& E, const T* Mt) {
    using I = typename Src::Index;
    const int tid = threadIdx.x;
    const int tx = tid % MEX, ty = tid / MEX;
    const int ex = m.ex0 + tx, ey = m.ey0 + ty;
    const bool exy = (ex < g.nx) & (ey < g.ny);
    const unsigned abase = exy ? ey * g.nx + ex : 0;
    const unsigned astride = g.nx * g.ny;
    const int xs = (ty + 1) * OXX + tx + 1;  // this element's exchange slot
    for (int i = tid; i < 3 * 4 * OXN; i += kBlock) (&L.xch[0][0][0])[i] = T(0);
#pragma unroll
    for (int set = 0; set < 2; ++set)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int q = tid + r * kBlock;
            if (q < MPN)
#pragma unroll
                for (int c = 0; c < 3; ++c) L.plane[set][c][q] = src.value(2 * set + r, c);
        }
    const int K = m.ez1 - m.ez0;
    T al_next = exy ? ld_at(alpha, (I)(m.ez0 * astride + abase)) : T(0);
    // every valid node slot of plane k (plane buffer buf): the sum of the four tile
    // elements around it (zero border outside the tile)
    auto emit_plane = [&](int k, int buf, auto top_plane) __attribute__((always_inline)) {
        constexpr bool TOP = decltype(top_plane)::value;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int q = tid + r * kBlock;
            if (sl.base[r] >= 0) {
                const int o = (q / MPX) * OXX + q % MPX;
                T y[3];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    y[c] = (L.xch[c][3][o] + L.xch[c][2][o + 1]) + (L.xch[c][1][o + OXX] + L.xch[c][0][o + OXX + 1]);
                E.template emit<TOP>(r, k, buf, y);
            }
        }
    };
    int bot = 0, topb = 1;  // buffers of node planes ez and ez + 1
    // one element layer s: the bottom face's edge sums fb in, the top face's ft out; the
    // upper corners of the layer below in top, replaced by this layer's (each entry read
    // before it is replaced)
    auto layer = [&](int s, const FaceSums<T>& fb, FaceSums<T>& ft, T (&top)[4][3])
                     __attribute__((always_inline)) {
        const int ez = m.ez0 + s;  // element layer between node planes ez and ez + 1
        if (s >= 1) {
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int q = tid + r * kBlock;
                if (q < MPN)
#pragma unroll
                    for (int c = 0; c < 3; ++c) L.plane[topb][c][q] = src.value(r, c);
            }
        }
        __syncthreads();
        const T al = al_next;
        if (s + 1 < K) {
#pragma unroll
            for (int r = 0; r < 2; ++r) src.fetch(r, once3_node(sl, r, ez + 2));
            al_next = exy ? ld_at(alpha, (I)((ez + 1) * astride + abase)) : T(0);
        }
        // the top face from the plane just staged; the bottom face again from its plane
        // (still in buffer bot), for the z-edge differences
        T at[4][3], ab[4][3];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int q = (ty + (f >> 1)) * MPX + tx + (f & 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                at[f][c] = L.plane[topb][c][q];
                ab[f][c] = L.plane[bot][c][q];
            }
        }
        face_sums(at, ft);
        T N[8][3], Y[8][3];
        neg_wht3_faces(ab, at, fb, ft, N);
        apply3_from_n(N, Mt, al, Y);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                L.xch[c][v][xs] = top[v][c] + Y[v][c];
                top[v][c] = Y[v + 4][c];
            }
        __syncthreads();
        emit_plane(ez, bot, std::false_type{});
        bot = topb;
        topb = topb == 2 ? 0 : topb + 1;
    };
    T top[4][3];
    FaceSums<T> sa, sb;
#pragma unroll
    for (int v = 0; v < 4; ++v) top[v][0] = top[v][1] = top[v][2] = T(0);
    __syncthreads();  // the prologue planes are staged
    {
        T fa[4][3];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int q = (ty + (f >> 1)) * MPX + tx + (f & 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) fa[f][c] = L.plane[0][c][q];
        }
        face_sums(fa, sa);
    }
    for (int s = 0; s < K; ++s) {
        layer(s, sa, sb, top);
        sa = sb;
    }
    // the chunk's top node plane (buffer bot now): the last layer's upper corners only,
    // written once every thread has emitted the plane below
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int c = 0; c < 3; ++c) L.xch[c][v][xs] = top[v][c];
    __syncthreads();
    emit_plane(m.ez1, bot, std::true_type{});
}

}  // namespace topo
