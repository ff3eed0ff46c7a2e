// Element operator in symmetry-blocked form: K_e = R^T R with R = L^T G H, where H is
// the Walsh-Hadamard transform of the nodal values over the element's 2^dim nodes
// (one per displacement component), G picks / combines the transformed values of one
// reflection character and drops the rigid translations and rotations exactly, and
// L^T is the upper-triangular Cholesky factor of the remaining block (Sec. 2.1 gives
// K_e; the factor itself is computed on the host from it, see element_factor).
//
// The transformed values are formed from edge differences only, so that a large
// common displacement never enters the arithmetic: N[m][c] = -sum_a (-1)^{m.a} A[a][c]
// for m != 0, with a = ax + 2 ay + 4 az.  (The overall sign is irrelevant wherever R
// appears as R^T R.)
#pragma once

#include "internal.hpp"

namespace topo {

constexpr int kRows2 = 5;   // rank of the Q4 element operator
constexpr int kRows3 = 18;  // rank of the H8 element operator

template <typename T>
__device__ __forceinline__ void neg_wht3(const T (&A)[8][3], T (&N)[8][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // edge differences along x (indexed by y, z), y (by x, z), z (by x, y)
        const T dx00 = A[1][c] - A[0][c], dx10 = A[3][c] - A[2][c];
        const T dx01 = A[5][c] - A[4][c], dx11 = A[7][c] - A[6][c];
        const T dy00 = A[2][c] - A[0][c], dy10 = A[3][c] - A[1][c];
        const T dy01 = A[6][c] - A[4][c], dy11 = A[7][c] - A[5][c];
        const T dz00 = A[4][c] - A[0][c], dz10 = A[5][c] - A[1][c];
        const T dz01 = A[6][c] - A[2][c], dz11 = A[7][c] - A[3][c];
        const T s0 = dx00 + dx01, s1 = dx10 + dx11, t0 = dx00 - dx01, t1 = dx10 - dx11;
        N[1][c] = s0 + s1;
        N[3][c] = s0 - s1;
        N[5][c] = t0 + t1;
        N[7][c] = t0 - t1;
        const T u0 = dy00 + dy10, u1 = dy01 + dy11;
        N[2][c] = u0 + u1;
        N[6][c] = u0 - u1;
        N[4][c] = (dz00 + dz10) + (dz01 + dz11);
        N[0][c] = T(0);
    }
}

// Upper-triangular 3x3 / 2x2 / 1x1 products with the factor slots of block n.
template <typename T>
__device__ __forceinline__ void tri3(const T* F, int n, T z0, T z1, T z2, T* D) {
    D[0] = F[6 * n + 0] * z0 + F[6 * n + 1] * z1 + F[6 * n + 2] * z2;
    D[1] = F[6 * n + 3] * z1 + F[6 * n + 4] * z2;
    D[2] = F[6 * n + 5] * z2;
}
template <typename T>
__device__ __forceinline__ void tri2(const T* F, int n, T z0, T z1, T* D) {
    D[0] = F[6 * n + 0] * z0 + F[6 * n + 1] * z1;
    D[1] = F[6 * n + 3] * z1;
}

// D = s * L^T G N (= -s R A when N = neg_wht3(A)).
template <typename T>
__device__ __forceinline__ void rows3_from_n(const T (&N)[8][3], const T* __restrict__ F, T s,
                                             T (&D)[kRows3]) {
    const T h0 = F[kFacH], h1 = F[kFacH + 1], h2 = F[kFacH + 2];
    tri3(F, 0, N[1][0], N[2][1], N[4][2], D + 0);              // normal strains
    tri2(F, 1, N[3][1], N[5][2], D + 3);                       // x translation dropped
    tri2(F, 2, N[3][0], N[6][2], D + 5);                       // y translation dropped
    tri2(F, 3, h0 * N[2][0] + h1 * N[1][1], N[7][2], D + 7);   // rotation about z dropped
    tri2(F, 4, N[5][0], N[6][1], D + 9);                       // z translation dropped
    tri2(F, 5, h0 * N[4][0] + h2 * N[1][2], N[7][1], D + 11);  // rotation about y dropped
    tri2(F, 6, h1 * N[4][1] + h2 * N[2][2], N[7][0], D + 13);  // rotation about x dropped
    tri3(F, 7, N[6][0], N[5][1], N[3][2], D + 15);
#pragma unroll
    for (int r = 0; r < kRows3; ++r) D[r] *= s;
}

// D = s * R A for one column: A[a][c] nodal values of the H8 element, F its factor.
template <typename T>
__device__ __forceinline__ void elem_rows3(const T (&A)[8][3], const T* __restrict__ F, T s,
                                           T (&D)[kRows3]) {
    T N[8][3];
    neg_wht3(A, N);
    rows3_from_n(N, F, s, D);
}

// Y = s K_e A for one element from N = neg_wht3(A), with the reduced blocks M = L L^T
// (table Mt: upper triangles in the factor's slots, element sizes at kFacH):
// z = G N, u = -s M z, V = G^T u, Y = H V.  The same product as applying R^T after R,
// with one symmetric block product in place of the two triangular ones.
template <typename T>
__device__ __forceinline__ void apply3_from_n(const T (&N)[8][3], const T* __restrict__ Mt, T s,
                                              T (&Y)[8][3]) {
    const T h0 = Mt[kFacH], h1 = Mt[kFacH + 1], h2 = Mt[kFacH + 2];
    const T ns = -s;
    auto sym3 = [&](int n, T z0, T z1, T z2, T& u0, T& u1, T& u2) {
        z0 *= ns;
        z1 *= ns;
        z2 *= ns;
        u0 = Mt[6 * n + 0] * z0 + Mt[6 * n + 1] * z1 + Mt[6 * n + 2] * z2;
        u1 = Mt[6 * n + 1] * z0 + Mt[6 * n + 3] * z1 + Mt[6 * n + 4] * z2;
        u2 = Mt[6 * n + 2] * z0 + Mt[6 * n + 4] * z1 + Mt[6 * n + 5] * z2;
    };
    auto sym2 = [&](int n, T z0, T z1, T& u0, T& u1) {
        z0 *= ns;
        z1 *= ns;
        u0 = Mt[6 * n + 0] * z0 + Mt[6 * n + 1] * z1;
        u1 = Mt[6 * n + 1] * z0 + Mt[6 * n + 3] * z1;
    };
    T V[8][3];
    T u0, u1, u2;
    V[0][0] = V[0][1] = V[0][2] = T(0);
    sym3(0, N[1][0], N[2][1], N[4][2], u0, u1, u2);                 // normal strains
    V[1][0] = u0; V[2][1] = u1; V[4][2] = u2;
    sym2(1, N[3][1], N[5][2], u0, u1);                              // x translation dropped
    V[3][1] = u0; V[5][2] = u1;
    sym2(2, N[3][0], N[6][2], u0, u1);                              // y translation dropped
    V[3][0] = u0; V[6][2] = u1;
    sym2(3, h0 * N[2][0] + h1 * N[1][1], N[7][2], u0, u1);          // rotation about z dropped
    V[2][0] = h0 * u0; V[1][1] = h1 * u0; V[7][2] = u1;
    sym2(4, N[5][0], N[6][1], u0, u1);                              // z translation dropped
    V[5][0] = u0; V[6][1] = u1;
    sym2(5, h0 * N[4][0] + h2 * N[1][2], N[7][1], u0, u1);          // rotation about y dropped
    V[4][0] = h0 * u0; V[1][2] = h2 * u0; V[7][1] = u1;
    sym2(6, h1 * N[4][1] + h2 * N[2][2], N[7][0], u0, u1);          // rotation about x dropped
    V[4][1] = h1 * u0; V[2][2] = h2 * u0; V[7][0] = u1;
    sym3(7, N[6][0], N[5][1], N[3][2], u0, u1, u2);
    V[6][0] = u0; V[5][1] = u1; V[3][2] = u2;
    // Y[a][c] = sum_m (-1)^{m.a} V[m][c]
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T w[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) w[m] = V[m][c];
#pragma unroll
        for (int bit = 1; bit < 8; bit <<= 1)
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (!(m & bit)) {
                    const T x0 = w[m], x1 = w[m | bit];
                    w[m] = x0 + x1;
                    w[m | bit] = x0 - x1;
                }
#pragma unroll
        for (int a = 0; a < 8; ++a) Y[a][c] = w[a];
    }
}

// D = s * R A for one column of the Q4 element (a = ax + 2 ay).
template <typename T>
__device__ __forceinline__ void elem_rows2(const T (&A)[4][2], const T* __restrict__ F, T s,
                                           T (&D)[kRows2]) {
    T N1[2], N2[2], N3[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T dx0 = A[1][c] - A[0][c], dx1 = A[3][c] - A[2][c];
        const T dy0 = A[2][c] - A[0][c], dy1 = A[3][c] - A[1][c];
        N1[c] = dx0 + dx1;
        N3[c] = dx0 - dx1;
        N2[c] = dy0 + dy1;
    }
    const T h0 = F[kFacH], h1 = F[kFacH + 1];
    tri2(F, 0, N1[0], N2[1], D + 0);   // normal strains
    D[2] = F[6] * N3[1];               // x translation dropped
    D[3] = F[12] * N3[0];              // y translation dropped
    D[4] = F[18] * (h0 * N2[0] + h1 * N1[1]);  // rotation dropped
#pragma unroll
    for (int r = 0; r < kRows2; ++r) D[r] *= s;
}

}  // namespace topo
