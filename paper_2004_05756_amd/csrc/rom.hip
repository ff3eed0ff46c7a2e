// Reduced-order model on the device (Sec. 3.1, 3.3, 3.4):
//   K_hat[b] = sum_e alpha_be (P_e^T Phi)^T K_e (P_e^T Phi)  -- per-element contraction
//              on the matrix cores (v_mfma 16x16x4, f32 or f64)
//   f_hat    = Phi^T f
//   y_hat    = K_hat^{-1} f_hat (float64 Cholesky), J_k = f_hat^T y_hat
//   ||f - K(rho) Phi y_hat||  with optional float64 reduced refinement.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "elemfac.hpp"
#include "reduce.hpp"
#include "stencil.hpp"

namespace topo {

int residual_fp64(Ctx* ctx, const Grid& g, const ElemTables* tb, const double* alpha64,
                  const uint8_t* mask, const double* u, const double* f, double* r, int B,
                  double* part, double* out, hipStream_t s);
int alpha_tables(Ctx* ctx, const Grid& g, const topo_mesh& m, const double* rho, int B,
                 double* a64, float* a32, hipStream_t s);

typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// The 16x16x4 float64 instruction takes A[i][kk] from lane i + 16 kk and B[kk][j] from
// lane j + 16 kk; output element D[i][j] lands in lane j + 16 (i % 4), entry i / 4 (rows
// interleaved with stride 4).
template <> struct Mfma<double> {
    typedef f64x4 acc_t;
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

// ----------------------------------------------------------------------------------
// K_hat contraction (Sec. 3.4).  K_hat = sum_e alpha_e Phi_e^T K_e Phi_e = Phi~^T W with
// W = K(rho) Phi~ (Phi~: the basis with its Dirichlet rows dropped, which the apply does
// by itself): the element products are formed once per node row by the batched apply
// (apply_columns, the basis columns as its vectors), and the k x k product over the N_u
// rows runs on the float64 matrix cores.  Both operands come as k rows of ld >= N_u
// entries (zero past N_u), stored as TS (float32 in the mixed build, float64 in the FP64
// one): Pt, the basis transposed (k_basis_rows), and Wt, the apply's output.  The
// product accumulates in float64 whatever TS is: for a basis column with a large
// translation-like part, Phi_i . (K Phi_j) sums terms far larger than the result (the
// translation is annihilated only by the element operators, not term by term), and a
// float32 accumulation lost it (K_hat 1e-2 off on the benchmark's basis).
//   grid.x : chunks of CH DOFs,  grid.y : groups of upper-triangle 16 x 16 tile pairs
// Per slab of SD DOFs the block stages that slab of every row of Pt and Wt in LDS with
// 16-byte loads (the next slab's loads in flight while the current one is multiplied),
// then each of its GW waves accumulates its NT tile pairs K_IJ += Pt_I Wt_J^T, 4 DOFs
// per instruction.  A block writes its chunk's tiles; k_chunk_sum adds the chunks in a
// fixed order.
// ----------------------------------------------------------------------------------
constexpr int GW = 8;       // waves per block
constexpr int MAX_NT = 4;   // most tile pairs per wave: 4 keep the kernel at 120 VGPRs, two
                            // blocks per CU; 6 (160 VGPRs, one block per CU, every slab read
                            // by two pair groups instead of three) took 10.2 against 8.7 ms per
                            // field at k = 200 on 5.4M DOF
constexpr int KP_MAX = 1024; // largest padded basis size
constexpr int GEMM_LD = 64; // the operands' row pitch is a multiple of this

__device__ __forceinline__ void pair_of(int p, int kt, int& I, int& J) {
    // enumerate (I, J), I <= J, row by row
    int i = 0;
    while (p >= kt - i) {
        p -= kt - i;
        ++i;
    }
    I = i;
    J = i + p;
}

// DOFs per staged slab: a multiple of the 4 of one matrix-core step, sized so that a
// slab of KP rows (up to 256, 512 or 1024) is at most 4 16-byte loads per thread and
// operand.  LDS row pitch SD + 2: the 32 lanes of a half-wave read 16 rows x 2 DOFs on
// distinct banks.
template <typename TC>
__host__ __device__ constexpr int gemm_sd(int KP) {
    return (KP <= 256 ? 128 : KP <= 512 ? 64 : 32) / (int)sizeof(TC);
}

template <typename TC> struct Vec16;
template <> struct Vec16<float> {
    typedef float4 type;
    static __device__ __forceinline__ float at(const float4& a, int v) {
        return v == 0 ? a.x : v == 1 ? a.y : v == 2 ? a.z : a.w;
    }
    // a, or zeros (per component: a select of the whole vector goes through memory)
    static __device__ __forceinline__ float4 keep(bool ok, const float4& a) {
        return float4{ok ? a.x : 0.f, ok ? a.y : 0.f, ok ? a.z : 0.f, ok ? a.w : 0.f};
    }
};
template <> struct Vec16<double> {
    typedef double2 type;
    static __device__ __forceinline__ double at(const double2& a, int v) { return v == 0 ? a.x : a.y; }
    static __device__ __forceinline__ double2 keep(bool ok, const double2& a) {
        return double2{ok ? a.x : 0.0, ok ? a.y : 0.0};
    }
};

template <typename TA, int SD, int NT>
__global__ __launch_bounds__(GW * 64) void k_rom_gemm(const TA* __restrict__ Pt, const double* __restrict__ Wt,
                                                     long long ld, long long nu, int k, int KP, int npairs,
                                                     int kt, int ch, double* __restrict__ partials) {
    constexpr int LSD = SD + 2;
    constexpr int NTH = GW * 64;
    constexpr int VA = 16 / sizeof(TA), VB = 2;  // entries per 16-byte load of Pt, of Wt
    constexpr int SVA = SD / VA, SVB = SD / VB;  // loads per row and slab
    constexpr int MAXB = 4;                      // loads per thread for Wt (KP * SVB <= 4 NTH)
    constexpr int MAXA = MAXB * VB / VA;          // and for Pt (KP * SVA <= MAXA NTH)
    static_assert(SD % VA == 0 && SD % VB == 0 && SD % 4 == 0, "slab of whole loads and steps");
    typedef typename Vec16<TA>::type veca_t;
    typedef typename Vec16<double>::type vecb_t;
    extern __shared__ __align__(16) unsigned char smem[];
    double* sB = (double*)smem;          // [KP][LSD] slab of Wt
    TA* sA = (TA*)(sB + (size_t)KP * LSD);  // [KP][LSD] slab of Pt
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long d0 = (long long)blockIdx.x * ch;
    const long long d1 = min(d0 + (long long)ch, nu);
    // this wave's tile pairs; past the last pair a wave repeats tile (0, 0) and drops it
    int myI[NT], myJ[NT];
    const int pbase = blockIdx.y * NT * GW + wave;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int p = pbase + GW * t;
        if (p < npairs) pair_of(p, kt, myI[t], myJ[t]);
        else myI[t] = myJ[t] = 0;
    }
    typedef typename Mfma<double>::acc_t acc_t;
    acc_t acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = acc_t{0, 0, 0, 0};
    // staging: load q = tid + NTH u is row q / SV, entries V (q % SV) .. + V - 1 of the
    // slab; rows >= k read as zeros, and entries past N_u are zeros of the operands (a
    // slab never passes ld, which is a multiple of SD)
    veca_t ra[MAXA];
    vecb_t rb[MAXB];
    const int nqa = KP * SVA, nqb = KP * SVB;
    auto fetch = [&](long long ds) {
#pragma unroll
        for (int u = 0; u < MAXA; ++u) {
            const int q = tid + NTH * u;
            const int r = q / SVA, c = (q % SVA) * VA;
            const bool ok = q < nqa && r < k;
            const size_t off = ok ? (size_t)r * (size_t)ld + (size_t)(ds + c) : 0;
            ra[u] = Vec16<TA>::keep(ok, *(const veca_t*)(Pt + off));
        }
#pragma unroll
        for (int u = 0; u < MAXB; ++u) {
            const int q = tid + NTH * u;
            const int r = q / SVB, c = (q % SVB) * VB;
            const bool ok = q < nqb && r < k;
            const size_t off = ok ? (size_t)r * (size_t)ld + (size_t)(ds + c) : 0;
            rb[u] = Vec16<double>::keep(ok, *(const vecb_t*)(Wt + off));
        }
    };
    fetch(d0);
    const int rl = lane & 15, cl = lane >> 4;  // operand row in the tile, DOF in the step
    for (long long ds = d0; ds < d1; ds += SD) {
        __syncthreads();  // the previous slab is consumed
#pragma unroll
        for (int u = 0; u < MAXA; ++u) {
            const int q = tid + NTH * u;
            if (q < nqa) {
                const int r = q / SVA, c = (q % SVA) * VA;
#pragma unroll
                for (int v = 0; v < VA; ++v) sA[r * LSD + c + v] = Vec16<TA>::at(ra[u], v);
            }
        }
#pragma unroll
        for (int u = 0; u < MAXB; ++u) {
            const int q = tid + NTH * u;
            if (q < nqb) {
                const int r = q / SVB, c = (q % SVB) * VB;
#pragma unroll
                for (int v = 0; v < VB; ++v) sB[r * LSD + c + v] = Vec16<double>::at(rb[u], v);
            }
        }
        __syncthreads();
        if (ds + SD < d1) fetch(ds + SD);  // in flight during the products
#pragma unroll
        for (int s4 = 0; s4 < SD / 4; ++s4) {
            const int c = s4 * 4 + cl;
            double av[NT], bv[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                av[t] = (double)sA[(myI[t] * 16 + rl) * LSD + c];
                bv[t] = sB[(myJ[t] * 16 + rl) * LSD + c];
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = Mfma<double>::run(av[t], bv[t], acc[t]);
        }
    }
    // the chunk's tiles: partials[chunk][pair][16 * 16]
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int p = pbase + GW * t;
        if (p < npairs) {
            double* dst = partials + ((size_t)blockIdx.x * npairs + p) * 256;
#pragma unroll
            for (int v = 0; v < 4; ++v) dst[Mfma<double>::row(lane, v) * 16 + (lane & 15)] = acc[t][v];
        }
    }
}

// Pt[j][d] = Phi[d][j] (j < k, d < N_u), and zeros at N_u <= d < ld: 64 x 64 tiles
// through LDS (reads along the basis rows, writes along the transposed ones).  Also
// zeroes the same tail of Wt's rows (the apply writes only the first N_u entries of each).
template <typename TP>
__global__ __launch_bounds__(256) void k_basis_rows(const TP* __restrict__ phi, int ldphi, long long nu, int k,
                                                    long long ld, TP* __restrict__ Pt, double* __restrict__ Wt) {
    __shared__ TP tile[64][65];
    const long long d0 = (long long)blockIdx.x * 64;
    const int j0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const long long d = d0 + r;
        const int j = j0 + tx;
        tile[r][tx] = (d < nu && j < k) ? phi[(size_t)d * ldphi + j] : TP(0);
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int j = j0 + r;
        const long long d = d0 + tx;
        if (j < k && d < ld) {
            Pt[(size_t)j * ld + d] = tile[tx][r];  // zero past N_u
            if (d >= nu) Wt[(size_t)j * ld + d] = 0.0;
        }
    }
}

// Partial 16 x 16 tiles of K_hat (npairs upper-triangle tile pairs): write the
// symmetric matrix from its upper triangle.
struct KhatOut {
    int k, kt;
    double* Khat;
    __device__ void operator()(int b, int e, double s) const {
        int I, J;
        pair_of(e / 256, kt, I, J);
        const int i = I * 16 + (e % 256) / 16, j = J * 16 + e % 16;
        if (i >= k || j >= k || i > j) return;
        double* Kb = Khat + (size_t)b * k * k;
        Kb[(size_t)i * k + j] = s;
        Kb[(size_t)j * k + i] = s;
    }
};


// ----------------------------------------------------------------------------------
// out[b][j] = sum_i Phi[i][j] v[b][i] over free rows i (float64 accumulation).
// grid.x: row chunks, grid.y: b.  Partials [b][chunk][k], summed by k_chunk_sum.
// ----------------------------------------------------------------------------------
// Phi is row-major, so a tile of rb consecutive rows is one contiguous stretch of
// memory: the block copies it into LDS with coalesced loads (rows padded to an odd
// stride), then thread j accumulates column j over the tile's rows.
template <typename TP>
__device__ __forceinline__ void stage_rows(const TP* __restrict__ phi, int ldphi, long long r0,
                                           int nr, int lds_ld, TP* __restrict__ tile) {
    const TP* src = phi + (size_t)r0 * ldphi;
    const int n = nr * ldphi;
    constexpr int V = 16 / sizeof(TP);  // elements per 16-byte load
    constexpr int U = 4;                // 16-byte loads in flight per thread
    if (((uintptr_t)src & 15) == 0) {
        const int nv = n / V;
        const uint4* s4 = (const uint4*)src;
        for (int q0 = threadIdx.x; q0 < nv; q0 += U * blockDim.x) {
            uint4 w[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * blockDim.x;
                if (q < nv) w[u] = s4[q];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * blockDim.x;
                if (q < nv) {
                    const TP* e = (const TP*)&w[u];
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const int idx = q * V + v;
                        const int r = idx / ldphi, c = idx - r * ldphi;
                        tile[r * lds_ld + c] = e[v];
                    }
                }
            }
        }
        for (int idx = nv * V + threadIdx.x; idx < n; idx += blockDim.x) {
            const int r = idx / ldphi, c = idx - r * ldphi;
            tile[r * lds_ld + c] = src[idx];
        }
    } else {
        for (int idx = threadIdx.x; idx < n; idx += blockDim.x) {
            const int r = idx / ldphi, c = idx - r * ldphi;
            tile[r * lds_ld + c] = src[idx];
        }
    }
}

// Fields of one projection launch share every staged basis tile: a block reads its rows
// of Phi once for a group of up to G fields (grid.y covers further groups); G = 16
// unless the per-thread accumulators or the coefficients in LDS would not fit.

// out[b][j] partials = sum_i Phi[i][j] v[b][i] over the chunk's free rows (float64).
// Thread t accumulates columns t + 256 q (q < CQ) for the group's nf fields.
template <typename TP, int CQ, int G>
__global__ __launch_bounds__(256) void k_phit_v(long long nrows, const TP* __restrict__ phi, int k,
                                                int ldphi, const uint8_t* __restrict__ mask,
                                                const double* __restrict__ v, long long vstride, int B,
                                                int rows_per_chunk, int rb,
                                                double* __restrict__ partials) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lds_ld = ldphi | 1;
    TP* tile = (TP*)smem;                                  // [rb][lds_ld]
    double* sv = (double*)(smem + (((size_t)rb * lds_ld * sizeof(TP) + 15) & ~(size_t)15));  // [nf][rb]
    const int b0 = blockIdx.y * G;
    const int nf = min(G, B - b0);
    const long long r0 = (long long)blockIdx.x * rows_per_chunk;
    const long long r1 = min(r0 + rows_per_chunk, nrows);
    double acc[CQ][G];
#pragma unroll
    for (int q = 0; q < CQ; ++q)
#pragma unroll
        for (int f = 0; f < G; ++f) acc[q][f] = 0.0;
    for (long long t0 = r0; t0 < r1; t0 += rb) {
        const int nr = (int)min((long long)rb, r1 - t0);
        __syncthreads();
        stage_rows(phi, ldphi, t0, nr, lds_ld, tile);
        for (int idx = threadIdx.x; idx < nf * rb; idx += blockDim.x) {
            const int f = idx / rb, r = idx - f * rb;
            sv[idx] = (r < nr && !mask[t0 + r]) ? v[(size_t)(b0 + f) * vstride + t0 + r] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < CQ; ++q) {
            const int j = threadIdx.x + q * blockDim.x;
            if (j < k) {
                for (int r = 0; r < nr; ++r) {
                    const double t = (double)tile[r * lds_ld + j];
#pragma unroll
                    for (int f = 0; f < G; ++f)
                        if (f < nf) acc[q][f] += t * sv[f * rb + r];
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < CQ; ++q) {
        const int j = threadIdx.x + q * blockDim.x;
        if (j < k)
#pragma unroll
            for (int f = 0; f < G; ++f)
                if (f < nf) partials[((size_t)(b0 + f) * gridDim.x + blockIdx.x) * k + j] = acc[q][f];
    }
}

// u[b][i] = Phi[i][:] . y[b][:] on free rows, 0 on Dirichlet rows (float64 accumulation),
// for the group's nf fields.  A block handles a contiguous tile of rb rows (staged in
// LDS with coalesced loads, read once for all the group's fields); 256 / rb threads
// share a row and combine their column sums with lane shuffles.
template <typename TP, int G>
__global__ __launch_bounds__(256) void k_phi_y(long long nrows, const TP* __restrict__ phi, int k,
                                               int ldphi, const uint8_t* __restrict__ mask,
                                               const double* __restrict__ y, int B, int rb,
                                               double* __restrict__ u) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int lds_ld = ldphi | 1;
    const int b0 = blockIdx.y * G;
    const int nf = min(G, B - b0);
    double* sy = (double*)smem;                           // [nf][k]
    TP* tile = (TP*)(sy + (((size_t)G * k + 1) & ~(size_t)1));  // [rb][lds_ld]
    for (int idx = threadIdx.x; idx < nf * k; idx += blockDim.x) sy[idx] = y[(size_t)b0 * k + idx];
    const long long r0 = (long long)blockIdx.x * rb;
    const int nr = (int)min((long long)rb, nrows - r0);
    stage_rows(phi, ldphi, r0, nr, lds_ld, tile);
    __syncthreads();
    const int tpr = blockDim.x / rb;            // threads per row (power of two <= 64)
    const int r = threadIdx.x / tpr, q = threadIdx.x - r * tpr;
    double s[G];
#pragma unroll
    for (int f = 0; f < G; ++f) s[f] = 0.0;
    if (r < nr)
        for (int j = q; j < k; j += tpr) {
            const double t = (double)tile[r * lds_ld + j];
#pragma unroll
            for (int f = 0; f < G; ++f)
                if (f < nf) s[f] += t * sy[f * k + j];
        }
#pragma unroll
    for (int f = 0; f < G; ++f) {
        if (f >= nf) break;
        double x = s[f];
        for (int off = tpr >> 1; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (q == 0 && r < nr) u[(size_t)(b0 + f) * nrows + r0 + r] = mask[r0 + r] ? 0.0 : x;
    }
}

// ----------------------------------------------------------------------------------
// Batched float64 Cholesky K = L L^T (one block of 256 threads per matrix,
// right-looking by column).  Column j is left unscaled at step j: the trailing update
// subtracts A[i][j] A[l][j] / A[j][j], and the output divides each column by the
// square root of its pivot.  status[b] = TOPO_ENOTSPD on a pivot that is not positive
// relative to the largest original diagonal entry (that pivot is then taken as 1).
//
// k <= CHOL_REG_MAX_K: the lower triangle lives in registers on a 16 x 16 thread grid
// (thread (ty, tx) holds rows ty + 16 r, columns tx + 16 c, c <= r).  At step j the 16
// threads holding column j publish it through a double-buffered LDS vector, and after
// one barrier every thread updates its own entries.  Larger k works on the global
// workspace copy in the same order.
// ----------------------------------------------------------------------------------
constexpr int CHOL_REG_MAX_K = 128;
constexpr int CHOL_LDS_MAX_K = 127;  // packed factor of the substitution kernel

__device__ __forceinline__ int tri_idx(int i, int l) { return i * (i + 1) / 2 + l; }

__device__ __forceinline__ double chol_pivot(double d, double tiny) {
    return (d > tiny && isfinite(d)) ? d : 1.0;
}

// 1 / p for a positive finite pivot: the hardware reciprocal refined by two Newton steps
// (a few dependent operations on the critical path of a column step, within an ulp).
__device__ __forceinline__ double chol_recip(double p) {
    double r = __builtin_amdgcn_rcp(p);
    r = fma(r, fma(-p, r, 1.0), r);
    return fma(r, fma(-p, r, 1.0), r);
}

// RM > 0: the register path for 16 (RM - 1) < k <= 16 RM (only the RM row blocks that
// exist are unrolled); RM = 0: the global-memory path for k > CHOL_REG_MAX_K.
template <int RM>
__global__ __launch_bounds__(256) void k_chol(int k, const double* __restrict__ Khat,
                                              double* __restrict__ Lout, int* __restrict__ status) {
    __shared__ double col[2][CHOL_REG_MAX_K];
    __shared__ double piv[CHOL_REG_MAX_K];
    __shared__ double dmax[256];
    __shared__ int bad;
    const int b = blockIdx.x;
    const double* Kb = Khat + (size_t)b * k * k;
    double* Lg = Lout + (size_t)b * k * k;
    const int ty = threadIdx.x / 16, tx = threadIdx.x % 16;  // blockDim.x == 256
    if (threadIdx.x == 0) bad = 0;
    // largest original diagonal entry (fixed-order tree)
    dmax[threadIdx.x] = threadIdx.x < k ? fabs(Kb[(size_t)threadIdx.x * k + threadIdx.x]) : 0.0;
    for (int q = 256 + threadIdx.x; q < k; q += 256) dmax[threadIdx.x] = fmax(dmax[threadIdx.x], fabs(Kb[(size_t)q * k + q]));
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) dmax[threadIdx.x] = fmax(dmax[threadIdx.x], dmax[threadIdx.x + h]);
        __syncthreads();
    }
    const double tiny = 64.0 * k * 2.220446049250313e-16 * dmax[0];
    if constexpr (RM > 0) {
        double a[RM][RM];
#pragma unroll
        for (int r = 0; r < RM; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) {
                const int i = ty + 16 * r, l = tx + 16 * c;
                a[r][c] = (i < k && l <= i) ? Kb[(size_t)i * k + l] : 0.0;
            }
#pragma unroll
        for (int c0 = 0; c0 < RM; ++c0) {
            if (16 * c0 >= k) break;
            const int jn = min(16, k - 16 * c0);
            for (int jj = 0; jj < jn; ++jj) {
                const int j = 16 * c0 + jj;
                double* cv = col[j & 1];
                if (tx == jj) {
#pragma unroll
                    for (int r = c0; r < RM; ++r) {
                        const int i = ty + 16 * r;
                        if (i >= j && i < k) cv[i] = a[r][c0];
                    }
                }
                __syncthreads();
                const double d = cv[j];
                const double p = chol_pivot(d, tiny);
                if (threadIdx.x == 0) {
                    piv[j] = p;
                    if (p != d) bad = 1;
                }
                const double inv = chol_recip(p);
                double li[RM], lc[RM];
#pragma unroll
                for (int r = c0; r < RM; ++r) {
                    const int i = ty + 16 * r, l = tx + 16 * r;
                    li[r] = (i > j && i < k) ? cv[i] * inv : 0.0;
                    lc[r] = (l > j && l < k) ? cv[l] : 0.0;
                }
                // entries with l <= j or i >= k meet a zero factor; those with l > i
                // (upper part of the diagonal tiles) are never written out
#pragma unroll
                for (int r = c0; r < RM; ++r)
#pragma unroll
                    for (int c = c0; c <= r; ++c) a[r][c] -= li[r] * lc[c];
            }
        }
        __syncthreads();
        // L[i][l] = A[i][l] / sqrt(pivot l), L[l][l] = sqrt(pivot l), 0 above
#pragma unroll
        for (int r = 0; r < RM; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) {
                const int i = ty + 16 * r, l = tx + 16 * c;
                if (i < k && l <= i) {
                    const double sp = sqrt(piv[l]);
                    Lg[(size_t)i * k + l] = l < i ? a[r][c] / sp : sp;
                }
            }
        for (int q = threadIdx.x; q < k * k; q += blockDim.x) {
            const int i = q / k, l = q - i * k;
            if (l > i) Lg[q] = 0.0;
        }
    } else {
        auto at = [&](int i, int l) -> double& { return Lg[(size_t)i * k + l]; };
        for (int q = threadIdx.x; q < k * k; q += blockDim.x) {
            const int i = q / k, l = q - i * k;
            Lg[q] = l <= i ? Kb[q] : 0.0;
        }
        __syncthreads();
        for (int j = 0; j < k; ++j) {
            const double d = at(j, j);
            const double p = chol_pivot(d, tiny);
            if (threadIdx.x == 0 && p != d) bad = 1;
            const double inv = 1.0 / p;
            for (int i = j + 1 + ty; i < k; i += 16) {
                const double lij = at(i, j) * inv;
                for (int l = j + 1 + tx; l <= i; l += 16) at(i, l) -= lij * at(l, j);
            }
            __syncthreads();
        }
        for (int q = threadIdx.x; q < k * k; q += blockDim.x) {
            const int i = q / k, l = q - i * k;
            if (l < i) Lg[q] /= sqrt(chol_pivot(Lg[(size_t)l * k + l], tiny));
        }
        __syncthreads();
        for (int l = threadIdx.x; l < k; l += blockDim.x)
            Lg[(size_t)l * k + l] = sqrt(chol_pivot(Lg[(size_t)l * k + l], tiny));
    }
    __syncthreads();
    if (threadIdx.x == 0) status[b] = bad ? TOPO_ENOTSPD : 0;
}

// Forward and back substitution L L^T x = rhs (one block per system) with the packed
// factor in LDS, run by the first wavefront alone: lane l owns rows l and l + 64, the
// value of the pivot row is broadcast with v_readlane, so no step waits on a barrier.
// Reciprocal pivots are formed once, up front.
template <int RM>
__device__ __forceinline__ void wave_trsv(int k, const double* __restrict__ sl, double (&v)[RM]) {
    const int lane = threadIdx.x;
    double rd[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int i = lane + 64 * r;
        rd[r] = i < k ? 1.0 / sl[tri_idx(i, i)] : 0.0;
    }
    auto bcast = [](double x, int src) -> double {
        const long long u = __double_as_longlong(x);
        const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), src);
        const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    };
    // forward, L w = rhs: after w_j is known, rows i > j drop L[i][j] w_j.  The factor
    // entries of step j + 1 are loaded during step j (they do not depend on w).
    auto fwd_load = [&](int j, double (&lv)[RM]) {
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            const int i = lane + 64 * r;
            lv[r] = (i > j && i < k) ? sl[tri_idx(i, j)] : 0.0;
        }
    };
    {
        double nxt[RM];
        fwd_load(0, nxt);
#pragma unroll
        for (int R = 0; R < RM; ++R) {
            const int jn = min(64, k - 64 * R);
            for (int jj = 0; jj < jn; ++jj) {
                const int j = 64 * R + jj;
                double cur[RM];
#pragma unroll
                for (int r = 0; r < RM; ++r) cur[r] = nxt[r];
                if (j + 1 < k) fwd_load(j + 1, nxt);
                const double wj = bcast(v[R], jj) * bcast(rd[R], jj);
                if (lane == jj) v[R] = wj;
#pragma unroll
                for (int r = R; r < RM; ++r) v[r] -= cur[r] * wj;  // zero where i <= j or i >= k
            }
        }
    }
    // backward, L^T y = w: after y_j is known, rows i < j drop L[j][i] y_j
    auto bwd_load = [&](int j, double (&lv)[RM]) {
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            const int i = lane + 64 * r;
            lv[r] = i < j ? sl[tri_idx(j, i)] : 0.0;
        }
    };
    {
        double nxt[RM];
        bwd_load(k - 1, nxt);
#pragma unroll
        for (int R = RM - 1; R >= 0; --R) {
            const int jn = min(64, k - 64 * R);
            for (int jj = jn - 1; jj >= 0; --jj) {
                const int j = 64 * R + jj;
                double cur[RM];
#pragma unroll
                for (int r = 0; r < RM; ++r) cur[r] = nxt[r];
                if (j > 0) bwd_load(j - 1, nxt);
                const double yj = bcast(v[R], jj) * bcast(rd[R], jj);
                if (lane == jj) v[R] = yj;
#pragma unroll
                for (int r = 0; r <= R; ++r) v[r] -= cur[r] * yj;  // zero where i >= j
            }
        }
    }
}

// x[b] = L^{-T} L^{-1} rhs[b] (or x[b] += stepw[b] * that when accumulate), and J[b] =
// c^T x[b] when J is given.
__global__ __launch_bounds__(256) void k_chol_solve(int k, const double* __restrict__ L,
                                                    const double* __restrict__ rhs, long long rstride,
                                                    double* __restrict__ x, int accumulate,
                                                    const double* __restrict__ stepw,
                                                    const double* __restrict__ cvec,
                                                    double* __restrict__ J) {
    __shared__ double sm[CHOL_LDS_MAX_K * (CHOL_LDS_MAX_K + 1) / 2];
    __shared__ double lds[16];
    const int b = blockIdx.x;
    const double* Lb = L + (size_t)b * k * k;
    const double* rb = rhs + (size_t)b * rstride;
    double* xb = x + (size_t)b * k;
    const double w = stepw ? stepw[b] : 1.0;
    if (accumulate && w == 0.0) return;  // x unchanged (whatever the factor holds)
    if (k <= CHOL_LDS_MAX_K) {
        // eight loads in flight per thread
        const int kk = k * k;
        for (int q0 = threadIdx.x; q0 < kk; q0 += 8 * 256) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = q0 + 256 * u;
                t[u] = q < kk ? Lb[q] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = q0 + 256 * u;
                const int i = q / k, l = q - i * k;
                if (q < kk && l <= i) sm[tri_idx(i, l)] = t[u];
            }
        }
        __syncthreads();
        if (threadIdx.x >= 64) return;
        const int lane = threadIdx.x;
        double v[2];
        v[0] = lane < k ? rb[lane] : 0.0;
        v[1] = lane + 64 < k ? rb[lane + 64] : 0.0;
        if (k <= 64) {
            double v1[1] = {v[0]};
            wave_trsv<1>(k, sm, v1);
            v[0] = v1[0];
        } else {
            wave_trsv<2>(k, sm, v);
        }
        double jsum = 0.0;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int i = lane + 64 * r;
            if (i < k) {
                const double xi = accumulate ? xb[i] + w * v[r] : v[r];
                xb[i] = xi;
                if (J) jsum += cvec[i] * xi;
            }
        }
        if (J) {
            for (int off = 32; off > 0; off >>= 1) jsum += __shfl_xor(jsum, off, 64);
            if (lane == 0) J[b] = jsum;
        }
        return;
    }
    // larger k: the vector in LDS, column-oriented substitution by the whole block
    double* sv = sm;  // [k], k <= 1024
    for (int i = threadIdx.x; i < k; i += blockDim.x) sv[i] = rb[i];
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (threadIdx.x == 0) sv[j] /= Lb[(size_t)j * k + j];
        __syncthreads();
        const double wj = sv[j];
        for (int i = j + 1 + threadIdx.x; i < k; i += blockDim.x) sv[i] -= Lb[(size_t)i * k + j] * wj;
        __syncthreads();
    }
    for (int j = k - 1; j >= 0; --j) {
        if (threadIdx.x == 0) sv[j] /= Lb[(size_t)j * k + j];
        __syncthreads();
        const double yj = sv[j];
        for (int i = threadIdx.x; i < j; i += blockDim.x) sv[i] -= Lb[(size_t)j * k + i] * yj;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < k; i += blockDim.x) xb[i] = accumulate ? xb[i] + w * sv[i] : sv[i];
    if (J) {
        __syncthreads();
        double s[1] = {0.0};
        for (int i = threadIdx.x; i < k; i += blockDim.x) s[0] += cvec[i] * xb[i];
        block_reduce<1>(s, lds);
        if (threadIdx.x == 0) J[b] = s[0];
    }
}

static void launch_chol(int k, int B, const double* Khat, double* L, int* st, hipStream_t s) {
    const int rm = k <= CHOL_REG_MAX_K ? (k + 15) / 16 : 0;
    switch (rm) {
#define TOPO_CHOL_CASE(n) \
    case n: hipLaunchKernelGGL(k_chol<n>, dim3(B), dim3(256), 0, s, k, Khat, L, st); break;
    TOPO_CHOL_CASE(1) TOPO_CHOL_CASE(2) TOPO_CHOL_CASE(3) TOPO_CHOL_CASE(4)
    TOPO_CHOL_CASE(5) TOPO_CHOL_CASE(6) TOPO_CHOL_CASE(7) TOPO_CHOL_CASE(8)
#undef TOPO_CHOL_CASE
    default: hipLaunchKernelGGL(k_chol<0>, dim3(B), dim3(256), 0, s, k, Khat, L, st);
    }
}

// resnorm[b] = sqrt(sum r^2), Jk[b] = f^T u  from the residual kernel's reductions
__global__ void k_estimate_out(int B, const double* __restrict__ out, double* __restrict__ resnorm,
                               double* __restrict__ Jk) {
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        resnorm[b] = sqrt(out[4 * b]);
        if (Jk) Jk[b] = out[4 * b + 1];
    }
}

// g2[b] = ||v[b]||^2 (one block per row, fixed order)
__global__ void k_sqnorm_rows(int k, const double* __restrict__ v, double* __restrict__ g2) {
    __shared__ double lds[16];
    const int b = blockIdx.x;
    double s[1] = {0.0};
    for (int j = threadIdx.x; j < k; j += blockDim.x) s[0] += v[(size_t)b * k + j] * v[(size_t)b * k + j];
    block_reduce<1>(s, lds);
    if (threadIdx.x == 0) g2[b] = s[0];
}

// Reduced refinement bookkeeping (one entry per field).  A field refines while its
// factor is valid and each step lowers its Galerkin residual ||Phi^T r||; `keep` holds
// the residual-kernel sums (||r||^2, f^T u) of the last accepted y.
__global__ void k_refine_begin(int B, const int* __restrict__ st, const double* __restrict__ out,
                               int* __restrict__ active, double* __restrict__ stepw,
                               double* __restrict__ keep) {
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        active[b] = st[b] == 0;
        stepw[b] = st[b] == 0 ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) keep[4 * b + q] = out[4 * b + q];
    }
}

// After a step: accept it (new sums kept) when the Galerkin residual dropped, else
// restore y from ysave and stop refining that field.  One block per field.
__global__ void k_refine_select(int k, const double* __restrict__ g2new, double* __restrict__ g2cur,
                                int* __restrict__ active, double* __restrict__ stepw,
                                const double* __restrict__ out, double* __restrict__ keep,
                                const double* __restrict__ ysave, double* __restrict__ y) {
    const int b = blockIdx.x;
    if (!active[b]) return;
    const bool ok = g2new[b] < g2cur[b];
    __syncthreads();
    if (ok) {
        if (threadIdx.x < 4) keep[4 * b + threadIdx.x] = out[4 * b + threadIdx.x];
        if (threadIdx.x == 0) g2cur[b] = g2new[b];
    } else {
        for (int j = threadIdx.x; j < k; j += blockDim.x) y[(size_t)b * k + j] = ysave[(size_t)b * k + j];
        if (threadIdx.x == 0) {
            active[b] = 0;
            stepw[b] = 0.0;
        }
    }
}

// ----------------------------------------------------------------------------------
// Host side
// ----------------------------------------------------------------------------------
static int check_basis(Ctx* ctx, const Grid& g, const void* phi, int k, int ldphi) {
    if (!phi) return set_error(ctx, TOPO_EINVAL, "phi is NULL");
    if (k < 1) return set_error(ctx, TOPO_EINVAL, "k must be >= 1");
    if ((long long)k > g.n_dofs) return set_error(ctx, TOPO_EINVAL, "k exceeds the number of DOFs");
    if (ldphi < k) return set_error(ctx, TOPO_EINVAL, "ldphi < k");
    if (ldphi > 1024) return set_error(ctx, TOPO_EINVAL, "ldphi > 1024 is not supported");
    return TOPO_OK;
}

// Rows per LDS tile of the basis-streaming kernels: as many as fit in 48 KB (a power of
// two between 1 and 256).
static int tile_rows(int ldphi, size_t esz) {
    const size_t row = (size_t)(ldphi | 1) * esz;
    int rb = 256;
    while (rb > 1 && (size_t)rb * row > 48 * 1024) rb >>= 1;
    return rb;
}

static size_t tile_bytes(int rb, int ldphi, size_t esz) {
    return (((size_t)rb * (ldphi | 1) * esz + 15) & ~(size_t)15);
}

static int phit_v(Ctx* ctx, const Grid& g, const void* phi, int fp32, int k, int ldphi,
                  const uint8_t* mask, const double* v, long long vstride, int B, double* out,
                  double* partials, int nchunks, hipStream_t s) {
    const long long nrows = g.n_dofs;
    // rows per chunk a multiple of 4: every tile starts 16-byte aligned in the basis
    const int rpc = (int)((nrows + nchunks - 1) / nchunks + 3) & ~3;
    const size_t esz = fp32 ? 4 : 8;
    const int rb = tile_rows(ldphi, esz);
    if (k > 1024) return set_error(ctx, TOPO_EINVAL, "k > 1024 not supported by the projection kernel");
    // columns per thread and fields per group: at most 32 float64 accumulators a thread
    const int cq = (k + 255) / 256;
    const int G = cq == 1 ? 16 : cq == 2 ? 8 : 4;
    const size_t lds = tile_bytes(rb, ldphi, esz) + (size_t)G * rb * sizeof(double);
    const dim3 grid(nchunks, (B + G - 1) / G);
    {
        TimedLaunch tl(ctx, KID_PHIT_V, s);
#define TOPO_PHIT_CASE(CQ, GG)                                                                          \
    case CQ:                                                                                           \
        if (fp32) {                                                                                    \
            TOPO_HIP(ensure_dynamic_lds((const void*)k_phit_v<float, CQ, GG>, lds));                  \
            hipLaunchKernelGGL((k_phit_v<float, CQ, GG>), grid, dim3(256), lds, s, nrows,              \
                               (const float*)phi, k, ldphi, mask, v, vstride, B, rpc, rb, partials);  \
        } else {                                                                                       \
            TOPO_HIP(ensure_dynamic_lds((const void*)k_phit_v<double, CQ, GG>, lds));                 \
            hipLaunchKernelGGL((k_phit_v<double, CQ, GG>), grid, dim3(256), lds, s, nrows,             \
                               (const double*)phi, k, ldphi, mask, v, vstride, B, rpc, rb, partials); \
        }                                                                                              \
        break;
        switch (cq) {
            TOPO_PHIT_CASE(1, 16) TOPO_PHIT_CASE(2, 8) TOPO_PHIT_CASE(3, 4) TOPO_PHIT_CASE(4, 4)
            default: return set_error(ctx, TOPO_EINVAL, "k > 1024 not supported by the projection kernel");
        }
#undef TOPO_PHIT_CASE
    }
    TOPO_CHECK_LAUNCH();
    launch_chunk_sum(k, nchunks, B, partials, ColsumOut{k, out}, s);
    TOPO_CHECK_LAUNCH();
    return TOPO_OK;
}

static int phi_y_launch(Ctx* ctx, const void* phi, int fp32, int k, int ldphi, const uint8_t* mask,
                        const double* y, long long N, int B, double* u, hipStream_t s) {
    const size_t esz = fp32 ? 4 : 8;
    const int rb = tile_rows(ldphi, esz);
    // the group's coefficients in LDS: at most 64 KB beside the 48 KB basis tile
    const int G = k <= 512 ? 16 : 8;
    const size_t lds = (((size_t)G * k + 1) & ~(size_t)1) * sizeof(double) + tile_bytes(rb, ldphi, esz);
    const dim3 grid(grid_blocks(N, rb), (B + G - 1) / G);
    {
        const void* kern = G == 16 ? (fp32 ? (const void*)k_phi_y<float, 16> : (const void*)k_phi_y<double, 16>)
                                   : (fp32 ? (const void*)k_phi_y<float, 8> : (const void*)k_phi_y<double, 8>);
        TOPO_HIP(ensure_dynamic_lds(kern, lds));
        TimedLaunch tl(ctx, KID_PHI_Y, s);
        if (G == 16) {
            if (fp32)
                hipLaunchKernelGGL((k_phi_y<float, 16>), grid, dim3(256), lds, s, N, (const float*)phi, k, ldphi,
                                   mask, y, B, rb, u);
            else
                hipLaunchKernelGGL((k_phi_y<double, 16>), grid, dim3(256), lds, s, N, (const double*)phi, k,
                                   ldphi, mask, y, B, rb, u);
        } else {
            if (fp32)
                hipLaunchKernelGGL((k_phi_y<float, 8>), grid, dim3(256), lds, s, N, (const float*)phi, k, ldphi,
                                   mask, y, B, rb, u);
            else
                hipLaunchKernelGGL((k_phi_y<double, 8>), grid, dim3(256), lds, s, N, (const double*)phi, k,
                                   ldphi, mask, y, B, rb, u);
        }
    }
    TOPO_CHECK_LAUNCH();
    return TOPO_OK;
}

static int phit_chunks(const Grid& g) {
    long long c = g.n_dofs / 256;
    return (int)std::max(1LL, std::min(c, 2048LL));
}

struct ContractPlan {
    int KP, kt, npairs, groups, nt, sd, ch, nchunks;
    long long ld;  // row pitch of the operands
    size_t lds_bytes;
};

// The plan depends on the mesh, k and the basis type only -- never on B -- so a field's
// K_hat is bitwise the same alone and inside a batch.  f64: the basis is float64.
static ContractPlan plan_contract(const Grid& g, int k, bool f64) {
    ContractPlan p;
    p.KP = (k + 15) / 16 * 16;
    p.kt = p.KP / 16;
    p.npairs = p.kt * (p.kt + 1) / 2;
    p.groups = (p.npairs + MAX_NT * GW - 1) / (MAX_NT * GW);
    p.nt = (p.npairs + p.groups * GW - 1) / (p.groups * GW);
    p.sd = gemm_sd<double>(p.KP);
    // DOFs per chunk (one float64 partial tile per chunk and pair): a multiple of 256
    // (whole slabs) between 1024 and 8192, sized for about 1024 blocks per launch, so that
    // a mesh of under a million DOFs still spreads over several blocks per CU (at 8192 a
    // 698k-DOF field made 86 blocks for 256 CUs)
    const long long want = (g.n_dofs * p.groups + 1023) / 1024;
    p.ch = (int)std::min(8192LL, std::max(1024LL, (want + 255) / 256 * 256));
    p.nchunks = (int)((g.n_dofs + p.ch - 1) / p.ch);
    p.ld = (g.n_dofs + GEMM_LD - 1) / GEMM_LD * GEMM_LD;
    p.lds_bytes = (size_t)p.KP * (p.sd + 2) * ((f64 ? 8 : 4) + 8);  // Pt in the basis type, Wt in float64
    return p;
}

template <typename TC, int SD, int NT>
static int launch_gemm_nt(Ctx* ctx, const ContractPlan& p, const TC* Pt, const double* Wt, long long nu, int k,
                          double* parts, hipStream_t s) {
    auto kern = k_rom_gemm<TC, SD, NT>;
    TOPO_HIP(ensure_dynamic_lds((const void*)kern, p.lds_bytes));
    hipLaunchKernelGGL(kern, dim3(p.nchunks, p.groups), dim3(GW * 64), p.lds_bytes, s, Pt, Wt, p.ld, nu, k, p.KP,
                       p.npairs, p.kt, p.ch, parts);
    TOPO_CHECK_LAUNCH();
    return TOPO_OK;
}

template <typename TC, int SD>
static int launch_gemm_sd(Ctx* ctx, const ContractPlan& p, const TC* Pt, const double* Wt, long long nu, int k,
                          double* parts, hipStream_t s) {
    // the smallest instantiated pair count per wave that covers the plan's
    if (p.nt <= 1) return launch_gemm_nt<TC, SD, 1>(ctx, p, Pt, Wt, nu, k, parts, s);
    if (p.nt <= 2) return launch_gemm_nt<TC, SD, 2>(ctx, p, Pt, Wt, nu, k, parts, s);
    if (p.nt <= 3) return launch_gemm_nt<TC, SD, 3>(ctx, p, Pt, Wt, nu, k, parts, s);
    return launch_gemm_nt<TC, SD, 4>(ctx, p, Pt, Wt, nu, k, parts, s);
}

template <typename TC>
static int launch_gemm(Ctx* ctx, const ContractPlan& p, const TC* Pt, const double* Wt, long long nu, int k,
                       double* parts, hipStream_t s) {
    constexpr int SD0 = gemm_sd<double>(256), SD1 = gemm_sd<double>(512), SD2 = gemm_sd<double>(1024);
    if (p.sd == SD0) return launch_gemm_sd<TC, SD0>(ctx, p, Pt, Wt, nu, k, parts, s);
    if (p.sd == SD1) return launch_gemm_sd<TC, SD1>(ctx, p, Pt, Wt, nu, k, parts, s);
    return launch_gemm_sd<TC, SD2>(ctx, p, Pt, Wt, nu, k, parts, s);
}

// K_hat of every field (the contraction and its chunk sums), from the basis Phi (TP):
// Pt [k][ld] (TP), Wt [k][ld] (float64) and parts [nchunks][npairs][256] are workspace;
// alpha [B][N_e] in float64.
template <typename TP>
static int contract_fields(Ctx* ctx, const Grid& g, const ElemTables* tb, const ContractPlan& p, const TP* phi,
                           int k, int ldphi, const uint8_t* mask, const double* alpha, int B, TP* Pt, double* Wt,
                           double* parts, double* Khat, hipStream_t s) {
    const long long nu = g.n_dofs;
    {
        TimedLaunch tl(ctx, KID_ROM_APPLY, s);
        hipLaunchKernelGGL((k_basis_rows<TP>), dim3((unsigned)(p.ld / 64), (k + 63) / 64), dim3(256), 0, s,
                           phi, ldphi, nu, k, p.ld, Pt, Wt);
    }
    TOPO_CHECK_LAUNCH();
    for (int b = 0; b < B; ++b) {
        int rc;
        {
            TimedLaunch tl(ctx, KID_ROM_APPLY, s);
            rc = apply_columns<TP>(ctx, g, tb, alpha + (size_t)b * g.n_elems, mask, Pt, Wt, k, p.ld, s);
        }
        if (rc) return rc;
        {
            TimedLaunch tl(ctx, KID_ROM_CONTRACT, s);
            rc = launch_gemm<TP>(ctx, p, Pt, Wt, nu, k, parts, s);
        }
        if (rc) return rc;
        {
            TimedLaunch tl(ctx, KID_ROM_REDUCE, s);
            launch_chunk_sum(p.npairs * 256, p.nchunks, 1, (const double*)parts,
                             KhatOut{k, p.kt, Khat + (size_t)b * k * k}, s);
        }
        TOPO_CHECK_LAUNCH();
    }
    return TOPO_OK;
}

}  // namespace topo

using namespace topo;

extern "C" {

int topo_rom_build(topo_ctx* ctx, const topo_mesh* mesh, const void* phi, int32_t phi_fp32,
                   int32_t k, int32_t ldphi, const uint8_t* mask, const double* f,
                   const double* rho, int32_t B, double* Khat, double* fhat, int32_t prec,
                   void* stream) {
    if (!ctx) return TOPO_EINVAL;
    int rc = validate_mesh(ctx, mesh);
    if (rc) return rc;
    const Grid g = make_grid(*mesh);
    rc = check_basis(ctx, g, phi, k, ldphi);
    if (rc) return rc;
    if (!mask || !rho || !Khat || B < 1) return set_error(ctx, TOPO_EINVAL, "bad argument");
    if (fhat && !f) return set_error(ctx, TOPO_EINVAL, "fhat requested without f");
    if (prec != TOPO_FP64 && prec != TOPO_MIXED) return set_error(ctx, TOPO_EINVAL, "bad precision");
    TOPO_HIP(hipSetDevice(ctx->device));
    const ElemTables* tb = get_tables(ctx, *mesh);
    if (!tb) return set_error(ctx, TOPO_EDEVICE, "element table upload failed");
    hipStream_t s = (hipStream_t)stream;
    // The contraction's arithmetic is float64 in both precisions (see k_rom_gemm): the
    // transposed basis keeps the basis's own type, W = K Phi is float64.
    (void)prec;
    const ContractPlan p = plan_contract(g, k, !phi_fp32);
    if (p.KP > KP_MAX) return set_error(ctx, TOPO_EINVAL, "k = %d too large for the contraction (at most %d)", k, KP_MAX);
    const int nc = phit_chunks(g);
    const size_t nk = (size_t)k * p.ld, np = (size_t)p.nchunks * p.npairs * 256;
    Arena ar;
    double *a64 = nullptr, *P64 = nullptr, *Wt = nullptr, *parts = nullptr, *pf = nullptr;
    float* P32 = nullptr;
    ar.take(&a64, (size_t)B * g.n_elems);
    if (phi_fp32) ar.take(&P32, nk);
    else ar.take(&P64, nk);
    ar.take(&Wt, nk);
    ar.take(&parts, np);
    ar.take(&pf, (size_t)nc * k);
    rc = ar.commit(ctx, s);
    if (rc) return rc;
    rc = alpha_tables(ctx, g, *mesh, rho, B, a64, nullptr, s);
    if (rc) return rc;
    rc = phi_fp32 ? contract_fields(ctx, g, tb, p, (const float*)phi, k, ldphi, mask, (const double*)a64, B, P32, Wt,
                                    parts, Khat, s)
                  : contract_fields(ctx, g, tb, p, (const double*)phi, k, ldphi, mask, (const double*)a64, B, P64, Wt,
                                    parts, Khat, s);
    if (rc) return rc;
    if (fhat) {
        rc = phit_v(ctx, g, phi, phi_fp32, k, ldphi, mask, f, 0, 1, fhat, pf, nc, s);
        if (rc) return rc;
    }
    return TOPO_OK;
}

int topo_rom_solve(topo_ctx* ctx, int32_t k, int32_t B, const double* Khat, const double* fhat,
                   double* yhat, double* Jk, int32_t* status, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    if (k < 1 || B < 1) return set_error(ctx, TOPO_EINVAL, "k and B must be >= 1");
    if (!Khat || !fhat || !yhat || !Jk) return set_error(ctx, TOPO_EINVAL, "null pointer argument");
    TOPO_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    Arena ar;
    double* L;
    int* st;
    ar.take(&L, (size_t)B * k * k);
    ar.take(&st, (size_t)B);
    int rc = ar.commit(ctx, s);
    if (rc) return rc;
    int* stp = status ? (int*)status : st;
    {
        TimedLaunch tl(ctx, KID_CHOL, s);
        launch_chol(k, B, Khat, L, stp, s);
    }
    TOPO_CHECK_LAUNCH();
    {
        TimedLaunch tl(ctx, KID_CHOL_SOLVE, s);
        hipLaunchKernelGGL(k_chol_solve, dim3(B), dim3(256), 0, s, k, L, fhat, 0LL, yhat,
                           0, (const double*)nullptr, fhat, Jk);
    }
    TOPO_CHECK_LAUNCH();
    if (!status) {
        std::vector<int> h(B);
        TOPO_HIP(hipMemcpyAsync(h.data(), st, B * sizeof(int), hipMemcpyDeviceToHost, s));
        TOPO_HIP(hipStreamSynchronize(s));
        for (int b = 0; b < B; ++b)
            if (h[b] != 0) return set_error(ctx, TOPO_ENOTSPD, "reduced operator %d is not SPD", b);
    }
    return TOPO_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------------
// Allocation-free reduced solve.  The Cholesky factors of topo_rom_solve live in this
// fixed device array instead of the context's workspace, for callers that cannot
// allocate device memory.  Each GPU holds its own copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns on that device
// (the array's name is not a device address in host code).
// ----------------------------------------------------------------------------------
namespace topo {

constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on the context's device (looked up once per device, with
// that device current).
static int noalloc_scratch(Ctx* ctx, void** out) {
    if (ctx->device < 0 || ctx->device >= kNoAllocMaxDevices)
        return set_error(ctx, TOPO_EINVAL, "device %d beyond the allocation-free path's range", ctx->device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[ctx->device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_error(ctx, TOPO_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        g_scratch_ptr[ctx->device] = p;
    }
    *out = g_scratch_ptr[ctx->device];
    return TOPO_OK;
}

}  // namespace topo

extern "C" {

size_t topo_rom_solve_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int topo_rom_solve_noalloc(topo_ctx* ctx, int32_t k, int32_t B, const double* Khat, const double* fhat,
                           double* yhat, double* Jk, int32_t* status, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    if (k < 1 || B < 1) return set_error(ctx, TOPO_EINVAL, "k and B must be >= 1");
    if (!Khat || !fhat || !yhat || !Jk || !status)
        return set_error(ctx, TOPO_EINVAL, "null pointer argument (status is required)");
    const size_t need = (size_t)B * (size_t)k * (size_t)k * sizeof(double);
    if (need > kNoAllocScratchBytes)
        return set_error(ctx, TOPO_EINVAL, "B k^2 doubles = %zu bytes exceed the fixed scratch of %zu bytes",
                         need, kNoAllocScratchBytes);
    TOPO_HIP(hipSetDevice(ctx->device));
    void* sp = nullptr;
    const int rc = noalloc_scratch(ctx, &sp);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    double* L = (double*)sp;  // every entry the solve reads is written by the factorisation
    launch_chol(k, B, Khat, L, (int*)status, s);
    TOPO_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_chol_solve, dim3(B), dim3(256), 0, s, k, (const double*)L, fhat, 0LL, yhat, 0,
                       (const double*)nullptr, fhat, Jk);
    TOPO_CHECK_LAUNCH();
    return TOPO_OK;
}

int topo_rom_estimate(topo_ctx* ctx, const topo_mesh* mesh, const void* phi, int32_t phi_fp32,
                      int32_t k, int32_t ldphi, const uint8_t* mask, const double* f,
                      const double* rho, int32_t B, const double* Khat, double* yhat, double* Jk,
                      double* resnorm, int32_t max_refine, double* dJ, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    int rc = validate_mesh(ctx, mesh);
    if (rc) return rc;
    const Grid g = make_grid(*mesh);
    rc = check_basis(ctx, g, phi, k, ldphi);
    if (rc) return rc;
    if (!mask || !f || !rho || !yhat || !resnorm || B < 1 || max_refine < 0)
        return set_error(ctx, TOPO_EINVAL, "bad argument");
    if (max_refine > 0 && !Khat) return set_error(ctx, TOPO_EINVAL, "refinement needs Khat");
    TOPO_HIP(hipSetDevice(ctx->device));
    const ElemTables* tb = get_tables(ctx, *mesh);
    if (!tb) return set_error(ctx, TOPO_EDEVICE, "element table upload failed");
    hipStream_t s = (hipStream_t)stream;
    const long long N = g.n_dofs;
    const int nb = stencil_blocks(g);
    const int nc = phit_chunks(g);
    Arena ar;
    double *a64, *u, *r, *part, *out, *keep = nullptr, *rhat, *L = nullptr, *pc, *ybest = nullptr;
    double *g2cur = nullptr, *g2new = nullptr, *stepw = nullptr;
    int *st = nullptr, *active = nullptr;
    ar.take(&a64, (size_t)B * g.n_elems);
    ar.take(&u, (size_t)B * N);
    ar.take(&r, (size_t)B * N);
    ar.take(&part, (size_t)B * 3 * nb);
    ar.take(&out, (size_t)4 * B);
    ar.take(&rhat, (size_t)B * k);
    ar.take(&pc, (size_t)B * nc * k);
    if (max_refine > 0) {
        ar.take(&keep, (size_t)4 * B);
        ar.take(&ybest, (size_t)B * k);
        ar.take(&g2cur, (size_t)B);
        ar.take(&g2new, (size_t)B);
        ar.take(&stepw, (size_t)B);
        ar.take(&L, (size_t)B * k * k);
        ar.take(&st, (size_t)B);
        ar.take(&active, (size_t)B);
    }
    rc = ar.commit(ctx, s);
    if (rc) return rc;
    rc = alpha_tables(ctx, g, *mesh, rho, B, a64, nullptr, s);
    if (rc) return rc;
    // u = Phi y_hat, r = f - K u, ||r||^2 and f^T u per field
    auto pass = [&]() -> int {
        int rc2 = phi_y_launch(ctx, phi, phi_fp32, k, ldphi, mask, yhat, N, B, u, s);
        if (rc2) return rc2;
        return residual_fp64(ctx, g, tb, a64, mask, u, f, r, B, part, out, s);
    };
    // Galerkin residual r_hat = Phi^T r and its squared norm per field
    auto galerkin = [&](double* g2) -> int {
        int rc2 = phit_v(ctx, g, phi, phi_fp32, k, ldphi, mask, r, N, B, rhat, pc, nc, s);
        if (rc2) return rc2;
        hipLaunchKernelGGL(k_sqnorm_rows, dim3(B), dim3(64), 0, s, k, (const double*)rhat, g2);
        TOPO_CHECK_LAUNCH();
        return TOPO_OK;
    };
    rc = pass();
    if (rc) return rc;
    if (max_refine > 0) {
        // Reduced iterative refinement: y += K_hat^{-1} Phi^T (f - K Phi y) with the
        // float64 residual, every decision taken on the device (no host round trip).
        launch_chol(k, B, Khat, L, st, s);
        TOPO_CHECK_LAUNCH();
        rc = galerkin(g2cur);
        if (rc) return rc;
        hipLaunchKernelGGL(k_refine_begin, dim3(1), dim3(64), 0, s, B, (const int*)st,
                           (const double*)out, active, stepw, keep);
        TOPO_CHECK_LAUNCH();
        for (int it = 0; it < max_refine; ++it) {
            TOPO_HIP(hipMemcpyAsync(ybest, yhat, (size_t)B * k * sizeof(double), hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_chol_solve, dim3(B), dim3(256), 0, s, k, L, rhat,
                               (long long)k, yhat, 1, (const double*)stepw, (const double*)nullptr,
                               (double*)nullptr);
            TOPO_CHECK_LAUNCH();
            rc = pass();
            if (rc) return rc;
            rc = galerkin(g2new);
            if (rc) return rc;
            hipLaunchKernelGGL(k_refine_select, dim3(B), dim3(64), 0, s, k, (const double*)g2new,
                               g2cur, active, stepw, (const double*)out, keep,
                               (const double*)ybest, yhat);
            TOPO_CHECK_LAUNCH();
        }
    }
    // ||r|| and J_k = f^T (Phi y_hat) of the returned y (reduced by the residual kernel)
    hipLaunchKernelGGL(k_estimate_out, dim3(1), dim3(64), 0, s, B,
                       (const double*)(max_refine > 0 ? keep : out), resnorm, Jk);
    TOPO_CHECK_LAUNCH();
    if (dJ) {
        // sensitivity at the returned y: u of the single pass, or re-formed after refinement
        if (max_refine > 0) {
            rc = phi_y_launch(ctx, phi, phi_fp32, k, ldphi, mask, yhat, N, B, u, s);
            if (rc) return rc;
        }
        rc = gradient_launch(ctx, g, *mesh, tb, rho, u, B, dJ, s);
        if (rc) return rc;
    }
    return TOPO_OK;
}

int topo_rom_gradient(topo_ctx* ctx, const topo_mesh* mesh, const void* phi, int32_t phi_fp32,
                      int32_t k, int32_t ldphi, const uint8_t* mask, const double* rho, int32_t B,
                      const double* yhat, double* dJ, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    int rc = validate_mesh(ctx, mesh);
    if (rc) return rc;
    const Grid g = make_grid(*mesh);
    rc = check_basis(ctx, g, phi, k, ldphi);
    if (rc) return rc;
    if (!mask || !rho || !yhat || !dJ || B < 1) return set_error(ctx, TOPO_EINVAL, "bad argument");
    TOPO_HIP(hipSetDevice(ctx->device));
    const ElemTables* tb = get_tables(ctx, *mesh);
    if (!tb) return set_error(ctx, TOPO_EDEVICE, "element table upload failed");
    hipStream_t s = (hipStream_t)stream;
    const long long N = g.n_dofs;
    Arena ar;
    double* u;
    ar.take(&u, (size_t)B * N);
    rc = ar.commit(ctx, s);
    if (rc) return rc;
    // u_k = Phi y_hat, then the element sensitivities of the compliance at u_k: for the
    // compliance the reduced adjoint is the reduced state itself
    rc = phi_y_launch(ctx, phi, phi_fp32, k, ldphi, mask, yhat, N, B, u, s);
    if (rc) return rc;
    return gradient_launch(ctx, g, *mesh, tb, rho, u, B, dJ, s);
}

}  // extern "C"

// Device workspace of the ROM entry points; each mirrors the take sequence of the
// corresponding call above (keep them in step).
namespace topo {

size_t ws_rom_build(const Grid& g, int k, int B, bool f64, int cu) {
    // f64: the basis is float64 (the contraction's own precision does not depend on the
    // build's)
    (void)cu;
    const ContractPlan p = plan_contract(g, k, f64);
    const int nc = phit_chunks(g);
    const size_t nk = (size_t)k * p.ld, np = (size_t)p.nchunks * p.npairs * 256;
    Arena ar;
    double *a64, *P64, *Wt, *parts, *pf;
    float* P32;
    ar.take(&a64, (size_t)B * g.n_elems);
    if (f64) ar.take(&P64, nk);
    else ar.take(&P32, nk);
    ar.take(&Wt, nk);
    ar.take(&parts, np);
    ar.take(&pf, (size_t)nc * k);
    return ar.total();
}

size_t ws_rom_solve(int k, int B) {
    Arena ar;
    double* L;
    int* st;
    ar.take(&L, (size_t)B * k * k);
    ar.take(&st, (size_t)B);
    return ar.total();
}

size_t ws_rom_estimate(const Grid& g, int k, int B, int max_refine) {
    const long long N = g.n_dofs;
    const int nb = stencil_blocks(g);
    const int nc = phit_chunks(g);
    Arena ar;
    double *a64, *u, *r, *part, *out, *keep, *rhat, *L, *pc, *ybest, *g2cur, *g2new, *stepw;
    int *st, *active;
    ar.take(&a64, (size_t)B * g.n_elems);
    ar.take(&u, (size_t)B * N);
    ar.take(&r, (size_t)B * N);
    ar.take(&part, (size_t)B * 3 * nb);
    ar.take(&out, (size_t)4 * B);
    ar.take(&rhat, (size_t)B * k);
    ar.take(&pc, (size_t)B * nc * k);
    if (max_refine > 0) {
        ar.take(&keep, (size_t)4 * B);
        ar.take(&ybest, (size_t)B * k);
        ar.take(&g2cur, (size_t)B);
        ar.take(&g2new, (size_t)B);
        ar.take(&stepw, (size_t)B);
        ar.take(&L, (size_t)B * k * k);
        ar.take(&st, (size_t)B);
        ar.take(&active, (size_t)B);
    }
    return ar.total();
}

}  // namespace topo
