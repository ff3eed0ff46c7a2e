// Reduced basis at a trust-region centre (Sec. 4.2): the POD of the window of the L most
// recent snapshots and one Gram-Schmidt step of the new snapshot against it.
//
// The window keeps its snapshots S_i (float64, one contiguous vector each) and their
// Gram matrix G_ij = S_i . S_j.  A push writes one slot and rewrites one row and column
// of G from a single streaming pass: a rank-one update of the window while it grows, a
// rank-two update (one snapshot in, the oldest out) once it is full.  The POD is taken by
// the method of snapshots: G = V diag(lambda) V^T by cyclic Jacobi rotations in one
// workgroup, and POD column j is S V_j / sqrt(lambda_j).  The Gram-Schmidt step, the norm
// of what is left of the new snapshot and the basis itself are then linear combinations
// of the window's snapshots and the new one, each a pass that streams them row by row.
#include <algorithm>
#include <cmath>

#include "internal.hpp"
#include "reduce.hpp"

namespace topo {

constexpr int kPodMaxL = TOPO_POD_MAX_WINDOW;  // window capacity (snapshots)
constexpr int kPodBlock = 256;
constexpr int kPodRows = 8;    // rows per thread in the dot and norm passes
constexpr int kPodWrite = 128; // rows per block of the basis writer

struct PodInfo {
    int n;         // POD columns kept
    int j;         // basis columns written: n, plus one when the new snapshot adds one
    int keep;      // 1 when the new snapshot added a column
    int pad;
    double vnorm;  // norm of the new snapshot after the Gram-Schmidt step
    double unorm;  // its norm before
};

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// partials[chunk][i] = sum over the chunk's rows of X_i[r] u[r], i = 0..m, where X_i = S_i
// for i < m except X_slot = u, and X_m = u.  With write_slot the pass also stores u into
// slot `slot` (never read here: its dot is u . u).
__global__ __launch_bounds__(kPodBlock) void k_pod_dots(long long n, double* S, int m, int slot,
                                                        int write_slot, const double* __restrict__ u,
                                                        double* __restrict__ partials) {
    __shared__ double red[kPodBlock / 64][kPodMaxL + 1];
    const long long base = (long long)blockIdx.x * kPodBlock * kPodRows + threadIdx.x;
    double uv[kPodRows];
#pragma unroll
    for (int q = 0; q < kPodRows; ++q) {
        const long long r = base + (long long)q * kPodBlock;
        uv[q] = r < n ? u[r] : 0.0;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = 0; i <= m; ++i) {
        double acc = 0.0;
        if (i == m || i == slot) {
#pragma unroll
            for (int q = 0; q < kPodRows; ++q) acc += uv[q] * uv[q];
        } else {
            const double* Si = S + (size_t)i * n;
            double x[kPodRows];
#pragma unroll
            for (int q = 0; q < kPodRows; ++q) {
                const long long r = base + (long long)q * kPodBlock;
                x[q] = r < n ? Si[r] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < kPodRows; ++q) acc += x[q] * uv[q];
        }
        acc = wave_sum64(acc);
        if (lane == 0) red[w][i] = acc;
    }
    if (write_slot) {
        double* Ss = S + (size_t)slot * n;
#pragma unroll
        for (int q = 0; q < kPodRows; ++q) {
            const long long r = base + (long long)q * kPodBlock;
            if (r < n) Ss[r] = uv[q];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= m; i += kPodBlock)
        partials[(size_t)blockIdx.x * (m + 1) + i] = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
}

// Row and column `slot` of the window's Gram matrix (entries e < m).
struct GramRowOut {
    double* G;
    int L, slot, m;
    __device__ void operator()(int, int e, double s) const {
        if (e >= m) return;
        G[(size_t)slot * L + e] = s;
        G[(size_t)e * L + slot] = s;
    }
};

// Plain vector of sums.
struct PodVecOut {
    double* out;
    __device__ void operator()(int, int e, double s) const { out[e] = s; }
};

// 1 / x and 1 / sqrt(x) in float64: the hardware approximation refined by two Newton
// steps (each doubles the number of correct bits).
__device__ __forceinline__ double pod_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double pod_rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double h = 0.5 * x * y;
        y = fma(y, fma(-h, y, 0.5), y);
    }
    return y;
}

constexpr int kEigThreads = 512;

// POD of the window from its Gram matrix, and the coefficients of the new basis as a
// combination of the window's snapshots and the new one.  One workgroup.
//
// Cyclic Jacobi: each step rotates m/2 disjoint index pairs (round-robin schedule, a
// dummy index when m is odd, every pair once per sweep).  For pairs a and b the 2 x 2
// block of A on rows {p_a, q_a} and columns {p_b, q_b} becomes J_a^T A_ab J_b, a function
// of that block alone, so one thread updates a whole block (and its mirror image) in
// place, and one thread a pair of entries V[r][p_b], V[r][q_b] of V <- V J: one phase per
// step, spread over all threads.  A pair is rotated only while a_pq^2 exceeds both
// 1e-30 a_pp a_qq and (2e-16 |diag A|)^2 (the rounding level of G); sweeps stop after a
// sweep without a rotation, or once the off-diagonal mass is below 1e-30 of the diagonal
// mass.  Eigenvalues are sorted descending; sigma_i = sqrt(max(lambda_i, 0)).  POD
// directions kept: the leading n <= min(m, nmax) with sigma_i > rtol * sigma_0.
//
// coef is (m + 1) x ldc, row i for snapshot i, row m for the new snapshot u:
//   columns j < n           : W_ij = V_i,order(j) / sigma_j  (POD column j = S W_j)
//   columns n .. ldc - 2    : zero (and column ldc - 1 when there is no u)
//   column ldc - 1 (u only) : the combination v = u - sum_j (Phi_j . u) Phi_j of the
//                             Gram-Schmidt step, with Phi_j . u = W_j . gu, gu_i = S_i . u.
__global__ __launch_bounds__(kEigThreads) void k_pod_eig(int m, int L, const double* __restrict__ G,
                                                         const double* __restrict__ gu, int nmax, double rtol,
                                                         double* __restrict__ coef, int ldc,
                                                         double* __restrict__ sigma, PodInfo* __restrict__ info) {
    constexpr int NW = kEigThreads / 64;
    __shared__ double A[kPodMaxL][kPodMaxL + 1];
    __shared__ double V[kPodMaxL][kPodMaxL + 1];
    __shared__ double cs[kPodMaxL / 2], sn[kPodMaxL / 2];
    __shared__ int pp[kPodMaxL / 2], pq[kPodMaxL / 2];
    __shared__ double red[2][NW];
    __shared__ int order[kPodMaxL];
    __shared__ double sig[kPodMaxL], rsig[kPodMaxL], cvec[kPodMaxL];
    __shared__ int s_n, s_rot, s_prev, s_step;
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    for (int i = wv; i < m; i += NW)
        if (lane < m) {
            A[i][lane] = G[(size_t)i * L + lane];
            V[i][lane] = i == lane ? 1.0 : 0.0;
        }
    __syncthreads();
    const int M = m + (m & 1);
    const int P = M / 2;
    // update items: A blocks e = ia + (ib << sa), V pairs e = r + (ib << sv)
    const int sa = P <= 8 ? 3 : P <= 16 ? 4 : 5;
    const int sv = m <= 16 ? 4 : m <= 32 ? 5 : 6;
    const int na = P << sa, nitems = na + (P << sv);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, dia = 0.0;
        if (lane < m)
            for (int i = wv; i < m; i += NW) {
                const double a = A[i][lane];
                if (i == lane) dia += a * a;
                else off += a * a;
            }
        off = wave_sum64(off);
        dia = wave_sum64(dia);
        if (lane == 0) {
            red[0][wv] = off;
            red[1][wv] = dia;
        }
        if (t == 0) s_rot = 0;
        if (t == 1) s_step = 0;
        __syncthreads();
        double offs = 0.0, dias = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            offs += red[0][w];
            dias += red[1][w];
        }
        __syncthreads();
        if (offs <= 1e-30 * dias || (sweep > 0 && s_prev == 0)) break;
        const double floor2 = 4e-32 * dias;  // (2e-16 |diag A|)^2
        for (int step = 0; step < M - 1; ++step) {
            if (t < P) {
                int a, b;
                if (t == 0) {
                    a = 0;
                    b = 1 + step;
                } else {
                    a = 1 + step + t;
                    if (a > M - 1) a -= M - 1;
                    b = 1 + step - t + M - 1;
                    if (b > M - 1) b -= M - 1;
                }
                const int p = min(a, b), q = max(a, b);
                double c = 1.0, s = 0.0;
                if (q < m) {
                    const double app = A[p][p], aqq = A[q][q], apq = A[p][q];
                    const double a2 = apq * apq;
                    if (a2 > floor2 && a2 > 1e-30 * fabs(app * aqq)) {
                        const double tau = (aqq - app) * pod_rcp(2.0 * apq);
                        const double at = fabs(tau);
                        double tt = at > 1e150 ? 0.5 / at : pod_rcp(at + sqrt(1.0 + tau * tau));
                        tt = tau < 0.0 ? -tt : tt;
                        c = pod_rsqrt(1.0 + tt * tt);
                        s = tt * c;
                        s_rot = 1;
                        s_step = step + 1;
                    }
                }
                pp[t] = p;
                pq[t] = q;
                cs[t] = c;
                sn[t] = s;
            }
            __syncthreads();
            if (s_step != step + 1) continue;  // no pair rotated in this step
            for (int e = t; e < nitems; e += kEigThreads) {
                if (e < na) {  // A: block (ia, ib), ia <= ib
                    const int ia = e & ((1 << sa) - 1), ib = e >> sa;
                    if (ia >= P || ia > ib) continue;
                    const int p1 = pp[ia], q1 = pq[ia], p2 = pp[ib], q2 = pq[ib];
                    const double c1 = cs[ia], s1 = sn[ia], c2 = cs[ib], s2 = sn[ib];
                    const bool h1 = q1 < m, h2 = q2 < m;  // false: the dummy index
                    const double x11 = A[p1][p2];
                    const double x12 = h2 ? A[p1][q2] : 0.0;
                    const double x21 = h1 ? A[q1][p2] : 0.0;
                    const double x22 = h1 && h2 ? A[q1][q2] : 0.0;
                    const double r1p = c1 * x11 - s1 * x21, r1q = c1 * x12 - s1 * x22;  // row p1 of J1^T X
                    const double r2p = s1 * x11 + c1 * x21, r2q = s1 * x12 + c1 * x22;  // row q1
                    const double y11 = r1p * c2 - r1q * s2, y12 = r1p * s2 + r1q * c2;
                    const double y21 = r2p * c2 - r2q * s2, y22 = r2p * s2 + r2q * c2;
                    A[p1][p2] = y11;
                    A[p2][p1] = y11;
                    if (h2) {
                        A[p1][q2] = y12;
                        A[q2][p1] = y12;
                    }
                    if (h1) {
                        A[q1][p2] = y21;
                        A[p2][q1] = y21;
                    }
                    if (h1 && h2) {
                        A[q1][q2] = y22;
                        A[q2][q1] = y22;
                    }
                } else {  // V <- V J: row r, pair ib
                    const int ev = e - na;
                    const int r = ev & ((1 << sv) - 1), ib = ev >> sv;
                    const int p2 = pp[ib], q2 = pq[ib];
                    if (r >= m || q2 >= m) continue;
                    const double c2 = cs[ib], s2 = sn[ib];
                    const double vp = V[r][p2], vq = V[r][q2];
                    V[r][p2] = c2 * vp - s2 * vq;
                    V[r][q2] = s2 * vp + c2 * vq;
                }
            }
            __syncthreads();
        }
        if (t == 0) s_prev = s_rot;
        __syncthreads();
    }
    // descending order by rank (ties by index)
    if (t < m) {
        const double li = A[t][t];
        int rank = 0;
        for (int k = 0; k < m; ++k) {
            const double lk = A[k][k];
            rank += (lk > li || (lk == li && k < t)) ? 1 : 0;
        }
        order[rank] = t;
    }
    __syncthreads();
    if (t < m) {
        const double sg = sqrt(fmax(A[order[t]][order[t]], 0.0));
        if (sigma) sigma[t] = sg;
        sig[t] = sg;
        rsig[t] = sg > 0.0 ? 1.0 / sg : 0.0;
    }
    __syncthreads();
    if (wv == 0) {
        const int lim = min(m, nmax);
        const bool ok = lane < lim && sig[lane] > 0.0 && sig[lane] > rtol * sig[0];
        const unsigned long long bad = __ballot(!ok);  // lanes >= lim are never ok
        if (lane == 0) s_n = __ffsll((long long)bad) - 1;
    }
    __syncthreads();
    const int n = s_n;
    const int vc = ldc - 1;
    const int wc = gu ? vc : ldc;  // POD coefficient columns (the last one is v's when u is given)
    for (int i = wv; i < m; i += NW)
        for (int j = lane; j < wc; j += 64) coef[(size_t)i * ldc + j] = j < n ? V[i][order[j]] * rsig[j] : 0.0;
    if (gu) {
        if (t < n) {
            double c = 0.0;
            for (int i = 0; i < m; ++i) c += (V[i][order[t]] * rsig[t]) * gu[i];
            cvec[t] = c;
        }
        __syncthreads();
        if (t < m) {
            double w = 0.0;
            for (int j = 0; j < n; ++j) w += (V[t][order[j]] * rsig[j]) * cvec[j];
            coef[(size_t)t * ldc + vc] = -w;
        }
        for (int j = t; j < vc; j += kEigThreads) coef[(size_t)m * ldc + j] = 0.0;
        if (t == 0) coef[(size_t)m * ldc + vc] = 1.0;
    }
    if (t == 0) {
        info->n = n;
        info->j = n;
        info->keep = 0;
        info->vnorm = 0.0;
        info->unorm = gu ? sqrt(gu[m]) : 0.0;
    }
}

// partials[chunk] = sum over the chunk's rows of v[r]^2, v = u + sum_i coef[i][vc] S_i.
__global__ __launch_bounds__(kPodBlock) void k_pod_vnorm(long long n, const double* __restrict__ S, int m,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ coef, int ldc,
                                                         double* __restrict__ partials) {
    __shared__ double red[kPodBlock / 64];
    const int vc = ldc - 1;
    const long long base = (long long)blockIdx.x * kPodBlock * kPodRows + threadIdx.x;
    double v[kPodRows];
#pragma unroll
    for (int q = 0; q < kPodRows; ++q) {
        const long long r = base + (long long)q * kPodBlock;
        v[q] = r < n ? u[r] : 0.0;
    }
    for (int i = 0; i < m; ++i) {
        const double w = coef[(size_t)i * ldc + vc];
        const double* Si = S + (size_t)i * n;
        double x[kPodRows];
#pragma unroll
        for (int q = 0; q < kPodRows; ++q) {
            const long long r = base + (long long)q * kPodBlock;
            x[q] = r < n ? Si[r] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kPodRows; ++q) v[q] += w * x[q];
    }
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kPodRows; ++q) acc += v[q] * v[q];
    acc = wave_sum64(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The basis rows: Phi[r][j] = sum_i coef[i][j] S_i[r] for the n POD columns, and, when the
// new snapshot is kept, Phi[r][n] = v[r] / |v| (v as in k_pod_vnorm, same order of
// operations).  The decision to keep it is taken here from |v| and |u|: |v| > rtol |u|.
// coef rows have exactly JMAX entries (zero past the POD columns, v's combination last),
// so every column is accumulated without a test and the compiler reads each coefficient
// row with wide scalar loads.  A thread computes one row; the block's rows are staged in
// LDS and stored row-major with consecutive threads on consecutive addresses.  Columns
// >= j are not touched.
template <typename TP, int JMAX>
__global__ __launch_bounds__(kPodWrite) void k_pod_write(long long n, const double* __restrict__ S, int m,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ coef,
                                                         const double* __restrict__ vsq, double rtol,
                                                         PodInfo* __restrict__ info, TP* __restrict__ phi,
                                                         int ldphi) {
    constexpr int LT = JMAX + 1;
    __shared__ TP tile[kPodWrite * LT];
    const int np = info->n;
    int keep = 0;
    double scale = 0.0, vn = 0.0;
    if (u) {
        vn = sqrt(*vsq);
        keep = vn > rtol * info->unorm ? 1 : 0;
        scale = keep ? 1.0 / vn : 0.0;
    }
    const int j = np + keep;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        info->j = j;
        info->keep = keep;
        info->vnorm = vn;
    }
    const long long r0 = (long long)blockIdx.x * kPodWrite;
    const long long r = r0 + threadIdx.x;
    double acc[JMAX];
#pragma unroll
    for (int c = 0; c < JMAX; ++c) acc[c] = 0.0;
    if (r < n) {
        if (u) acc[JMAX - 1] = u[r];
        for (int i = 0; i < m; ++i) {
            const double x = S[(size_t)i * n + r];
            const double* ci = coef + (size_t)i * JMAX;
#pragma unroll
            for (int c = 0; c < JMAX; ++c) acc[c] += ci[c] * x;
        }
    }
    TP* row = tile + threadIdx.x * LT;
#pragma unroll
    for (int c = 0; c < JMAX; ++c)
        if (c < np) row[c] = (TP)acc[c];
    if (keep) row[np] = (TP)(acc[JMAX - 1] * scale);
    __syncthreads();
    const int nr = (int)min((long long)kPodWrite, n - r0);
    for (int e = threadIdx.x; e < nr * j; e += kPodWrite) {
        const int rr = e / j, c = e - rr * j;
        phi[(size_t)(r0 + rr) * ldphi + c] = tile[rr * LT + c];
    }
}

static int pod_chunks(long long n) {
    return (int)((n + (long long)kPodBlock * kPodRows - 1) / ((long long)kPodBlock * kPodRows));
}

// Coefficient row length (and register tile) for a basis of at most jbound columns.
static int pod_ldc(int jbound) {
    for (int J : {8, 16, 24, 32, 40}) if (jbound <= J) return J;
    return kPodMaxL + 1;
}

template <typename TP>
static void launch_pod_write(int ldc, long long n, const double* S, int m, const double* u, const double* coef,
                             const double* vsq, double rtol, PodInfo* info, TP* phi, int ldphi, hipStream_t s) {
    const dim3 grid((unsigned)((n + kPodWrite - 1) / kPodWrite));
#define TOPO_POD_WRITE(J)                                                                                  \
    hipLaunchKernelGGL((k_pod_write<TP, J>), grid, dim3(kPodWrite), 0, s, n, S, m, u, coef, vsq, rtol, info, \
                       phi, ldphi)
    switch (ldc) {
        case 8: TOPO_POD_WRITE(8); break;
        case 16: TOPO_POD_WRITE(16); break;
        case 24: TOPO_POD_WRITE(24); break;
        case 32: TOPO_POD_WRITE(32); break;
        case 40: TOPO_POD_WRITE(40); break;
        default: TOPO_POD_WRITE(kPodMaxL + 1); break;
    }
#undef TOPO_POD_WRITE
}

}  // namespace topo

using namespace topo;

extern "C" {

int topo_pod_push(topo_ctx* ctx, int64_t n, int32_t L, double* S, double* G, int32_t* count,
                  int32_t* next, const double* u, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    if (!S || !G || !count || !next || !u) return set_error(ctx, TOPO_EINVAL, "null pointer argument");
    if (n < 1 || L < 1 || L > kPodMaxL)
        return set_error(ctx, TOPO_EINVAL, "n >= 1 and 1 <= L <= %d required", kPodMaxL);
    const int c = *count, nx = *next;
    if (c < 0 || c > L || nx < 0 || nx >= L || (c < L && nx != 0))
        return set_error(ctx, TOPO_EINVAL, "window state (count %d, next %d) invalid for L = %d", c, nx, L);
    TOPO_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int slot = c < L ? c : nx;
    const int after = c < L ? c + 1 : L;
    const int nch = pod_chunks(n);
    Arena ar;
    double* part;
    ar.take(&part, (size_t)nch * (after + 1));
    int rc = ar.commit(ctx, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_pod_dots, dim3(nch), dim3(kPodBlock), 0, s, (long long)n, S, after, slot, 1, u, part);
    TOPO_CHECK_LAUNCH();
    launch_chunk_sum(after + 1, nch, 1, (const double*)part, GramRowOut{G, L, slot, after}, s);
    TOPO_CHECK_LAUNCH();
    *count = after;
    if (c == L) *next = (nx + 1) % L;
    return TOPO_OK;
}

int topo_pod_basis(topo_ctx* ctx, int64_t n, int32_t L, const double* S, const double* G, int32_t count,
                   const double* u, int32_t nmax, double rtol, void* phi, int32_t phi_fp32, int32_t ldphi,
                   int32_t* ncols, int32_t* npod, double* sigma, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    if (!phi || !ncols || (count > 0 && (!S || !G))) return set_error(ctx, TOPO_EINVAL, "null pointer argument");
    if (n < 1 || L < 1 || L > kPodMaxL)
        return set_error(ctx, TOPO_EINVAL, "n >= 1 and 1 <= L <= %d required", kPodMaxL);
    if (count < 0 || count > L) return set_error(ctx, TOPO_EINVAL, "count %d outside [0, L]", count);
    if (nmax < 0) return set_error(ctx, TOPO_EINVAL, "nmax must be >= 0");
    if (!(rtol >= 0.0 && rtol < 1.0)) return set_error(ctx, TOPO_EINVAL, "rtol must lie in [0, 1)");
    const int nb = std::min<int>(count, nmax);
    const int jbound = nb + (u ? 1 : 0);
    if (jbound < 1) return set_error(ctx, TOPO_EINVAL, "no column to build (empty window or nmax = 0, no snapshot)");
    if (ldphi < jbound) return set_error(ctx, TOPO_EINVAL, "ldphi %d < %d columns the basis may take", ldphi, jbound);
    TOPO_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const int m = count;
    const int ldc = pod_ldc(jbound);
    const int nch = pod_chunks(n);
    Arena ar;
    double *part, *gu, *vsq, *coef, *infod;
    ar.take(&part, (size_t)nch * (m + 1));
    ar.take(&gu, (size_t)m + 1);
    ar.take(&vsq, 1);
    ar.take(&coef, (size_t)(m + 1) * ldc);
    ar.take(&infod, (sizeof(PodInfo) + 7) / 8);
    int rc = ar.commit(ctx, s);
    if (rc) return rc;
    PodInfo* info = (PodInfo*)infod;
    if (u) {
        hipLaunchKernelGGL(k_pod_dots, dim3(nch), dim3(kPodBlock), 0, s, (long long)n, (double*)S, m, -1, 0, u,
                           part);
        TOPO_CHECK_LAUNCH();
        launch_chunk_sum(m + 1, nch, 1, (const double*)part, PodVecOut{gu}, s);
        TOPO_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_pod_eig, dim3(1), dim3(kEigThreads), 0, s, m, (int)L, G, u ? (const double*)gu : nullptr,
                       (int)nmax, rtol, coef, ldc, sigma, info);
    TOPO_CHECK_LAUNCH();
    if (u) {
        hipLaunchKernelGGL(k_pod_vnorm, dim3(nch), dim3(kPodBlock), 0, s, (long long)n, S, m, u,
                           (const double*)coef, ldc, part);
        TOPO_CHECK_LAUNCH();
        launch_chunk_sum(1, nch, 1, (const double*)part, PodVecOut{vsq}, s);
        TOPO_CHECK_LAUNCH();
    }
    if (phi_fp32)
        launch_pod_write<float>(ldc, n, S, m, u, coef, vsq, rtol, info, (float*)phi, ldphi, s);
    else
        launch_pod_write<double>(ldc, n, S, m, u, coef, vsq, rtol, info, (double*)phi, ldphi, s);
    TOPO_CHECK_LAUNCH();
    void* pin;
    rc = pinned_host(ctx, sizeof(PodInfo), &pin);
    if (rc) return rc;
    TOPO_HIP(hipMemcpyAsync(pin, info, sizeof(PodInfo), hipMemcpyDeviceToHost, s));
    TOPO_HIP(hipStreamSynchronize(s));
    const PodInfo h = *(const PodInfo*)pin;
    *ncols = h.j;
    if (npod) *npod = h.n;
    return TOPO_OK;
}

}  // extern "C"
