// Helmholtz density filter (Sec. 2.2) and the gradient through it (Sec. 2.4), on the
// nodal grid of the mesh, for B fields at once:
//   forward:  H phi = b(psi), b_n = w sum_{e ∋ n} psi_e,   rho_e = (1/nen) sum_{n ∈ e} phi_n
//   adjoint:  H mu = q(v),    q_n = (1/nen) sum_{e ∋ n} v_e,  g_e = w sum_{n ∈ e} mu_n
// with H = sum_e (r^2 L_e + M_e) the bilinear / trilinear Helmholtz matrix (homogeneous
// Neumann boundary: no constrained node), w = |Omega_e| / nen the entries of b_e.  H is
// symmetric, so both directions use one solver: Jacobi-PCG in float64, matrix-free.
//
// PCG per iteration in 3D: k_helm_apply3m forms the new direction p = z + beta p_old on
// the fly for its stencil (p double-buffered) and q = H p with per-block partials of
// p . q; k_helm_update advances x, r and z = D^-1 r with partials of r . z and r . r.  In
// 2D one kernel per iteration, k_helm_step2 (the single-reduction form of CG).  Each
// kernel sums the partials it needs itself, every block in the same fixed order (the
// partials are kept for two iterations, by parity).  A stopped field is left as it is
// from the first check, every kHelmCheck iterations, where |r| <= rtol |b|; the checks
// fall at the same iterations whatever the batch, so a field's result does not depend
// on its batch.  The iterations between checks are replayed as one graph.
#include <algorithm>
#include <cmath>

#include "graphs.hpp"
#include "internal.hpp"
#include "reduce.hpp"

namespace topo {

constexpr int kHelmBlock = 256;
// Nodes per thread in the PCG kernels: 4 in 3D (fewer block partials to sum), 1 in 2D
// (the 2D meshes are small: one node per thread keeps every CU busy).
template <int DIM>
constexpr int helm_npt() { return DIM == 3 ? 4 : 1; }
constexpr int kHelmCheck = 8;
constexpr int kHelmScal = 12;  // per-field scalars: rz (two copies), -, rr, bb, active, -, - (initial values);
                               // 2D one-reduction recursion: gamma by parity (8, 9), alpha by parity (10, 11)

// Element Helmholtz matrix of the box element, local node order x fastest.
struct HelmElem {
    double H[64];
    double S[27];  // assembled stencil of an interior node, offset (di, dj, dk) at 13 + di + 3 dj + 9 dk
    double w;      // |Omega_e| / nen
    double diag;   // H[0][0]: every diagonal entry is equal on a box
};

// H_e = r^2 (sum over axes of K1 (x) M1 (x) M1 with K1 on that axis) + M1 (x) M1 (x) M1,
// K1 = [1 -1; -1 1] / h, M1 = h [2 1; 1 2] / 6 per axis.
static HelmElem helm_element(const topo_mesh& m, double r) {
    HelmElem E{};
    const int d = m.dim, nen = 1 << d;
    double K1[3][2][2], M1[3][2][2];
    for (int a = 0; a < d; ++a) {
        const double h = m.h[a];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                K1[a][i][j] = (i == j ? 1.0 : -1.0) / h;
                M1[a][i][j] = h * (i == j ? 2.0 : 1.0) / 6.0;
            }
    }
    double vol = 1.0;
    for (int a = 0; a < d; ++a) vol *= m.h[a];
    for (int li = 0; li < nen; ++li)
        for (int lj = 0; lj < nen; ++lj) {
            double mass = 1.0, lap = 0.0;
            for (int a = 0; a < d; ++a) mass *= M1[a][(li >> a) & 1][(lj >> a) & 1];
            for (int a = 0; a < d; ++a) {
                double t = K1[a][(li >> a) & 1][(lj >> a) & 1];
                for (int c = 0; c < d; ++c)
                    if (c != a) t *= M1[c][(li >> c) & 1][(lj >> c) & 1];
                lap += t;
            }
            E.H[li * nen + lj] = r * r * lap + mass;
        }
    E.w = vol / nen;
    E.diag = E.H[0];
    // interior node: the rows of its 2^d elements, summed per neighbour offset
    for (int c = (d == 3 ? -1 : 0); c <= 0; ++c)
        for (int b = -1; b <= 0; ++b)
            for (int a = -1; a <= 0; ++a) {
                const int li = (-a) + 2 * (-b) + 4 * (-c);
                for (int lj = 0; lj < nen; ++lj) {
                    const int di = a + (lj & 1), dj = b + ((lj >> 1) & 1), dk = c + ((lj >> 2) & 1);
                    E.S[13 + di + 3 * dj + 9 * dk] += E.H[li * nen + lj];
                }
            }
    return E;
}

__device__ __forceinline__ void node_ijk(const Grid& g, int n, int& i, int& j, int& k) {
    const unsigned t = g.dnx1.div((unsigned)n), kk = g.dny1.div(t);
    i = n - (int)t * g.nx1;
    j = (int)(t - kk * (unsigned)g.ny1);
    k = (int)kk;
}

// out[b][n] = scale * sum over the elements around node n of in[b][e].
template <int DIM>
__global__ __launch_bounds__(kHelmBlock) void k_helm_e2n(Grid g, const double* __restrict__ in, double scale,
                                                         double* __restrict__ out) {
    const int n = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (n >= g.n_nodes) return;
    const double* ib = in + (size_t)blockIdx.y * g.n_elems;
    int i, j, k;
    node_ijk(g, n, i, j, k);
    double s = 0.0;
    for (int c = (DIM == 3 ? -1 : 0); c <= 0; ++c)
        for (int b = -1; b <= 0; ++b)
            for (int a = -1; a <= 0; ++a) {
                const int ei = i + a, ej = j + b, ek = k + c;
                if (ei < 0 || ej < 0 || ek < 0 || ei >= g.nx || ej >= g.ny || ek >= g.nz) continue;
                s += ib[ei + g.nx * (ej + g.ny * ek)];
            }
    out[(size_t)blockIdx.y * g.n_nodes + n] = scale * s;
}

// out[b][e] = scale * sum over the nodes of element e of in[b][n].
template <int DIM>
__global__ __launch_bounds__(kHelmBlock) void k_helm_n2e(Grid g, const double* __restrict__ in, double scale,
                                                         double* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= g.n_elems) return;
    const double* ib = in + (size_t)blockIdx.y * g.n_nodes;
    const int i = e % g.nx, t = e / g.nx, j = t % g.ny, k = t / g.ny;
    double s = 0.0;
    for (int c = 0; c < (DIM == 3 ? 2 : 1); ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) s += ib[(i + a) + g.nx1 * ((j + b) + g.ny1 * (k + c))];
    out[(size_t)blockIdx.y * g.n_elems + e] = scale * s;
}

// (H x)_n for the node (i, j, k): sum over the elements around it of their row.
template <int DIM, typename F>
__device__ __forceinline__ double helm_row(const Grid& g, const HelmElem& E, int i, int j, int k, F x) {
    constexpr int nen = 1 << DIM;
    double s = 0.0;
    for (int c = (DIM == 3 ? -1 : 0); c <= 0; ++c)
        for (int b = -1; b <= 0; ++b)
            for (int a = -1; a <= 0; ++a) {
                const int ei = i + a, ej = j + b, ek = k + c;
                if (ei < 0 || ej < 0 || ek < 0 || ei >= g.nx || ej >= g.ny || ek >= g.nz) continue;
                const int li = (-a) + 2 * (-b) + 4 * (-c);
                const double* row = E.H + li * nen;
#pragma unroll
                for (int lj = 0; lj < nen; ++lj) {
                    const int ni = ei + (lj & 1), nj = ej + ((lj >> 1) & 1), nk = ek + ((lj >> 2) & 1);
                    s += row[lj] * x(ni + g.nx1 * (nj + g.ny1 * nk));
                }
            }
    return s;
}

// Jacobi diagonal of node (i, j, k): the number of elements around it times H_e[0][0].
__device__ __forceinline__ double helm_dinv(const Grid& g, double diag, int i, int j, int k) {
    const int cx = (i > 0) + (i < g.nx), cy = (j > 0) + (j < g.ny);
    const int cz = g.dim == 3 ? (k > 0) + (k < g.nz) : 1;
    return 1.0 / (diag * (cx * cy * cz));
}

// r = bvec - H x (warm: x holds the initial guess) or x = 0, r = bvec; z = D^-1 r,
// p_old = 0; partials of r . z, r . r and b . b.
template <int DIM>
__global__ __launch_bounds__(kHelmBlock) void k_helm_init(Grid g, HelmElem E, int warm,
                                                          const double* __restrict__ bvec, double* __restrict__ x,
                                                          double* __restrict__ r, double* __restrict__ z,
                                                          double* __restrict__ p, double* __restrict__ part,
                                                          double* __restrict__ prz, double* __restrict__ prr) {
    __shared__ double lds[48];
    const int n0 = xcd_block(blockIdx.x, gridDim.x) * (helm_npt<DIM>() * kHelmBlock) + threadIdx.x;
    const size_t base = (size_t)blockIdx.y * g.n_nodes;
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < helm_npt<DIM>(); ++t) {
        const int n = n0 + t * kHelmBlock;
        if (n >= g.n_nodes) break;
        const size_t o = base + n;
        int i, j, k;
        node_ijk(g, n, i, j, k);
        const double bb = bvec[o];
        double rb = bb;
        if (warm) {
            const double* xb = x + base;
            rb -= helm_row<DIM>(g, E, i, j, k, [&](int m) { return xb[m]; });
        } else {
            x[o] = 0.0;
        }
        const double zz = rb * helm_dinv(g, E.diag, i, j, k);
        r[o] = rb;
        z[o] = zz;
        p[o] = 0.0;
        v[0] += rb * zz;
        v[1] += rb * rb;
        v[2] += bb * bb;
    }
    block_reduce<3>(v, lds);
    if (threadIdx.x == 0) {
        const size_t bi = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        double* pb = part + bi * 3;
        pb[0] = v[0];
        pb[1] = v[1];
        pb[2] = v[2];
        prz[bi] = v[0];
        prr[bi] = v[1];
    }
}

// beta = rz / rz_prev from the update's block partials of field blockIdx.y (every block
// sums them in the same order); 0 on the first iteration or when r = 0 exactly.
__device__ __forceinline__ double helm_beta(int first, int nrz, const double* rz_cur, const double* rz_prev,
                                            double* lds) {
    if (first) return 0.0;
    const double rc = block_sum_array(rz_cur + (size_t)blockIdx.y * nrz, nrz, lds);
    const double rp = block_sum_array(rz_prev + (size_t)blockIdx.y * nrz, nrz, lds);
    return rp == 0.0 ? 0.0 : rc / rp;
}

// p_new = z + beta p_old (beta = rz / rz_prev, 0 on the first iteration), q = H p_new,
// partials of p_new . q.
template <int DIM>
__global__ __launch_bounds__(kHelmBlock) void k_helm_apply(Grid g, HelmElem E, int first, int nrz,
                                                           const double* __restrict__ rz_cur,
                                                           const double* __restrict__ rz_prev,
                                                           const double* __restrict__ z,
                                                           const double* __restrict__ pold,
                                                           double* __restrict__ pnew, double* __restrict__ q,
                                                           double* __restrict__ ppq) {
    __shared__ double lds[32];
    const int nb = gridDim.x;
    const int n0 = xcd_block(blockIdx.x, nb) * (helm_npt<DIM>() * kHelmBlock) + threadIdx.x;
    const size_t base = (size_t)blockIdx.y * g.n_nodes;
    const double* zb = z + base;
    const double* pb = pold + base;
    double v[1] = {0.0};
    if (DIM == 2) {
        // one node per thread: its 3 x 3 neighbourhood is loaded before beta is summed
        const int n = n0;
        const bool in = n < g.n_nodes;
        int i = 0, j = 0, k = 0;
        if (in) node_ijk(g, n, i, j, k);
        const bool interior = in && i > 0 && i < g.nx && j > 0 && j < g.ny;
        double zn[9], pn9[9];
        if (interior) {
#pragma unroll
            for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
                for (int di = -1; di <= 1; ++di) {
                    const int m = n + di + g.nx1 * dj;
                    zn[4 + di + 3 * dj] = zb[m];
                    pn9[4 + di + 3 * dj] = pb[m];
                }
        }
        const double beta = helm_beta(first, nrz, rz_cur, rz_prev, lds);
        if (in) {
            double pn, qn = 0.0;
            if (interior) {
                pn = zn[4] + beta * pn9[4];
#pragma unroll
                for (int e = 0; e < 9; ++e) qn += E.S[13 + (e % 3 - 1) + 3 * (e / 3 - 1)] * (zn[e] + beta * pn9[e]);
            } else {
                pn = zb[n] + beta * pb[n];
                qn = helm_row<DIM>(g, E, i, j, k, [&](int m) { return zb[m] + beta * pb[m]; });
            }
            pnew[base + n] = pn;
            q[base + n] = qn;
            v[0] += pn * qn;
        }
    } else {
        const double beta = helm_beta(first, nrz, rz_cur, rz_prev, lds);
        for (int t = 0; t < helm_npt<DIM>(); ++t) {
            const int n = n0 + t * kHelmBlock;
            if (n >= g.n_nodes) break;
            int i, j, k;
            node_ijk(g, n, i, j, k);
            const double pn = zb[n] + beta * pb[n];
            const double qn = helm_row<DIM>(g, E, i, j, k, [&](int m) { return zb[m] + beta * pb[m]; });
            pnew[base + n] = pn;
            q[base + n] = qn;
            v[0] += pn * qn;
        }
    }
    block_reduce<1>(v, lds);
    if (threadIdx.x == 0) ppq[(size_t)blockIdx.y * nb + blockIdx.x] = v[0];
}

// 3D apply as a march: a block owns a 32 x 8 tile of node columns over a run of z planes
// and keeps three planes of v = z + beta p_old (tile plus a one-node halo) in LDS, so each
// value is formed once per block instead of once per neighbour; interior nodes take the
// 27-point stencil from LDS, boundary nodes the element rows from global memory.  Same
// outputs as k_helm_apply: p_new and q of the owned nodes, partials of p_new . q.
constexpr int kHX = 32, kHY = 8, kHLX = kHX + 2, kHLY = kHY + 2;
struct HelmMarch {
    int tx, ty, chunks, kz;  // tiles along x and y, z chunks, planes per chunk
};
static HelmMarch helm_march(const Grid& g) {
    HelmMarch h;
    h.tx = (g.nx1 + kHX - 1) / kHX;
    h.ty = (g.ny1 + kHY - 1) / kHY;
    const int target = 1024;  // about four blocks per CU
    const int want = std::max(1, target / (h.tx * h.ty));
    h.kz = std::max(2, (g.nz1 + want - 1) / want);
    h.chunks = (g.nz1 + h.kz - 1) / h.kz;
    return h;
}

__global__ __launch_bounds__(kHelmBlock) void k_helm_apply3m(Grid g, HelmElem E, HelmMarch hm, int first, int nrz,
                                                             const double* __restrict__ rz_cur,
                                                             const double* __restrict__ rz_prev,
                                                             const double* __restrict__ z,
                                                             const double* __restrict__ pold,
                                                             double* __restrict__ pnew, double* __restrict__ q,
                                                             double* __restrict__ ppq) {
    __shared__ double lds[32];
    __shared__ double pl[3][kHLY][kHLX];
    const int nb = gridDim.x;
    const int lb = xcd_block(blockIdx.x, nb);
    const int txi = lb % hm.tx, t2 = lb / hm.tx, tyi = t2 % hm.ty, ch = t2 / hm.ty;
    const int i0 = txi * kHX, j0 = tyi * kHY, k0 = ch * hm.kz, k1 = min(k0 + hm.kz, g.nz1);
    const size_t base = (size_t)blockIdx.y * g.n_nodes;
    const double beta = helm_beta(first, nrz, rz_cur, rz_prev, lds);
    const double* zb = z + base;
    const double* pb = pold + base;
    const int lx = threadIdx.x % kHX, ly = threadIdx.x / kHX;
    const int i = i0 + lx, j = j0 + ly;
    const int sy = g.nx1, sz = g.nx1 * g.ny1;
    auto load_plane = [&](int k, int slot) {
        for (int e = threadIdx.x; e < kHLX * kHLY; e += kHelmBlock) {
            const int ex = e % kHLX, ey = e / kHLX;
            const int gi = i0 - 1 + ex, gj = j0 - 1 + ey;
            double val = 0.0;
            if (k >= 0 && k < g.nz1 && gi >= 0 && gi < g.nx1 && gj >= 0 && gj < g.ny1) {
                const int m = gi + sy * gj + sz * k;
                val = zb[m] + beta * pb[m];
            }
            pl[slot][ey][ex] = val;
        }
    };
    load_plane(k0 - 1, (k0 + 2) % 3);
    load_plane(k0, k0 % 3);
    double v[1] = {0.0};
    for (int k = k0; k < k1; ++k) {
        load_plane(k + 1, (k + 1) % 3);
        __syncthreads();
        if (i < g.nx1 && j < g.ny1) {
            const int n = i + sy * j + sz * k;
            const double pn = pl[k % 3][ly + 1][lx + 1];
            double qn = 0.0;
            if (i > 0 && i < g.nx && j > 0 && j < g.ny && k > 0 && k < g.nz) {
#pragma unroll
                for (int dk = -1; dk <= 1; ++dk) {
                    const int slot = (k + dk + 3) % 3;
#pragma unroll
                    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
                        for (int di = -1; di <= 1; ++di)
                            qn += E.S[13 + di + 3 * dj + 9 * dk] * pl[slot][ly + 1 + dj][lx + 1 + di];
                }
            } else {
                qn = helm_row<3>(g, E, i, j, k, [&](int m) { return zb[m] + beta * pb[m]; });
            }
            pnew[base + n] = pn;
            q[base + n] = qn;
            v[0] += pn * qn;
        }
        __syncthreads();  // the oldest plane is overwritten next
    }
    block_reduce<1>(v, lds);
    if (threadIdx.x == 0) ppq[(size_t)blockIdx.y * nb + blockIdx.x] = v[0];
}

// For an active field alpha = rz / pq, x += alpha p, r -= alpha q, z = D^-1 r; partials
// of r . z and r . r.
template <int DIM>
__global__ __launch_bounds__(kHelmBlock) void k_helm_update(Grid g, double diag, const double* __restrict__ sc,
                                                            int npq, const double* __restrict__ rz_cur,
                                                            const double* __restrict__ ppq,
                                                            const double* __restrict__ p,
                                                            const double* __restrict__ q,
                                                            double* __restrict__ x, double* __restrict__ r,
                                                            double* __restrict__ z, double* __restrict__ rz_new,
                                                            double* __restrict__ rr_new) {
    __shared__ double lds[32];
    const int nb = gridDim.x;
    const int n0 = xcd_block(blockIdx.x, nb) * (helm_npt<DIM>() * kHelmBlock) + threadIdx.x;
    constexpr int NPT = helm_npt<DIM>();
    // A stopped field is left as it is (its p may be meaningless, e.g. 0/0 for b = 0).
    const bool active = sc[blockIdx.y * kHelmScal + 5] != 0.0;
    // the node values are loaded before the partial sums, so both latencies overlap
    double xv[NPT], rv[NPT], zv[NPT], pv[NPT], qv[NPT];
#pragma unroll
    for (int t = 0; t < NPT; ++t) {
        const int n = n0 + t * kHelmBlock;
        if (n < g.n_nodes) {
            const size_t o = (size_t)blockIdx.y * g.n_nodes + n;
            xv[t] = x[o];
            rv[t] = r[o];
            zv[t] = z[o];
            pv[t] = p[o];
            qv[t] = q[o];
        }
    }
    const double rz = block_sum_array(rz_cur + (size_t)blockIdx.y * nb, nb, lds);
    const double pq = block_sum_array(ppq + (size_t)blockIdx.y * npq, npq, lds);
    const double alpha = pq != 0.0 ? rz / pq : 0.0;
    double v[2] = {0.0, 0.0};
#pragma unroll
    for (int t = 0; t < NPT; ++t) {
        const int n = n0 + t * kHelmBlock;
        if (n >= g.n_nodes) break;
        const size_t o = (size_t)blockIdx.y * g.n_nodes + n;
        double rn = rv[t], zn = zv[t];
        if (active) {
            int i, j, k;
            node_ijk(g, n, i, j, k);
            x[o] = xv[t] + alpha * pv[t];
            rn -= alpha * qv[t];
            zn = rn * helm_dinv(g, diag, i, j, k);
            r[o] = rn;
            z[o] = zn;
        }
        v[0] += rn * zn;
        v[1] += rn * rn;
    }
    block_reduce<2>(v, lds);
    if (threadIdx.x == 0) {
        rz_new[(size_t)blockIdx.y * nb + blockIdx.x] = v[0];
        rr_new[(size_t)blockIdx.y * nb + blockIdx.x] = v[1];
    }
}

// 2D: one kernel per iteration (the one-reduction form of CG, as in the 2D elasticity
// solve).  With u = D^-1 r, w = H u and s = H p carried by s_i = w_i + beta_i s_{i-1},
// beta_i = gamma_i / gamma_{i-1} and alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1})
// (gamma = r.u, delta = w.u) come from the previous launch's partials.  A step rebuilds
// u_{i+1} = D^-1 (r_i - alpha_i (w_i + beta_i s_{i-1})) on its node's neighbourhood, updates
// s, r, p, x of its node (r, w, s double-buffered by parity) and forms w_{i+1} = H u_{i+1};
// partials of gamma, delta and r.r of the new residual.  Stopped fields are left as they
// are.  Block 0 of a field records gamma_i, alpha_i by parity (read back one step later).
__global__ __launch_bounds__(kHelmBlock) void k_helm_step2(Grid g, HelmElem E, int first, int cur,
                                                           const double* __restrict__ Rin,
                                                           const double* __restrict__ Win,
                                                           const double* __restrict__ Sin,
                                                           double* __restrict__ Rout, double* __restrict__ Wout,
                                                           double* __restrict__ Sout, double* __restrict__ P,
                                                           double* __restrict__ x, double* __restrict__ sc,
                                                           const double* __restrict__ gam_cur,
                                                           const double* __restrict__ dlt_cur,
                                                           double* __restrict__ gam_nxt, double* __restrict__ dlt_nxt,
                                                           double* __restrict__ rr_nxt) {
    __shared__ double lds[48];
    double* f = sc + (size_t)blockIdx.y * kHelmScal;
    if (f[5] == 0.0) return;
    const int nb = gridDim.x;
    const int n = xcd_block(blockIdx.x, nb) * kHelmBlock + threadIdx.x;
    const size_t base = (size_t)blockIdx.y * g.n_nodes;
    const double *rb = Rin + base, *wb = Win + base, *sb = Sin + base;
    const bool in = n < g.n_nodes;
    int i = 0, j = 0, k = 0;
    if (in) node_ijk(g, n, i, j, k);
    const bool interior = in && i > 0 && i < g.nx && j > 0 && j < g.ny;
    // the node's loads (its 3 x 3 neighbourhood inside the grid) before the partial sums
    double rn9[9], wn9[9], sn9[9];
    double pv = 0.0, xv = 0.0;
    if (interior) {
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
            for (int di = -1; di <= 1; ++di) {
                const int m = n + di + g.nx1 * dj;
                rn9[4 + di + 3 * dj] = rb[m];
                wn9[4 + di + 3 * dj] = wb[m];
                sn9[4 + di + 3 * dj] = sb[m];
            }
    } else if (in) {
        rn9[4] = rb[n];
        wn9[4] = wb[n];
        sn9[4] = sb[n];
    }
    if (in) {
        pv = P[base + n];
        xv = x[base + n];
    }
    const double* arrs[2] = {gam_cur + (size_t)blockIdx.y * nb, dlt_cur + (size_t)blockIdx.y * nb};
    double red[2];
    block_sum_arrays<2>(arrs, nb, red, lds);
    const double gam = red[0], dlt = red[1];
    const int prv = cur ^ 1;
    double be = 0.0, den = dlt;
    if (!first) {
        const double gp = f[8 + prv], ap = f[10 + prv];
        be = gp != 0.0 ? gam / gp : 0.0;
        den = dlt - (ap != 0.0 ? be * gam / ap : 0.0);
    }
    // alpha = 0 (no step) once gamma is exactly 0 or the denominator is not positive
    double ah = den > 0.0 ? gam / den : 0.0;
    if (!isfinite(ah) || !isfinite(be)) ah = be = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        f[8 + cur] = gam;
        f[10 + cur] = ah;
    }
    double v[3] = {0.0, 0.0, 0.0};
    if (in) {
        auto unew = [&](double r, double w, double s_, int ii, int jj) {
            return (r - ah * (w + be * s_)) * helm_dinv(g, E.diag, ii, jj, 0);
        };
        const double si = wn9[4] + be * sn9[4];
        const double rnew = rn9[4] - ah * si;
        const double dv = helm_dinv(g, E.diag, i, j, 0);
        const double uown = rnew * dv;
        const double pn = rn9[4] * dv + be * pv;  // u_i + beta p_{i-1}
        double wn = 0.0;
        if (interior) {
#pragma unroll
            for (int e = 0; e < 9; ++e)
                wn += E.S[13 + (e % 3 - 1) + 3 * (e / 3 - 1)] *
                      unew(rn9[e], wn9[e], sn9[e], i + e % 3 - 1, j + e / 3 - 1);
        } else {
            wn = helm_row<2>(g, E, i, j, k, [&](int m) {
                return unew(rb[m], wb[m], sb[m], m % g.nx1, m / g.nx1);
            });
        }
        P[base + n] = pn;
        x[base + n] = xv + ah * pn;
        Sout[base + n] = si;
        Rout[base + n] = rnew;
        Wout[base + n] = wn;
        v[0] = rnew * uown;
        v[1] = wn * uown;
        v[2] = rnew * rnew;
    }
    block_reduce<3>(v, lds);
    if (threadIdx.x == 0) {
        const size_t o = (size_t)blockIdx.y * nb + blockIdx.x;
        gam_nxt[o] = v[0];
        dlt_nxt[o] = v[1];
        rr_nxt[o] = v[2];
    }
}

// Chunk-sum epilogue of the initial residual into the per-field scalars.
struct HelmInitOut {  // entries: r.z, r.r of the initial residual, b.b
    double* sc;
    __device__ void operator()(int b, int e, double s) const {
        double* f = sc + b * kHelmScal;
        if (e == 0) {
            f[0] = s;
            f[1] = s;
        } else if (e == 1) {
            f[3] = s;
        } else {
            f[4] = s;
        }
    }
};
// A field starts active unless its initial residual already meets the tolerance.
__global__ void k_helm_start(int B, double rtol2, double* __restrict__ sc) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double* f = sc + b * kHelmScal;
    f[5] = (f[4] > 0.0 && f[3] > rtol2 * f[4]) ? 1.0 : 0.0;
}

// Stop the fields that have converged (|r|^2 <= rtol^2 |b|^2, r.r summed from the block
// partials); count the active ones; record iterations.  One block per field.
__global__ __launch_bounds__(kHelmBlock) void k_helm_check(int nb, double rtol2, int it,
                                                           const double* __restrict__ prr,
                                                           double* __restrict__ sc, int* __restrict__ nactive,
                                                           int* __restrict__ iters) {
    __shared__ double lds[32];
    const int b = blockIdx.x;
    const double rr = block_sum_array(prr + (size_t)b * nb, nb, lds);
    if (threadIdx.x != 0) return;
    double* f = sc + b * kHelmScal;
    if (f[5] == 0.0) return;
    iters[b] = it;
    if (rr <= rtol2 * f[4]) f[5] = 0.0;
    else atomicAdd(nactive, 1);
}

// Workspace of one filter call (all pieces from one arena: every arena starts at the
// beginning of the context's workspace).
struct HelmWork {
    double *bvec, *x, *r, *z, *p0, *p1, *q, *part, *sc;
    double *prz, *prr, *ppq;  // block partials of r.z and r.r ([2][B][nb], by iteration parity), p.q
    double *e0, *e1, *pdl;    // 2D: two more vectors and the partials of w.u ([2][B][nb])
    int *cnt, *its;
};

template <int DIM>
static int helm_solve(Ctx* ctx, const Grid& g, const HelmElem& E, int B, const HelmWork& w, bool warm,
                      double rtol, int maxit, int* iters_out, hipStream_t s) {
    const int nb = grid_blocks(g.n_nodes, helm_npt<DIM>() * kHelmBlock);
    double *x = w.x, *r = w.r, *z = w.z, *p0 = w.p0, *p1 = w.p1, *q = w.q, *part = w.part, *sc = w.sc;
    int *cnt = w.cnt, *its = w.its;
    const double* bvec = w.bvec;
    void* pin;
    int rc = pinned_host(ctx, sizeof(int) * std::max(B, 2), &pin);
    if (rc) return rc;
    const dim3 grid(nb, B);
    const size_t BN = (size_t)B * nb;
    const HelmMarch hm = helm_march(g);
    const int nbm = hm.tx * hm.ty * hm.chunks;  // blocks of the 3D march apply
    const int npq = DIM == 3 ? nbm : nb;        // its partials of p . q per field
    hipLaunchKernelGGL(k_helm_init<DIM>, grid, dim3(kHelmBlock), 0, s, g, E, warm ? 1 : 0, bvec, x, r, z, p0,
                       part, w.prz, w.prr);
    TOPO_CHECK_LAUNCH();
    launch_chunk_sum(3, nb, B, (const double*)part, HelmInitOut{sc}, s);
    TOPO_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_helm_start, dim3((B + 63) / 64), dim3(64), 0, s, B, rtol * rtol, sc);
    TOPO_CHECK_LAUNCH();
    TOPO_HIP(hipMemsetAsync(its, 0, sizeof(int) * B, s));
    int it = 0, active = B;
    // One iteration's launches: 2D the one-kernel step (r, w, s double-buffered by parity,
    // p in place), 3D the march apply and the update (p_old / p_new by parity).
    double* R2[2] = {r, z};
    double* W2[2] = {q, w.e0};
    double* S2[2] = {p0, w.e1};
    auto iteration = [&](LaunchSink& L, int at) {
        const int cur = at & 1, nxt = cur ^ 1;
        const int first = at == 0 ? 1 : 0;
        if constexpr (DIM == 2) {
            L((const void*)k_helm_step2, grid, dim3(kHelmBlock), g, E, first, cur, (const double*)R2[cur],
              (const double*)W2[cur], (const double*)S2[cur], R2[nxt], W2[nxt], S2[nxt], p1, x, sc,
              (const double*)(w.prz + (size_t)cur * BN), (const double*)(w.pdl + (size_t)cur * BN),
              w.prz + (size_t)nxt * BN, w.pdl + (size_t)nxt * BN, w.prr + (size_t)nxt * BN);
        } else {
            double* pold = cur ? p1 : p0;
            double* pnew = cur ? p0 : p1;
            const double* rz_cur = w.prz + (size_t)cur * BN;
            const double* rz_prev = w.prz + (size_t)nxt * BN;
            L((const void*)k_helm_apply3m, dim3(nbm, B), dim3(kHelmBlock), g, E, hm, first, nb, rz_cur, rz_prev,
              (const double*)z, (const double*)pold, pnew, q, w.ppq);
            L((const void*)k_helm_update<3>, grid, dim3(kHelmBlock), g, E.diag, (const double*)sc, npq, rz_cur,
              (const double*)w.ppq, (const double*)pnew, (const double*)q, x, r, z, w.prz + (size_t)nxt * BN,
              w.prr + (size_t)nxt * BN);
        }
    };
    // Graph of kHelmCheck iterations (even, so that every replay keeps the parity); the
    // first chunk differs by its first iteration's flag.
    auto chunk_graph = [&](bool first_chunk, hipGraphExec_t* out) -> int {
        std::vector<uintptr_t> key = {(uintptr_t)0xF17, (uintptr_t)DIM, (uintptr_t)first_chunk, (uintptr_t)B,
                                      (uintptr_t)g.nx, (uintptr_t)g.ny, (uintptr_t)g.nz, (uintptr_t)nb,
                                      (uintptr_t)nbm, (uintptr_t)x, (uintptr_t)r, (uintptr_t)z, (uintptr_t)p0,
                                      (uintptr_t)p1, (uintptr_t)q, (uintptr_t)w.e0, (uintptr_t)w.e1,
                                      (uintptr_t)w.prz, (uintptr_t)w.prr, (uintptr_t)w.pdl, (uintptr_t)w.ppq,
                                      (uintptr_t)sc};
        uint64_t words[(sizeof(HelmElem) + 7) / 8] = {};
        std::memcpy(words, &E, sizeof(HelmElem));
        for (uint64_t v : words) key.push_back((uintptr_t)v);
        return cached_graph(ctx, key, [&](LaunchSink& G) {
            for (int c = 0; c < kHelmCheck; ++c) iteration(G, first_chunk ? c : kHelmCheck + c);
        }, out, s);
    };
    // The check after a chunk stops the converged fields on the device (their later
    // launches return at once) and counts the active ones; the host reads the count one
    // chunk behind, so it never waits for the chunk it has just launched.
    int* hp = (int*)pin;
    hipEvent_t ev[2];
    TOPO_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    TOPO_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    auto launch_check = [&](int at, int sl) -> int {
        TOPO_HIP(hipMemsetAsync(cnt + sl, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_helm_check, dim3(B), dim3(kHelmBlock), 0, s, nb, rtol * rtol, at,
                           (const double*)(w.prr + (size_t)(at & 1) * BN), sc, cnt + sl, its);
        TOPO_CHECK_LAUNCH();
        TOPO_HIP(hipMemcpyAsync(hp + sl, cnt + sl, sizeof(int), hipMemcpyDeviceToHost, s));
        TOPO_HIP(hipEventRecord(ev[sl], s));
        return TOPO_OK;
    };
    if (warm) {  // a guess that already meets the tolerance needs no iteration
        rc = launch_check(0, 0);
        if (rc) return rc;
        TOPO_HIP(hipEventSynchronize(ev[0]));
        active = hp[0];
    }
    if (DIM == 2 && active > 0) {
        // w_0 = H D^-1 r_0 and the partials of delta_0 = w_0 . u_0: the apply with beta = 0
        // (p_old = S[0] is zero from the initialisation; p_new = z_0 lands in p, where the
        // first step's beta = 0 meets it)
        hipLaunchKernelGGL(k_helm_apply<2>, grid, dim3(kHelmBlock), 0, s, g, E, 1, nb, (const double*)w.prz,
                           (const double*)w.prz, (const double*)z, (const double*)p0, p1, q, w.pdl);
        TOPO_CHECK_LAUNCH();
    }
    LaunchSink L;
    L.s = s;
    bool pending[2] = {false, false};
    int slot = 0;
    while (active > 0 && it < maxit) {
        const int n_it = std::min(kHelmCheck, maxit - it);
        if (graphs_enabled() && n_it == kHelmCheck) {
            hipGraphExec_t exec = nullptr;
            rc = chunk_graph(it == 0, &exec);
            if (rc) return rc;
            TOPO_HIP(hipGraphLaunch(exec, s));
        } else {
            for (int c = 0; c < n_it; ++c) iteration(L, it + c);
            TOPO_HIP(L.err);
        }
        it += n_it;
        rc = launch_check(it, slot);
        if (rc) return rc;
        pending[slot] = true;
        if (it >= maxit) {  // the last check decides
            TOPO_HIP(hipEventSynchronize(ev[slot]));
            active = hp[slot];
            break;
        }
        const int other = slot ^ 1;
        if (pending[other]) {
            TOPO_HIP(hipEventSynchronize(ev[other]));
            pending[other] = false;
            if (hp[other] == 0) {
                active = 0;
                break;
            }
        }
        slot = other;
    }
    TOPO_HIP(hipStreamSynchronize(s));
    TOPO_HIP(hipEventDestroy(ev[0]));
    TOPO_HIP(hipEventDestroy(ev[1]));
    TOPO_HIP(hipMemcpyAsync(pin, its, sizeof(int) * B, hipMemcpyDeviceToHost, s));
    TOPO_HIP(hipStreamSynchronize(s));
    int mx = 0;
    for (int b = 0; b < B; ++b) mx = std::max(mx, ((const int*)pin)[b]);
    if (iters_out) *iters_out = mx;
    if (active > 0) return set_error(ctx, TOPO_ENOCONV, "filter solve: %d field(s) not converged in %d iterations",
                                     active, maxit);
    return TOPO_OK;
}

static int filter_checks(Ctx* ctx, const topo_mesh* mesh, double r, const void* in, int B, const void* out,
                         double rtol, int maxit) {
    int rc = validate_mesh(ctx, mesh);
    if (rc) return rc;
    if (!in || !out) return set_error(ctx, TOPO_EINVAL, "null pointer argument");
    if (B < 1) return set_error(ctx, TOPO_EINVAL, "B must be >= 1");
    if (!(r >= 0.0) || !std::isfinite(r)) return set_error(ctx, TOPO_EINVAL, "filter length r must be >= 0");
    if (!(rtol > 0.0 && rtol < 1.0)) return set_error(ctx, TOPO_EINVAL, "rtol must lie in (0, 1)");
    if (maxit < 1) return set_error(ctx, TOPO_EINVAL, "maxit must be >= 1");
    return TOPO_OK;
}

template <int DIM>
static int filter_run(Ctx* ctx, const topo_mesh& m, double r, const double* in, int B, double* out,
                      double* nodal, bool warm, double rtol, int maxit, int* iters, bool adjoint, hipStream_t s) {
    const Grid g = make_grid(m);
    const HelmElem E = helm_element(m, r);
    constexpr int nen = 1 << DIM;
    const int nb = grid_blocks(g.n_nodes, helm_npt<DIM>() * kHelmBlock);
    const size_t NV = (size_t)B * g.n_nodes;
    HelmWork w{};
    Arena ar;
    ar.take(&w.bvec, NV);
    if (!nodal) ar.take(&w.x, NV);
    ar.take(&w.r, NV);
    ar.take(&w.z, NV);
    ar.take(&w.p0, NV);
    ar.take(&w.p1, NV);
    ar.take(&w.q, NV);
    ar.take(&w.part, (size_t)B * nb * 3);
    ar.take(&w.prz, (size_t)2 * B * nb);
    ar.take(&w.prr, (size_t)2 * B * nb);
    ar.take(&w.ppq, (size_t)B * std::max(nb, DIM == 3 ? helm_march(g).tx * helm_march(g).ty * helm_march(g).chunks : 0));
    ar.take(&w.sc, (size_t)B * kHelmScal);
    if (DIM == 2) {
        ar.take(&w.e0, NV);
        ar.take(&w.e1, NV);
        ar.take(&w.pdl, (size_t)2 * B * nb);
    }
    ar.take(&w.cnt, 2);  // active-field counters of two checks in flight
    ar.take(&w.its, (size_t)B);
    int rc = ar.commit(ctx, s);
    if (rc) return rc;
    if (nodal) w.x = nodal;
    const dim3 gn(grid_blocks(g.n_nodes, kHelmBlock), B), ge(grid_blocks(g.n_elems, kHelmBlock), B);
    hipLaunchKernelGGL(k_helm_e2n<DIM>, gn, dim3(kHelmBlock), 0, s, g, in, adjoint ? 1.0 / nen : E.w, w.bvec);
    TOPO_CHECK_LAUNCH();
    rc = helm_solve<DIM>(ctx, g, E, B, w, warm && nodal, rtol, maxit, iters, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_helm_n2e<DIM>, ge, dim3(kHelmBlock), 0, s, g, (const double*)w.x,
                       adjoint ? E.w : 1.0 / nen, out);
    TOPO_CHECK_LAUNCH();
    return TOPO_OK;
}

}  // namespace topo

using namespace topo;

extern "C" {

int topo_filter_forward(topo_ctx* ctx, const topo_mesh* mesh, double r, const double* psi, int32_t B,
                        double* rho, double* phi, double rtol, int32_t maxit, int32_t flags, int32_t* iters,
                        void* stream) {
    if (!ctx) return TOPO_EINVAL;
    int rc = filter_checks(ctx, mesh, r, psi, B, rho, rtol, maxit);
    if (rc) return rc;
    TOPO_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const bool warm = (flags & TOPO_FILTER_WARM) != 0;
    return mesh->dim == 2 ? filter_run<2>(ctx, *mesh, r, psi, B, rho, phi, warm, rtol, maxit, iters, false, s)
                          : filter_run<3>(ctx, *mesh, r, psi, B, rho, phi, warm, rtol, maxit, iters, false, s);
}

int topo_filter_adjoint(topo_ctx* ctx, const topo_mesh* mesh, double r, const double* v, int32_t B, double* g,
                        double* mu, double rtol, int32_t maxit, int32_t flags, int32_t* iters, void* stream) {
    if (!ctx) return TOPO_EINVAL;
    int rc = filter_checks(ctx, mesh, r, v, B, g, rtol, maxit);
    if (rc) return rc;
    TOPO_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    const bool warm = (flags & TOPO_FILTER_WARM) != 0;
    return mesh->dim == 2 ? filter_run<2>(ctx, *mesh, r, v, B, g, mu, warm, rtol, maxit, iters, true, s)
                          : filter_run<3>(ctx, *mesh, r, v, B, g, mu, warm, rtol, maxit, iters, true, s);
}

}  // extern "C"
