// Context, workspace arena, element tables and argument validation.
#include <algorithm>
#include <cmath>
#include <cstdarg>

#include "internal.hpp"

namespace topo {

Grid make_grid(const topo_mesh& m) {
    Grid g;
    g.dim = m.dim;
    g.nx = m.nel[0];
    g.ny = m.nel[1];
    g.nz = m.dim == 3 ? m.nel[2] : 1;
    g.nx1 = g.nx + 1;
    g.ny1 = g.ny + 1;
    g.nz1 = m.dim == 3 ? g.nz + 1 : 1;
    g.n_nodes = g.nx1 * g.ny1 * g.nz1;
    g.n_elems = g.nx * g.ny * g.nz;
    g.n_dofs = (long long)g.dim * g.n_nodes;
    g.dnx1 = make_fastdiv((unsigned)g.nx1);
    g.dny1 = make_fastdiv((unsigned)g.ny1);
    return g;
}

int march3_target(const Ctx* ctx, const void* kernel) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess ||
        per_cu < 1 || ctx->cu_count < 1) {
        (void)hipGetLastError();
        return 1024;
    }
    return per_cu * ctx->cu_count;
}

// Element stiffness of the rectangular bilinear / trilinear element written as sums
// of tensor products of exact 1D integrals of the linear shape functions
// f0 = 1 - x/h, f1 = x/h on [0, h]:
//   mass  M[a][b] = int f_a f_b     = h/3 (a == b), h/6 (a != b)
//   stiff S[a][b] = int f_a' f_b'   = +1/h (a == b), -1/h (a != b)
//   mixed G[a][b] = int f_a' f_b    = s(a)/2 with s(0) = -1, s(1) = +1.
// The strain energy of the element (Sec. 2.1) then gives every entry in closed form.
void element_stiffness(const topo_mesh& m, std::vector<double>& K) {
    const int dim = m.dim;
    const int nen = 1 << dim;
    const int ne = dim * nen;
    K.assign((size_t)ne * ne, 0.0);
    double M[3][2][2], S[3][2][2], G[3][2][2];
    for (int ax = 0; ax < dim; ++ax) {
        const double h = m.h[ax];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                M[ax][a][b] = (a == b) ? h / 3.0 : h / 6.0;
                S[ax][a][b] = (a == b) ? 1.0 / h : -1.0 / h;
                G[ax][a][b] = (a == 0 ? -1.0 : 1.0) / 2.0;
            }
    }
    // I(a, b, da, db) = int (d_da N_a)(d_db N_b); da/db = -1 means no derivative.
    auto I = [&](int a, int b, int da, int db) {
        double v = 1.0;
        for (int ax = 0; ax < dim; ++ax) {
            const int ia = (a >> ax) & 1, ib = (b >> ax) & 1;
            if (da == ax && db == ax) v *= S[ax][ia][ib];
            else if (da == ax) v *= G[ax][ia][ib];
            else if (db == ax) v *= G[ax][ib][ia];
            else v *= M[ax][ia][ib];
        }
        return v;
    };
    const double E = 1.0, nu = m.nu;
    if (dim == 2) {
        double D11, D12, D33;
        if (m.plane == 0) {  // plane stress
            const double c = E / (1.0 - nu * nu);
            D11 = c;
            D12 = c * nu;
            D33 = c * (1.0 - nu) / 2.0;
        } else {  // plane strain
            const double c = E / ((1.0 + nu) * (1.0 - 2.0 * nu));
            D11 = c * (1.0 - nu);
            D12 = c * nu;
            D33 = c * (1.0 - 2.0 * nu) / 2.0;
        }
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                const double xx = I(a, b, 0, 0), yy = I(a, b, 1, 1);
                const double xy = I(a, b, 0, 1), yx = I(a, b, 1, 0);
                K[(2 * a) * ne + 2 * b] = D11 * xx + D33 * yy;
                K[(2 * a + 1) * ne + 2 * b + 1] = D11 * yy + D33 * xx;
                K[(2 * a) * ne + 2 * b + 1] = D12 * xy + D33 * yx;
                K[(2 * a + 1) * ne + 2 * b] = D12 * yx + D33 * xy;
            }
    } else {
        const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        const double mu = E / (2.0 * (1.0 + nu));
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b)
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) {
                        double v;
                        if (p == q) {
                            v = (lam + 2.0 * mu) * I(a, b, p, p);
                            for (int r = 0; r < 3; ++r)
                                if (r != p) v += mu * I(a, b, r, r);
                        } else {
                            v = lam * I(a, b, p, q) + mu * I(a, b, q, p);
                        }
                        K[(3 * a + p) * ne + 3 * b + q] = v;
                    }
    }
}

bool element_factor(const topo_mesh& m, const std::vector<double>& K, std::vector<double>& F,
                    std::vector<double>* Mt) {
    const int dim = m.dim, nen = 1 << dim, ne = dim * nen;
    auto H = [](int mm, int a) { return (__builtin_popcount(mm & a) & 1) ? -1.0 : 1.0; };
    // Kt[(mm,c),(mp,d)] = nen^-2 sum_ab H[mm][a] K[(a,c),(b,d)] H[mp][b]
    auto Kt = [&](int mm, int c, int mp, int d) {
        double s = 0.0;
        for (int a = 0; a < nen; ++a)
            for (int b = 0; b < nen; ++b) s += H(mm, a) * K[(size_t)(dim * a + c) * ne + dim * b + d] * H(mp, b);
        return s / (double)(nen * nen);
    };
    F.assign(kFacSize, 0.0);
    for (int c = 0; c < dim; ++c) F[kFacH + c] = m.h[c];
    if (Mt) {
        Mt->assign(kFacSize, 0.0);
        for (int c = 0; c < dim; ++c) (*Mt)[kFacH + c] = m.h[c];
    }
    // R rows, for the reconstruction check
    std::vector<std::vector<double>> R;
    for (int n = 0; n < nen; ++n) {
        // block entries (n ^ e_c, c); reduction rows G (r x dim) over them
        double B[3][3];
        for (int c = 0; c < dim; ++c)
            for (int d = 0; d < dim; ++d) B[c][d] = Kt(n ^ (1 << c), c, n ^ (1 << d), d);
        double G[3][3] = {};
        int r = 0;
        const int pc = __builtin_popcount(n);
        if (pc == 1) {  // a rigid translation: drop its component
            for (int c = 0; c < dim; ++c)
                if (n != (1 << c)) G[r++][c] = 1.0;
        } else if (pc == 2) {  // a rigid rotation in the plane of the two set axes
            int cd[2], q = 0;
            for (int c = 0; c < dim; ++c)
                if ((n >> c) & 1) cd[q++] = c;
            G[r][cd[0]] = m.h[cd[0]];
            G[r][cd[1]] = m.h[cd[1]];
            ++r;
            for (int c = 0; c < dim; ++c)
                if (!((n >> c) & 1)) G[r++][c] = 1.0;
        } else {
            for (int c = 0; c < dim; ++c) G[r++][c] = 1.0;
        }
        // M = (G G^T)^-1 G B G^T (G G^T)^-1 (rows of G are orthogonal)
        double gg[3], Mb[3][3];
        for (int i = 0; i < r; ++i) {
            gg[i] = 0.0;
            for (int c = 0; c < dim; ++c) gg[i] += G[i][c] * G[i][c];
        }
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < r; ++j) {
                double s = 0.0;
                for (int c = 0; c < dim; ++c)
                    for (int d = 0; d < dim; ++d) s += G[i][c] * B[c][d] * G[j][d];
                Mb[i][j] = s / (gg[i] * gg[j]);
            }
        // Cholesky M = L L^T
        double L[3][3] = {};
        for (int i = 0; i < r; ++i)
            for (int j = 0; j <= i; ++j) {
                double s = Mb[i][j];
                for (int q = 0; q < j; ++q) s -= L[i][q] * L[j][q];
                if (i == j) {
                    if (!(s > 0.0)) return false;
                    L[i][i] = std::sqrt(s);
                } else {
                    L[i][j] = s / L[j][j];
                }
            }
        const int slot[3][3] = {{0, 1, 2}, {-1, 3, 4}, {-1, -1, 5}};
        for (int i = 0; i < r; ++i)
            for (int j = i; j < r; ++j) {
                F[6 * n + slot[i][j]] = L[j][i];  // (L^T)[i][j]
                if (Mt) (*Mt)[6 * n + slot[i][j]] = Mb[i][j];
            }
        // rows of R: (L^T G)[i][c] times H[n ^ e_c][a] on DOF (a, c)
        for (int i = 0; i < r; ++i) {
            std::vector<double> row(ne, 0.0);
            for (int c = 0; c < dim; ++c) {
                double w = 0.0;
                for (int j = i; j < r; ++j) w += L[j][i] * G[j][c];
                for (int a = 0; a < nen; ++a) row[dim * a + c] += w * H(n ^ (1 << c), a);
            }
            R.push_back(row);
        }
    }
    // K must equal R^T R, and every block must be closed under the reflections
    double kmax = 0.0, err = 0.0;
    for (int i = 0; i < ne * ne; ++i) kmax = std::max(kmax, std::fabs(K[i]));
    for (int i = 0; i < ne; ++i)
        for (int j = 0; j < ne; ++j) {
            double s = 0.0;
            for (auto& row : R) s += row[i] * row[j];
            err = std::max(err, std::fabs(s - K[(size_t)i * ne + j]));
        }
    return err <= 1e-12 * kmax && (int)R.size() == (dim == 2 ? 5 : 18);
}

int set_error(Ctx* c, int code, const char* fmt, ...) {
    if (c) {
        char buf[1024];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

int Arena::commit(Ctx* ctx, hipStream_t s) {
    const size_t total = this->total();
    if (total > ctx->ws_bytes) {
        if (ctx->ws) {
            // the old arena is last used by this context's work on s (calls of one
            // context on other streams are ordered by the caller), so draining s is
            // enough; other contexts on the device keep running
            TOPO_HIP(hipStreamSynchronize(s));
            TOPO_HIP(hipFree(ctx->ws));
            ctx->ws = nullptr;
            ctx->ws_bytes = 0;
        }
        size_t want = grown(total);
        if (ctx->budget > 0 && want > ctx->budget) {
            if (total > ctx->budget)
                return set_error(ctx, TOPO_ENOMEM, "workspace of %zu bytes exceeds the context budget of %zu bytes",
                                 total, ctx->budget);
            want = ctx->budget;  // no growth margin beyond the budget
        }
        if (hipMalloc(&ctx->ws, want) != hipSuccess) {
            (void)hipGetLastError();
            ctx->ws = nullptr;
            return set_error(ctx, TOPO_ENOMEM, "workspace allocation of %zu bytes failed", want);
        }
        ctx->ws_bytes = want;
    }
    char* p = (char*)ctx->ws;
    for (auto& r : reqs) {
        *r.out = p;
        p += (r.bytes + 255) & ~size_t(255);
    }
    reqs.clear();
    return TOPO_OK;
}

hipError_t ensure_dynamic_lds(const void* kernel, size_t bytes) {
    static std::mutex mu;
    static std::map<const void*, size_t> set;
    std::lock_guard<std::mutex> lk(mu);
    size_t& have = set[kernel];
    if (bytes <= have) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) have = bytes;
    return e;
}

int pinned_host(Ctx* ctx, size_t bytes, void** out) {
    if (bytes > ctx->pinned_bytes) {
        if (ctx->pinned) TOPO_HIP(hipHostFree(ctx->pinned));
        ctx->pinned = nullptr;
        TOPO_HIP(hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault));
        ctx->pinned_bytes = bytes;
    }
    *out = ctx->pinned;
    return TOPO_OK;
}

const ElemTables* get_tables(Ctx* ctx, const topo_mesh& m) {
    const int dim = m.dim;
    auto key = std::make_tuple(dim, m.h[0], m.h[1], dim == 3 ? m.h[2] : 0.0, m.nu,
                               dim == 2 ? m.plane : 0);
    auto it = ctx->tables.find(key);
    if (it != ctx->tables.end()) return &it->second;
    ElemTables t;
    element_stiffness(m, t.host);
    t.ne = dim * (1 << dim);
    const size_t n = (size_t)t.ne * t.ne;
    std::vector<float> k32(n);
    for (size_t i = 0; i < n; ++i) k32[i] = (float)t.host[i];
    for (int c = 0; c < 3; ++c) t.diag[c] = c < dim ? t.host[(size_t)c * t.ne + c] : 0.0;
    if (hipMalloc(&t.K64, n * sizeof(double)) != hipSuccess) return nullptr;
    if (hipMalloc(&t.K32, n * sizeof(float)) != hipSuccess) return nullptr;
    if (hipMemcpy(t.K64, t.host.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return nullptr;
    if (hipMemcpy(t.K32, k32.data(), n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return nullptr;
    std::vector<double> fac, mblk;
    if (!element_factor(m, t.host, fac, &mblk)) return nullptr;
    std::vector<float> fac32(fac.begin(), fac.end()), mblk32(mblk.begin(), mblk.end());
    if (hipMalloc(&t.F64, kFacSize * sizeof(double)) != hipSuccess) return nullptr;
    if (hipMalloc(&t.F32, kFacSize * sizeof(float)) != hipSuccess) return nullptr;
    if (hipMalloc(&t.M64, kFacSize * sizeof(double)) != hipSuccess) return nullptr;
    if (hipMalloc(&t.M32, kFacSize * sizeof(float)) != hipSuccess) return nullptr;
    if (hipMemcpy(t.F64, fac.data(), kFacSize * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t.F32, fac32.data(), kFacSize * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t.M64, mblk.data(), kFacSize * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t.M32, mblk32.data(), kFacSize * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return nullptr;
    for (int i = 0; i < kFacSize; ++i) {
        t.Mv64.m[i] = mblk[i];
        t.Mv32.m[i] = mblk32[i];
    }
    return &(ctx->tables[key] = t);
}

const char* const kKernelNames[KID_COUNT] = {
    "apply", "pcg_apply", "pcg_update", "residual", "rom_contract", "rom_reduce",
    "phit_v", "phi_y", "chol", "chol_solve", "gradient", "pcg_step", "rom_apply"};

static hipEvent_t timing_event(Ctx* c) {
    if (!c->timing.pool.empty()) {
        hipEvent_t e = c->timing.pool.back();
        c->timing.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

TimedLaunch::TimedLaunch(Ctx* ctx, int k, hipStream_t st, int mode, bool ik)
    : c(ctx), kid(k), s(st), in_kernel(ik) {
    if (!c || mode == kTimeOff) return;
    Timing& t = c->timing;
    if (t.every <= 0) return;
    if (!in_kernel) ++t.launched[kid];  // the PCG kernels are counted by their phase driver
    if ((t.seen[kid]++ / kTimeRun) % t.every != 0 && mode != kTimeForced) return;
    a = timing_event(c);
    if (!a) return;
    if (in_kernel) {
        b = timing_event(c);
        if (!b) {
            t.pool.push_back(a);
            a = nullptr;
        }
        return;
    }
    if (hipEventRecord(a, s) != hipSuccess) {
        t.pool.push_back(a);
        a = nullptr;
    }
}

TimedLaunch::~TimedLaunch() {
    if (!a) return;
    if (!in_kernel) {
        b = timing_event(c);
        if (!b || hipEventRecord(b, s) != hipSuccess) {
            c->timing.pool.push_back(a);
            if (b) c->timing.pool.push_back(b);
            return;
        }
    }
    c->timing.pending.push_back({a, b, kid});
    if (c->timing.pending.size() > 8192) timing_drain(c);
}

void timing_drain(Ctx* c) {
    Timing& t = c->timing;
    for (auto& r : t.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            t.samples[r.kid] += 1;
            t.total_ms[r.kid] += ms;
        }
        t.pool.push_back(r.a);
        t.pool.push_back(r.b);
    }
    t.pending.clear();
}

int validate_mesh(Ctx* ctx, const topo_mesh* m) {
    if (!m) return set_error(ctx, TOPO_EINVAL, "mesh is NULL");
    if (m->dim != 2 && m->dim != 3) return set_error(ctx, TOPO_EINVAL, "dim must be 2 or 3");
    for (int d = 0; d < m->dim; ++d) {
        if (m->nel[d] < 1) return set_error(ctx, TOPO_EINVAL, "nel[%d] < 1", d);
        if (!(m->h[d] > 0.0) || !std::isfinite(m->h[d]))
            return set_error(ctx, TOPO_EINVAL, "h[%d] must be positive", d);
    }
    double nodes = 1.0;
    for (int d = 0; d < m->dim; ++d) nodes *= (m->nel[d] + 1.0);
    if (nodes * m->dim > 2.0e9) return set_error(ctx, TOPO_EINVAL, "mesh too large");
    if (!(m->nu > -1.0 && m->nu < 0.5)) return set_error(ctx, TOPO_EINVAL, "nu must lie in (-1, 0.5)");
    if (!(m->Emin >= 0.0) || !(m->E0 > m->Emin) || !std::isfinite(m->E0))
        return set_error(ctx, TOPO_EINVAL, "need 0 <= Emin < E0");
    if (!(m->penal >= 1.0) || !std::isfinite(m->penal))
        return set_error(ctx, TOPO_EINVAL, "penal must be >= 1");
    if (m->dim == 2 && m->plane != 0 && m->plane != 1)
        return set_error(ctx, TOPO_EINVAL, "plane must be 0 (stress) or 1 (strain)");
    return TOPO_OK;
}

}  // namespace topo

using namespace topo;

extern "C" {

int topo_ctx_create(topo_ctx** out, int32_t device, size_t hbm_budget_bytes) {
    if (!out) return TOPO_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
        (void)hipGetLastError();
        return TOPO_EDEVICE;
    }
    if (device < 0 || device >= n) return TOPO_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return TOPO_EDEVICE;
    topo_ctx* c = new topo_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->cu_count = prop.multiProcessorCount;
    *out = c;
    return TOPO_OK;
}

int topo_ctx_destroy(topo_ctx* c) {
    if (!c) return TOPO_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    timing_drain(c);
    for (hipEvent_t e : c->timing.pool) (void)hipEventDestroy(e);
    for (auto& kv : c->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    for (auto& kv : c->tables) {
        (void)hipFree(kv.second.K64);
        (void)hipFree(kv.second.K32);
        (void)hipFree(kv.second.F64);
        (void)hipFree(kv.second.F32);
        (void)hipFree(kv.second.M64);
        (void)hipFree(kv.second.M32);
    }
    if (c->ws) (void)hipFree(c->ws);
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
    return TOPO_OK;
}

const char* topo_last_error(const topo_ctx* c) { return c ? c->err.c_str() : "no context"; }

size_t topo_ctx_workspace_bytes(const topo_ctx* c) { return c ? c->ws_bytes : 0; }

const char* topo_strerror(int32_t code) {
    switch (code) {
        case TOPO_OK: return "TOPO_OK";
        case TOPO_EINVAL: return "TOPO_EINVAL";
        case TOPO_ENOMEM: return "TOPO_ENOMEM";
        case TOPO_ENOCONV: return "TOPO_ENOCONV";
        case TOPO_ENOTSPD: return "TOPO_ENOTSPD";
        case TOPO_EDEVICE: return "TOPO_EDEVICE";
        case TOPO_EAGAIN: return "TOPO_EAGAIN";
        default: return "TOPO_UNKNOWN";
    }
}

int topo_ctx_set_timing(topo_ctx* c, int32_t every) {
    if (!c || every < 0) return TOPO_EINVAL;
    c->timing.every = every;
    return TOPO_OK;
}

int topo_ctx_kernel_time(topo_ctx* c, const char* kernel, int64_t* samples, double* total_ms,
                         int64_t* launches, int32_t reset) {
    if (!c || !kernel) return TOPO_EINVAL;
    int kid = -1;
    for (int i = 0; i < KID_COUNT; ++i)
        if (std::strcmp(kernel, kKernelNames[i]) == 0) kid = i;
    if (kid < 0) return set_error(c, TOPO_EINVAL, "unknown kernel name '%s'", kernel);
    (void)hipSetDevice(c->device);
    timing_drain(c);
    if (samples) *samples = c->timing.samples[kid];
    if (total_ms) *total_ms = c->timing.total_ms[kid];
    if (launches) *launches = c->timing.launched[kid];
    if (reset) {
        c->timing.launched[kid] = 0;
        c->timing.samples[kid] = 0;
        c->timing.total_ms[kid] = 0.0;
        c->timing.seen[kid] = 0;
    }
    return TOPO_OK;
}

int topo_element_stiffness(const topo_mesh* mesh, double* K0) {
    if (!K0) return TOPO_EINVAL;
    int rc = validate_mesh(nullptr, mesh);
    if (rc) return rc;
    std::vector<double> K;
    element_stiffness(*mesh, K);
    std::memcpy(K0, K.data(), K.size() * sizeof(double));
    return TOPO_OK;
}

int topo_element_factor(const topo_mesh* mesh, double* F) {
    if (!F) return TOPO_EINVAL;
    int rc = validate_mesh(nullptr, mesh);
    if (rc) return rc;
    std::vector<double> K, fac;
    element_stiffness(*mesh, K);
    if (!element_factor(*mesh, K, fac)) return TOPO_EINVAL;
    std::memcpy(F, fac.data(), fac.size() * sizeof(double));
    return TOPO_OK;
}

}  // extern "C"
