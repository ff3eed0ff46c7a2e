// Internal declarations shared by the translation units of libtopo_rom.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "topo_rom.h"

namespace topo {

// ----------------------------------------------------------------------------------
// Structured grid as seen by the kernels
// ----------------------------------------------------------------------------------
struct Grid {
    int dim;
    int nx, ny, nz;     // elements per axis (nz = 1 in 2D)
    int nx1, ny1, nz1;  // nodes per axis (nz1 = 1 in 2D)
    int n_nodes;
    int n_elems;
    long long n_dofs;
};

Grid make_grid(const topo_mesh& m);

// Element tables of one (dim, h, nu, plane) combination, resident on the device.
struct ElemTables {
    int ne;            // element DOFs: 8 (Q4) or 24 (H8)
    double* K64;       // device [ne*ne]
    float* K32;        // device [ne*ne]
    double diag[3];    // K_e diagonal per displacement component (host copy)
    std::vector<double> host;  // host copy of K64
};

// Exact element stiffness of the rectangular Q4 / H8 element (host).
void element_stiffness(const topo_mesh& m, std::vector<double>& K);

// ----------------------------------------------------------------------------------
// Context: device, element-table cache, grow-only workspace arena
// ----------------------------------------------------------------------------------
struct Ctx {
    int device = 0;
    std::string err;
    std::map<std::tuple<int, double, double, double, double, int>, ElemTables> tables;
    void* ws = nullptr;        // device workspace
    size_t ws_bytes = 0;
    void* pinned = nullptr;    // small pinned host buffer for scalar read-backs
    size_t pinned_bytes = 0;
    int cu_count = 256;
};

int set_error(Ctx* c, int code, const char* fmt, ...);

// Workspace bump allocator over ctx->ws.  Acquire all pieces first, then call
// commit(), which grows the arena if needed (synchronising the stream when the old
// arena is released).
struct Arena {
    struct Req { void** out; size_t bytes; };
    std::vector<Req> reqs;
    template <typename T>
    void take(T** out, size_t count) { reqs.push_back({(void**)out, count * sizeof(T)}); }
    int commit(Ctx* c, hipStream_t s);
};

int pinned_host(Ctx* c, size_t bytes, void** out);
const ElemTables* get_tables(Ctx* c, const topo_mesh& m);

#define TOPO_HIP(call)                                                             \
    do {                                                                           \
        hipError_t _e = (call);                                                    \
        if (_e != hipSuccess)                                                      \
            return ::topo::set_error(ctx, TOPO_EDEVICE, "%s:%d %s: %s", __FILE__,  \
                                     __LINE__, #call, hipGetErrorString(_e));      \
    } while (0)

#define TOPO_CHECK_LAUNCH() TOPO_HIP(hipGetLastError())

int validate_mesh(Ctx* c, const topo_mesh* m);

// ----------------------------------------------------------------------------------
// Device helpers
// ----------------------------------------------------------------------------------
constexpr int kBlock = 256;

__host__ __device__ inline double simp_alpha(double rho, double E0, double Emin, double p) {
    // alpha = Emin + (E0 - Emin) rho^p, with the common integer exponent done by
    // multiplication so FP64 and FP32 tables agree with the definition to rounding.
    double rp;
    if (p == 3.0) rp = rho * rho * rho;
    else if (p == 1.0) rp = rho;
    else if (p == 2.0) rp = rho * rho;
    else rp = pow(rho, p);
    return Emin + (E0 - Emin) * rp;
}

// Deterministic block reduction of NV doubles (all threads get the results).
template <int NV>
__device__ inline void block_reduce(double (&v)[NV], double* lds /* >= NV*16 */) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) lds[i * 16 + wave] = x;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[i * 16 + w];
        v[i] = s;
    }
    __syncthreads();
}

// "Last block done" ticket: returns true in every thread of the block that arrives
// last.  Partial results must have been written before the call.  The last block
// resets the counter for the next use.
__device__ inline bool last_block(unsigned* counter) {
    __shared__ bool is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = atomicAdd(counter, 1u);
        is_last = (t == gridDim.x * gridDim.y * gridDim.z - 1);
    }
    __syncthreads();
    if (is_last) {
        __threadfence();
        if (threadIdx.x == 0) atomicExch(counter, 0u);
    }
    return is_last;
}

// Sum n doubles with a fixed order inside one block (result in every thread).
__device__ inline double block_sum_array(const double* a, int n, double* lds) {
    double s[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) s[0] += a[i];
    block_reduce<1>(s, lds);
    return s[0];
}

inline int grid_blocks(long long n, int block = kBlock) {
    return (int)((n + block - 1) / block);
}

}  // namespace topo

// The opaque handle of the C ABI is the context itself.
struct topo_ctx : topo::Ctx {};
