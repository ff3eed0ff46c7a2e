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

// Division by a divisor fixed at launch: floor(n / d) = (n m) >> s for 0 <= n < 2^31 and
// 1 <= d < 2^31, with s = 31 + ceil(log2 d) and m = ceil(2^s / d) (the round-up method of
// Granlund and Montgomery): m d - 2^s < d bounds the error n (m d - 2^s) / (d 2^s) below
// 1/d, the distance from n / d up to the next integer, and m < 2^32.
struct FastDiv {
    unsigned d = 1, m = 1u << 31;
    int s = 31;
    __host__ __device__ unsigned div(unsigned n) const {
        return (unsigned)(((unsigned long long)n * m) >> s);
    }
};

inline FastDiv make_fastdiv(unsigned d) {
    FastDiv f;
    int l = 0;
    while ((1ull << l) < d) ++l;
    f.d = d;
    f.s = 31 + l;
    f.m = (unsigned)(((1ull << f.s) + d - 1) / d);
    return f;
}

// Element access at index i of an array whose base is uniform: with a 32-bit index the
// byte offset is formed in 32 bits, so that a load or store takes the base in scalar
// registers and one 32-bit offset (no 64-bit address per access); with a 64-bit index
// (arrays of 4 GiB or more, and the float64 apply) it is a plain subscript.
template <typename T>
__device__ __forceinline__ T ld_at(const T* __restrict__ b, unsigned i) {
    return *(const T*)((const char*)b + i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T ld_at(const T* __restrict__ b, size_t i) {
    return b[i];
}
template <typename T>
__device__ __forceinline__ void st_at(T* __restrict__ b, unsigned i, T v) {
    *(T*)((char*)b + i * (unsigned)sizeof(T)) = v;
}
template <typename T>
__device__ __forceinline__ void st_at(T* __restrict__ b, size_t i, T v) {
    b[i] = v;
}

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
    int mtarget = 0;    // 3D march: resident blocks of the kernel per field (0: 1024)
    FastDiv dnx1, dny1; // division by nx1, ny1 (node coordinates from a node index)
};

Grid make_grid(const topo_mesh& m);

// Symmetry-blocked factor K_e = R^T R of the box element (R has 5 rows for Q4, 18 for
// H8).  The reflections of the box commute with K_e, so in the Walsh-Hadamard basis of
// the nodal values (per displacement component) K_e splits into one small block per
// reflection character.  The rigid translations and rotations occupy fixed directions
// of these blocks and are dropped exactly; each remaining block is SPD and stored as
// its upper-triangular Cholesky factor.  Table layout: 8 blocks x 6 slots
// (L00 L01 L02 L11 L12 L22 of the block's transposed factor), then h[0..2].
constexpr int kFacSize = 51;
constexpr int kFacH = 48;

// The reduced blocks as a by-value kernel argument: uniform values that the kernel reads
// from its argument segment into scalar registers instead of holding them in vector
// registers or LDS.
template <typename T>
struct FacTab {
    T m[kFacSize];
};

// Element tables of one (dim, h, nu, plane) combination, resident on the device.
struct ElemTables {
    int ne;            // element DOFs: 8 (Q4) or 24 (H8)
    double* K64;       // device [ne*ne]
    float* K32;        // device [ne*ne]
    double* F64 = nullptr;  // device [kFacSize] symmetry-blocked factor
    float* F32 = nullptr;   // device [kFacSize]
    double* M64 = nullptr;  // device [kFacSize] the reduced blocks M = L L^T themselves
    float* M32 = nullptr;   // device [kFacSize]
    FacTab<double> Mv64{};  // host copies of M64 / M32 (kernel arguments)
    FacTab<float> Mv32{};
    double diag[3];    // K_e diagonal per displacement component (host copy)
    std::vector<double> host;  // host copy of K64
};

// Exact element stiffness of the rectangular Q4 / H8 element (host).
void element_stiffness(const topo_mesh& m, std::vector<double>& K);

// The symmetry-blocked factor of K (kFacSize values) and, when Mt is given, the reduced
// blocks M = L L^T in the same slots (upper triangles; element sizes at kFacH); false if
// K does not have the block structure of a box element or a block is not positive
// definite.
bool element_factor(const topo_mesh& m, const std::vector<double>& K, std::vector<double>& F,
                    std::vector<double>* Mt = nullptr);

// ----------------------------------------------------------------------------------
// Sampled kernel timing (instrumentation): one launch in `every` of each hot kernel is
// bracketed by a pair of HIP events on its own stream.
// ----------------------------------------------------------------------------------
enum KernelId {
    KID_APPLY, KID_PCG_APPLY, KID_PCG_UPDATE, KID_RESIDUAL, KID_ROM_CONTRACT, KID_ROM_REDUCE,
    KID_PHIT_V, KID_PHI_Y, KID_CHOL, KID_CHOL_SOLVE, KID_GRADIENT, KID_PCG_STEP, KID_ROM_APPLY, KID_COUNT
};
extern const char* const kKernelNames[KID_COUNT];

struct Timing {
    int every = 0;
    long long seen[KID_COUNT] = {};
    long long launched[KID_COUNT] = {};  // launches issued (graph replays included)
    long long samples[KID_COUNT] = {};
    double total_ms[KID_COUNT] = {};
    struct Rec { hipEvent_t a, b; int kid; };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
};

struct Ctx;
void timing_drain(Ctx* c);

// mode: kTimeOff never records (e.g. while building a graph), kTimeSampled records one
// run of kTimeRun consecutive launches in `every` runs, kTimeForced records whenever
// timing is enabled.  Runs of 8: the 3D PCG update alternates seven cheaper launches
// with one that also updates the correction (a group of 8 steps), so a sample of whole
// runs averages the two kinds in their proportion.  With in_kernel,
// a sampled launch gets the event pair (a, b) to pass to hipExtLaunchKernel, which
// stamps them when the kernel itself starts and ends (no marker packets around it);
// otherwise a and b are recorded on the stream before and after the launch.
enum { kTimeOff = 0, kTimeSampled = 1, kTimeForced = 2 };
constexpr int kTimeRun = 8;
struct TimedLaunch {
    Ctx* c;
    int kid;
    hipStream_t s;
    bool in_kernel;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(Ctx* ctx, int kid, hipStream_t s, int mode = kTimeSampled, bool in_kernel = false);
    ~TimedLaunch();
};

// ----------------------------------------------------------------------------------
// Context: device, element-table cache, grow-only workspace arena
// ----------------------------------------------------------------------------------
// Instantiated HIP graphs of launch-bound kernel sequences, keyed by every value baked
// into their kernel arguments.
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct Ctx {
    int device = 0;
    Timing timing;
    std::map<std::vector<uintptr_t>, GraphEntry> graphs;
    std::string err;
    std::map<std::tuple<int, double, double, double, double, int>, ElemTables> tables;
    void* ws = nullptr;        // device workspace
    size_t ws_bytes = 0;
    size_t budget = 0;         // most workspace bytes the context may hold (0: no limit)
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
    // bytes the pending requests need, and what the arena allocates when it must grow
    size_t total() const {
        size_t t = 0;
        for (const auto& r : reqs) t += (r.bytes + 255) & ~size_t(255);
        return t;
    }
    static size_t grown(size_t total) { return total + total / 4 + (size_t(1) << 20); }
};

// Device workspace (bytes, before the arena's growth margin) of each entry point.
size_t ws_hdm_solve(const Grid& g, bool mixed, int B);
size_t ws_rom_build(const Grid& g, int k, int B, bool f64, int cu);
size_t ws_rom_solve(int k, int B);
size_t ws_rom_estimate(const Grid& g, int k, int B, int max_refine);

int pinned_host(Ctx* c, size_t bytes, void** out);

// Raise a kernel's dynamic LDS limit to at least `bytes` (hipFuncSetAttribute), once per
// kernel and size for the whole process: the attribute is process-wide state of the
// kernel, so worker threads launching the same kernel never rewrite it concurrently.
hipError_t ensure_dynamic_lds(const void* kernel, size_t bytes);
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

// Sum each of NV arrays of n doubles in one pass (fixed order; result in every thread).
template <int NV>
__device__ inline void block_sum_arrays(const double* const (&a)[NV], int n, double (&out)[NV],
                                        double* lds /* >= NV*16 */) {
#pragma unroll
    for (int q = 0; q < NV; ++q) out[q] = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x)
#pragma unroll
        for (int q = 0; q < NV; ++q) out[q] += a[q][i];
    block_reduce<NV>(out, lds);
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

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD b % 8),
// and each XCD has its own L2.  Stencil kernels therefore map block b to the logical
// tile / node range xcd_block(b, nb), which gives every XCD one contiguous eighth of
// the grid, so that the halo rows a block re-reads are mostly in its own L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b % kXcds, q = nb / kXcds, r = nb % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// Field and block of a batched stencil launch (grid nb x B, one field per blockIdx.y):
// the linear workgroup id is mapped XCD-aware over the whole batch, so that every XCD
// takes one contiguous range of (field, block) pairs and the halo a block re-reads
// stays in its own L2.  With B = 1 this is xcd_block(blockIdx.x, nb).
struct FieldBlock {
    int field, blk;
};
__device__ __forceinline__ FieldBlock field_block() {
    const int gx = gridDim.x;
    const int l = xcd_block(blockIdx.x + gx * blockIdx.y, gx * gridDim.y);
    const int f = l / gx;
    return {f, l - f * gx};
}

// 3D element-centric march: a block owns 31 x 7 node columns (a 32 x 8 tile of element
// columns) over KZ node planes, with KZ chosen so that a field's blocks fit in one
// resident wave of the kernel (mtarget blocks, from its occupancy): a partial second
// wave of long marches left most of the chip idle (96x48x48 float64: 49 -> 42 ms).
constexpr int MEX = 32, MEY = 8;             // element tile (one thread each)
constexpr int MOX = MEX - 1, MOY = MEY - 1;  // owned node columns
__host__ __device__ inline int march3_tiles_x(const Grid& g) { return (g.nx1 + MOX - 1) / MOX; }
__host__ __device__ inline int march3_tiles_y(const Grid& g) { return (g.ny1 + MOY - 1) / MOY; }
__host__ __device__ inline int march3_kz(const Grid& g) {
    const int xy = march3_tiles_x(g) * march3_tiles_y(g);
    const int target = g.mtarget > 0 ? g.mtarget : 1024;
    const int chunks = target > xy ? target / xy : 1;
    const int kz = (g.nz1 + chunks - 1) / chunks;
    return kz < 2 ? 2 : kz;
}
__host__ __device__ inline int march3_blocks(const Grid& g) {
    const int kz = march3_kz(g);
    return march3_tiles_x(g) * march3_tiles_y(g) * ((g.nz1 + kz - 1) / kz);
}

// Element-once 3D march (the PCG apply): a block owns a 32 x 8 tile of element columns
// (no overlap with its neighbours) over KZ element layers, so every element is
// evaluated exactly once.  A node shared by several blocks (on the high x / y / z face
// of one block and inside or on the low face of another) is completed later: the
// block whose tile holds the element at the node's own (i, j, k) corner, its primary
// block, writes its part to the main array, every other block writes its part to one
// of seven side sections (by which of its high faces the node lies on), and the
// consumer adds the sections in a fixed order.  KZ is sized like march3_kz.
__host__ __device__ inline int once3_tiles_x(const Grid& g) { return (g.nx + MEX - 1) / MEX; }
__host__ __device__ inline int once3_tiles_y(const Grid& g) { return (g.ny + MEY - 1) / MEY; }
__host__ __device__ inline int once3_kz(const Grid& g) {
    const int xy = once3_tiles_x(g) * once3_tiles_y(g);
    const int target = g.mtarget > 0 ? g.mtarget : 1024;
    const int chunks = target > xy ? target / xy : 1;
    return (g.nz + chunks - 1) / chunks;
}
__host__ __device__ inline int once3_chunks(const Grid& g) {
    const int kz = once3_kz(g);
    return (g.nz + kz - 1) / kz;
}
__host__ __device__ inline int once3_blocks(const Grid& g) {
    return once3_tiles_x(g) * once3_tiles_y(g) * once3_chunks(g);
}

// Side sections s = 1..7 (bit 1: the contributing block is below the node in x, bit 2:
// in y, bit 4: in z).  Along an axis in s the section holds only the interior block
// boundaries (index = boundary number - 1), along the others every node; the sections
// follow each other in the order of s, one component after the other ([c][total]).
struct SideGeom {
    int nbx, nby, nbz;  // interior block boundaries along x, y, z
    int nnx, nny, nnz;  // nodes along x, y, z
    int kz;             // element layers per chunk
    long long total;    // nodes over all sections
    FastDiv dnx, dny, dkz;  // division by nnx, nny, kz
    // extent of section s along x / y / z
    __host__ __device__ int ex(int s) const { return s & 1 ? nbx : nnx; }
    __host__ __device__ int ey(int s) const { return s & 2 ? nby : nny; }
    __host__ __device__ int ez(int s) const { return s & 4 ? nbz : nnz; }
};

__host__ __device__ inline long long side_count(const SideGeom& sg, int s) {
    return (long long)sg.ex(s) * sg.ey(s) * sg.ez(s);
}

inline SideGeom side_geom(const Grid& g) {
    SideGeom sg;
    sg.kz = once3_kz(g);
    sg.nbx = once3_tiles_x(g) - 1;
    sg.nby = once3_tiles_y(g) - 1;
    sg.nbz = once3_chunks(g) - 1;
    sg.nnx = g.nx1;
    sg.nny = g.ny1;
    sg.nnz = g.nz1;
    sg.total = 0;
    for (int t = 1; t < 8; ++t) sg.total += side_count(sg, t);
    sg.dnx = make_fastdiv((unsigned)sg.nnx);
    sg.dny = make_fastdiv((unsigned)sg.nny);
    sg.dkz = make_fastdiv((unsigned)sg.kz);
    return sg;
}

// Index in section s of node (i, j, k) (s's axes on a block boundary of the node).
__host__ __device__ inline long long side_index(const SideGeom& sg, int s, int i, int j, int k) {
    long long off = 0;
#pragma unroll
    for (int t = 1; t < 7; ++t) off += t < s ? side_count(sg, t) : 0;
    const int a = s & 1 ? i / MEX - 1 : i;
    const int b = s & 2 ? j / MEY - 1 : j;
    const int c = s & 4 ? (int)sg.dkz.div((unsigned)k) - 1 : k;
    return off + ((long long)c * sg.ey(s) + b) * sg.ex(s) + a;
}

// Axes along which node (i, j, k) lies on an interior block boundary (bit per axis).
__host__ __device__ inline int side_axes(const Grid& g, const SideGeom& sg, int i, int j, int k) {
    return (i % MEX == 0 && i > 0 && i < g.nx ? 1 : 0) | (j % MEY == 0 && j > 0 && j < g.ny ? 2 : 0) |
           (k - (int)sg.dkz.div((unsigned)k) * sg.kz == 0 && k > 0 && k < g.nz ? 4 : 0);
}

// Element sensitivities dc_e = -alpha'(rho_e) u_e^T K_e u_e of B fields (rho [B][N_e],
// u [B][N_u], dc [B][N_e], all float64 device arrays).
int gradient_launch(Ctx* ctx, const Grid& g, const topo_mesh& m, const ElemTables* tb,
                    const double* rho, const double* u, int B, double* dc, hipStream_t s);

// Resident blocks of a 256-thread kernel on the whole device (its occupancy times the
// CU count); 1024 when the runtime cannot tell.
int march3_target(const Ctx* ctx, const void* kernel);
struct ElemTables;
template <typename TX>
int apply_columns(Ctx* ctx, const Grid& g, const ElemTables* tb, const double* alpha, const uint8_t* mask,
                  const TX* x, double* y, int ncols, long long ld, hipStream_t s);

// Blocks of a node-stencil launch (apply, PCG apply, residual): one per march column
// in 3D, one per kBlock consecutive nodes in 2D.
inline int stencil_blocks(const Grid& g) {
    return g.dim == 2 ? grid_blocks(g.n_nodes) : march3_blocks(g);
}

// Largest block count of a PCG launch whose per-block partials every block of the next
// kernel sums by itself; larger launches get one summing kernel in between, so that the
// redundant sums never cost more than a few hundred kilobytes of cache reads per block.
constexpr int kPcgMaxBlocks = 2048;

// Stride of the per-block partial arrays shared by the stencil and the node-linear
// PCG kernels.
inline int partial_stride(const Grid& g) {
    const int a = stencil_blocks(g), b = grid_blocks(g.n_nodes);
    const int c = g.dim == 3 ? once3_blocks(g) : 0;
    const int ab = a > b ? a : b;
    return ab > c ? ab : c;
}

// Sum each of NV arrays (array q has n[q] doubles) in one pass, fixed order.
template <int NV>
__device__ inline void block_sum_arrays_n(const double* const (&a)[NV], const int (&n)[NV],
                                          double (&out)[NV], double* lds /* >= NV*16 */) {
    int nmax = 0;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        out[q] = 0.0;
        nmax = n[q] > nmax ? n[q] : nmax;
    }
    for (int i = threadIdx.x; i < nmax; i += blockDim.x)
#pragma unroll
        for (int q = 0; q < NV; ++q)
            if (i < n[q]) out[q] += a[q][i];
    block_reduce<NV>(out, lds);
}

}  // namespace topo

// The opaque handle of the C ABI is the context itself.
struct topo_ctx : topo::Ctx {};
