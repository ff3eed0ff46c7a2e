// Deterministic sums of per-chunk partials, shared by the reduced-order kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace topo {

// ----------------------------------------------------------------------------------
// Sum of per-chunk partials: out(b, e) = sum_c partials[b][c][e] for e < m (float64 sums
// of float32 or float64 partials).  A block of
// 1024 threads covers CW = 1024 / S consecutive entries with S chunk slices; slice s
// sums chunks s, s + S, ... (eight loads in flight), and the S slice sums are combined
// by a pairwise tree in LDS.  The order depends on nchunks and S only, and S on
// nchunks only, so a field's result is bitwise the same alone and inside a batch.
// ----------------------------------------------------------------------------------
constexpr int kSumBlock = 1024;

inline int chunk_slices(int nchunks) {
    int S = 1;
    while (S < 32 && (nchunks + S - 1) / S > 32) S *= 2;
    return S;
}

template <typename Epi, typename P>
__global__ __launch_bounds__(kSumBlock) void k_chunk_sum(int m, int nchunks, int S,
                                                         const P* __restrict__ partials, Epi epi) {
    __shared__ double red[kSumBlock];
    const int CW = kSumBlock / S;
    const int col = threadIdx.x % CW, sl = threadIdx.x / CW;
    const int e = blockIdx.x * CW + col;
    const int b = blockIdx.y;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (e < m) {
        const P* src = partials + (size_t)b * nchunks * m + e;
        int c = sl;
        for (; c + 7 * S < nchunks; c += 8 * S)
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] += (double)src[(size_t)(c + q * S) * m];
#pragma unroll
        for (int q = 0; q < 7; ++q)
            if (c + q * S < nchunks) acc[q] += (double)src[(size_t)(c + q * S) * m];
    }
    red[threadIdx.x] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    for (int h = S >> 1; h > 0; h >>= 1) {
        if (sl < h) red[threadIdx.x] += red[threadIdx.x + h * CW];
        __syncthreads();
    }
    if (sl == 0 && e < m) epi(b, e, red[threadIdx.x]);
}

// Column sums: out[b][j], m = k.
struct ColsumOut {
    int k;
    double* out;
    __device__ void operator()(int b, int j, double s) const { out[(size_t)b * k + j] = s; }
};

template <typename Epi, typename P>
inline void launch_chunk_sum(int m, int nchunks, int B, const P* partials, Epi epi, hipStream_t s) {
    const int S = chunk_slices(nchunks);
    const int CW = kSumBlock / S;
    hipLaunchKernelGGL((k_chunk_sum<Epi, P>), dim3((m + CW - 1) / CW, B), dim3(kSumBlock), 0, s, m, nchunks, S,
                       partials, epi);
}

}  // namespace topo
