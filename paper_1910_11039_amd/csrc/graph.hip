// Vertex renumbering of the uploaded graph (hub-first order in HBM) and the
// per-vertex permutations between the caller's numbering and the internal
// one.
#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "kad_internal.h"

namespace kad {
namespace {

// A wave per output row: row i copies row orig[i] of the input, mapping
// every neighbour through newid; the neighbour order is kept.
__global__ void k_relabel_rows(int32_t n, const int64_t *rp_in, const int32_t *ci_in, const int32_t *orig,
                               const int32_t *newid, const int64_t *rp_out, int32_t *ci_out)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = wave; i < n; i += waves) {
        const int32_t v = orig[i];
        const int64_t b = rp_in[v], e = rp_in[v + 1], o = rp_out[i];
        for (int64_t k = lane; k < e - b; k += 64) ci_out[o + k] = newid[ci_in[b + k]];
    }
}

// Clears `words` 32-bit words (a kernel, not a memset node, so that it is
// safe under stream capture).
__global__ void k_zero_words(uint32_t *p, size_t words)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0u;
}

__global__ void k_degrees(int32_t n, const int64_t *rp, uint32_t *deg)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        deg[v] = (uint32_t)(rp[v + 1] - rp[v]);
}

template <typename T>
__global__ void k_to_caller(int32_t n, const int32_t *orig, const T *in, T *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[orig[i]] = in[i];
}

template <typename T>
__global__ void k_from_caller(int32_t n, const int32_t *orig, const T *in, T *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[orig[i]];
}

__global__ void k_to_caller_rows3(int32_t n, const int32_t *orig, const float *in, float *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = orig[i];
        out[3 * o + 0] = in[3 * i + 0];
        out[3 * o + 1] = in[3 * i + 1];
        out[3 * o + 2] = in[3 * i + 2];
    }
}

unsigned blocks_for(int64_t n, int per = 256)
{
    int64_t b = (n + per - 1) / per;
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned)b;
}

}  // namespace

hipError_t launch_relabel_rows(int32_t n, const int64_t *rp_in, const int32_t *ci_in, const int32_t *orig,
                               const int32_t *newid, const int64_t *rp_out, int32_t *ci_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_relabel_rows, dim3(8192), dim3(256), 0, st, n, rp_in, ci_in, orig, newid, rp_out, ci_out);
    return hipGetLastError();
}

hipError_t sort_rows(int32_t n, int64_t nnz, const int64_t *rp, const int32_t *in, int32_t *out, hipStream_t st)
{
    if (nnz > 0x7fffffffll) return hipErrorInvalidValue;
    size_t bytes = 0;
    hipError_t e = hipcub::DeviceSegmentedSort::SortKeys(nullptr, bytes, in, out, (int)nnz, (int)n, rp, rp + 1, st);
    if (e != hipSuccess) return e;
    void *tmp = nullptr;
    if ((e = hipMallocAsync(&tmp, std::max<size_t>(bytes, 16), st)) != hipSuccess) return e;
    e = hipcub::DeviceSegmentedSort::SortKeys(tmp, bytes, in, out, (int)nnz, (int)n, rp, rp + 1, st);
    const hipError_t f = hipFreeAsync(tmp, st);
    return e != hipSuccess ? e : f;
}

hipError_t launch_zero_words(uint32_t *p, size_t words, hipStream_t st)
{
    if (words == 0) return hipSuccess;
    size_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, st, p, words);
    return hipGetLastError();
}

hipError_t launch_degrees(int32_t n, const int64_t *rp, uint32_t *deg, hipStream_t st)
{
    hipLaunchKernelGGL(k_degrees, dim3(blocks_for(n)), dim3(256), 0, st, n, rp, deg);
    return hipGetLastError();
}

hipError_t launch_to_caller_u32(int32_t n, const int32_t *orig, const uint32_t *in, uint32_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_caller<uint32_t>, dim3(blocks_for(n)), dim3(256), 0, st, n, orig, in, out);
    return hipGetLastError();
}

hipError_t launch_to_caller_f64(int32_t n, const int32_t *orig, const double *in, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_caller<double>, dim3(blocks_for(n)), dim3(256), 0, st, n, orig, in, out);
    return hipGetLastError();
}

hipError_t launch_to_caller_f32x3(int32_t n, const int32_t *orig, const float *in, float *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_caller_rows3, dim3(blocks_for(n)), dim3(256), 0, st, n, orig, in, out);
    return hipGetLastError();
}

hipError_t launch_from_caller_f64(int32_t n, const int32_t *orig, const double *in, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_from_caller<double>, dim3(blocks_for(n)), dim3(256), 0, st, n, orig, in, out);
    return hipGetLastError();
}

}  // namespace kad
