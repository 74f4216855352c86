// Batched vector products with a BCSS tensor (the CP case of §2.5, where the
// matrix of sttsm is a single vector): for vectors x_v,
//   y_v = A x_v^(m-1)   (y_v[i] = sum over i_2..i_m of a_{i i_2 .. i_m} x_v[i_2] ... x_v[i_m])
//   s_v = A x_v^m = x_v . y_v.
// Every stored block adds to the rows of y of each distinct block index it
// holds: with the free index at the first stored position carrying that
// index, contracted with x in every other position, times the number of
// block tuples with that leading index that sort to the block (VecEntry).
// Deterministic: the first kernel writes one partial per (chunk of terms,
// vector, row), the second adds each row's chunks in a fixed order and forms
// the dot products with a fixed reduction tree.  No atomics.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace symt {
namespace {

template <class E>
__device__ __forceinline__ float ld(const E *p, int64_t i);
template <>
__device__ __forceinline__ float ld<float>(const float *p, int64_t i)
{
    return p[i];
}
template <>
__device__ __forceinline__ float ld<uint16_t>(const uint16_t *p, int64_t i)
{
    return __uint_as_float(((uint32_t)p[i]) << 16);
}

constexpr int kVecLdsBlock = 8192;   // entries of a block staged in LDS

// Workgroup = (chunk of terms, group of VB vectors).  For each term the
// stored block is staged in LDS with the free position's index fastest
// (entry (l, rest) at l + b * rest, rest counting the other positions in
// stored order) and the x segments of the other positions next to it; then
// thread (l, vl, os) sums the rest combinations o = os, os + OS, ... of its
// row l and vector vl.  The OS partial sums of a (row, vector) are added in
// a fixed order at the end.
template <class E>
__global__ __launch_bounds__(256) void vec_partial_kernel(const E *__restrict__ A, const E *__restrict__ x,
                                                          int64_t rs_x, int64_t V, int m, int64_t n, int b, int64_t bm,
                                                          const VecEntry *__restrict__ entries,
                                                          const int32_t *__restrict__ chunk_begin,
                                                          float *__restrict__ part, int VB, int OS)
{
    __shared__ float s_blk[kVecLdsBlock];
    __shared__ float s_x[kMaxOrder * 256];   // [rest position k][vl][d], VB * b <= 256
    __shared__ float s_red[256];
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    const int l = tid % b, vl = (tid / b) % VB, os = tid / (b * VB);
    const int64_t v0 = (int64_t)blockIdx.y * VB;
    const bool live = os < OS && v0 + vl < V;
    const int e0 = chunk_begin[c], e1 = chunk_begin[c + 1];
    float acc = 0.f;
    for (int e = e0; e < e1; ++e) {
        const VecEntry en = entries[e];
        int64_t rbase[kMaxOrder];
        int R = 0;
        for (int j = 0; j < m; ++j)
            if (j != en.q) rbase[R++] = (int64_t)en.s[j] * b;
        __syncthreads();   // the previous term is done with the LDS
        // stage the block, free index fastest
        const E *blk = A + (int64_t)en.r * bm;
        for (int g = tid; g < (int)bm; g += 256) {
            int rem = g, dq = 0, rest = 0, w = 1;
            for (int j = 0; j < m; ++j) {
                const int d = rem % b;
                rem /= b;
                if (j == en.q) dq = d;
                else { rest += d * w; w *= b; }
            }
            s_blk[dq + b * rest] = ld(blk, g);
        }
        // x segments of the rest positions for the VB vectors (zero beyond n)
        for (int t = tid; t < R * VB * b; t += 256) {
            const int d = t % b, vv = (t / b) % VB, k = t / (b * VB);
            const int64_t xi = rbase[k] + d, v = v0 + vv;
            s_x[t] = (v < V && xi < n) ? ld(x, v * rs_x + xi) : 0.f;
        }
        __syncthreads();
        if (live) {
            int outer = 1;
            for (int k = 1; k < R; ++k) outer *= b;
            float sum = 0.f;
            const float *x0 = s_x + (0 * VB + vl) * b;
            for (int o = os; o < outer; o += OS) {
                int rem = o;
                float P = 1.f;
                for (int k = 1; k < R; ++k) {
                    P *= s_x[(k * VB + vl) * b + rem % b];
                    rem /= b;
                }
                const float *row = s_blk + l + (int64_t)b * b * o;
                float t = 0.f;
                for (int d0 = 0; d0 < b; ++d0) t += row[b * d0] * x0[d0];
                sum += P * t;
            }
            acc += en.w * sum;
        }
    }
    // fixed-order sum over the OS slices of each (row, vector)
    __syncthreads();
    s_red[tid] = acc;
    __syncthreads();
    if (os == 0 && live) {
        float tot = 0.f;
        for (int k = 0; k < OS; ++k) tot += s_red[tid + k * b * VB];
        part[((int64_t)c * V + v0 + vl) * b + l] = tot;
    }
}

// One workgroup per vector: y_v row by row (chunks of the row's block index
// added in order), then s_v = x_v . y_v by a fixed tree over the threads.
template <class E>
__global__ __launch_bounds__(256) void vec_reduce_kernel(const float *__restrict__ part,
                                                         const int32_t *__restrict__ u_chunk,
                                                         const E *__restrict__ x, int64_t rs_x, int64_t V, int64_t n,
                                                         int b, float *__restrict__ y, int64_t rs_y,
                                                         float *__restrict__ s)
{
    __shared__ float red[256];
    const int64_t v = blockIdx.x;
    float dot = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t u = i / b, l = i - u * b;
        float yi = 0.f;
        for (int c = u_chunk[u]; c < u_chunk[u + 1]; ++c) yi += part[((int64_t)c * V + v) * b + l];
        y[v * rs_y + i] = yi;
        dot += ld(x, v * rs_x + i) * yi;
    }
    red[threadIdx.x] = dot;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && s) s[v] = red[0];
}

template <class E>
int launch_vec_t(const void *A, const void *x, int64_t rs_x, int64_t V, int m, int64_t n, int b,
                 const VecEntry *d_entries, const int32_t *d_chunk_begin, const int32_t *d_u_chunk, int nchunks,
                 float *part, float *y, int64_t rs_y, float *s, hipStream_t st)
{
    int64_t bm = 1;
    for (int j = 0; j < m; ++j) bm *= b;
    if (bm > kVecLdsBlock || b > 256) return -1;
    // VB vectors per workgroup (a power of two up to 256 / b, no more than
    // needed), and OS slices of the rest loop for the threads left over.
    int VB = 1;
    while (VB * 2 * b <= 256 && VB < V) VB *= 2;
    const int OS = std::max(1, 256 / (b * VB));
    const int64_t vgroups = (V + VB - 1) / VB;
    if (vgroups > 65535 || V > INT32_MAX) return -1;
    if (nchunks > 0)
        hipLaunchKernelGGL(vec_partial_kernel<E>, dim3((unsigned)nchunks, (unsigned)vgroups), dim3(256), 0, st,
                           (const E *)A, (const E *)x, rs_x, V, m, n, b, bm, d_entries, d_chunk_begin, part, VB, OS);
    hipLaunchKernelGGL(vec_reduce_kernel<E>, dim3((unsigned)V), dim3(256), 0, st, (const float *)part, d_u_chunk,
                       (const E *)x, rs_x, V, n, b, y, rs_y, s);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int launch_vectors(int dtype, const void *A, const void *x, int64_t rs_x, int64_t V, int m, int64_t n, int b,
                   const VecEntry *d_entries, const int32_t *d_chunk_begin, const int32_t *d_u_chunk, int nchunks,
                   float *part, float *y, int64_t rs_y, float *s, hipStream_t st)
{
    if (V <= 0) return 0;
    if (dtype == F32)
        return launch_vec_t<float>(A, x, rs_x, V, m, n, b, d_entries, d_chunk_begin, d_u_chunk, nchunks, part, y,
                                   rs_y, s, st);
    if (dtype == BF16)
        return launch_vec_t<uint16_t>(A, x, rs_x, V, m, n, b, d_entries, d_chunk_begin, d_u_chunk, nchunks, part, y,
                                      rs_y, s, st);
    return -1;
}

}  // namespace symt
