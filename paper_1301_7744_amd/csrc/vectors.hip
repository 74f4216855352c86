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
// the dot products with a fixed reduction tree.  No atomics.  For m = 3 the
// first kernel is block-major instead (vec_block3_kernel: every stored block
// read once per batch, one partial per term).
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

// Block-major form for m = 3: one workgroup per stored block (entry
// (d0, d1, d2) at stored digits d, block tuple s0 <= s1 <= s2), which it reads
// once into LDS and then contracts with every vector of the batch, VB = 256/B
// vectors per pass.  Thread (vl, d2) runs over the block's (d0, d1) plane at
// its d2:
//   g1[d1]  = sum_d0 a x0[d0]           (no x2: gives position 2 and, times
//   T2[d2]  = sum_d1 x1[d1] g1[d1]       x2, position 1's partial)
//   T0[d0]  = x2 sum_d1 a x1[d1]        (partial over d2)
//   T1[d1]  = x2 g1[d1]                 (partial over d2)
// with x_j the vector's segment at block index s_j.  The partials over d2 are
// added through LDS in a fixed order (d2 = 0, 1, ...).  Each of the block's
// terms (the first position q of each distinct index, weight w) writes
// w T_q to its own partial slot; the rows of y add their slots in order.
template <class E, int B>
__global__ __launch_bounds__(256) void vec_block3_kernel(const E *__restrict__ A, const E *__restrict__ x,
                                                         int64_t rs_x, int64_t V, int64_t n,
                                                         const VecEntry *__restrict__ entries,
                                                         const int32_t *__restrict__ blk_begin,
                                                         const int32_t *__restrict__ blk_terms,
                                                         float *__restrict__ part)
{
    constexpr int VB = 256 / B;
    constexpr int S2 = B * B + 1;   // LDS stride of digit 2 (spreads the d2 threads over banks)
    __shared__ float s_blk[B * S2];
    __shared__ float s_x[3][VB][B];
    __shared__ float s_red[2][VB][B][B + 1];
    const int64_t r = blockIdx.x;
    const int tid = threadIdx.x, vl = tid / B, d2 = tid % B;
    const int t0 = blk_begin[r], t1 = blk_begin[r + 1];
    const VecEntry e0 = entries[blk_terms[t0]];
    const int64_t seg[3] = {(int64_t)e0.s[0] * B, (int64_t)e0.s[1] * B, (int64_t)e0.s[2] * B};
    const E *blk = A + r * (B * B * B);
    // (Loops with a fixed trip count, unrolled, so that each thread's loads
    // all go out before the first one is waited for.)
    constexpr int BLK_IT = (B * B * B + 255) / 256;
#pragma unroll
    for (int it = 0; it < BLK_IT; ++it) {
        const int g = tid + 256 * it;
        if (g < B * B * B) s_blk[(g % (B * B)) + (g / (B * B)) * S2] = ld(blk, g);
    }
    // The block's terms (one per distinct block index: at most 3), read once
    // for every pass over the vectors.
    const int nterm = t1 - t0;
    int tidx[3] = {0, 0, 0}, tq[3] = {0, 0, 0};
    float tw[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int e = 0; e < 3; ++e)
        if (e < nterm) tidx[e] = blk_terms[t0 + e];
#pragma unroll
    for (int e = 0; e < 3; ++e)
        if (e < nterm) {
            tq[e] = entries[tidx[e]].q;
            tw[e] = entries[tidx[e]].w;
        }
    for (int64_t v0 = 0; v0 < V; v0 += VB) {
        const int64_t v = v0 + vl;
        const bool live = v < V;
        __syncthreads();   // the block is staged; the previous pass is done with s_x and s_red
        constexpr int X_IT = (3 * VB * B + 255) / 256;
#pragma unroll
        for (int it = 0; it < X_IT; ++it) {
            const int t = tid + 256 * it;
            if (t < 3 * VB * B) {
                const int j = t / (VB * B), vv = (t / B) % VB, d = t % B;
                const int64_t xi = seg[j] + d, xv = v0 + vv;
                s_x[j][vv][d] = (xv < V && xi < n) ? ld(x, xv * rs_x + xi) : 0.f;
            }
        }
        __syncthreads();
        float x0[B], x1[B], T0[B], g1[B];
#pragma unroll
        for (int d = 0; d < B; ++d) {
            x0[d] = s_x[0][vl][d];
            x1[d] = s_x[1][vl][d];
            T0[d] = 0.f;
            g1[d] = 0.f;
        }
        const float x2 = s_x[2][vl][d2];
        const float *ab = s_blk + d2 * S2;
#pragma unroll
        for (int d1 = 0; d1 < B; ++d1)
#pragma unroll
            for (int d0 = 0; d0 < B; ++d0) {
                const float av = ab[d0 + B * d1];
                g1[d1] += av * x0[d0];
                T0[d0] += av * x1[d1];
            }
        float T2 = 0.f;
#pragma unroll
        for (int d1 = 0; d1 < B; ++d1) T2 += x1[d1] * g1[d1];
#pragma unroll
        for (int d = 0; d < B; ++d) {
            s_red[0][vl][d2][d] = x2 * T0[d];
            s_red[1][vl][d2][d] = x2 * g1[d];
        }
        __syncthreads();
        float R0 = 0.f, R1 = 0.f;   // rows l = d2 of positions 0 and 1, added over the d2 slices in order
#pragma unroll
        for (int k = 0; k < B; ++k) {
            R0 += s_red[0][vl][k][d2];
            R1 += s_red[1][vl][k][d2];
        }
        if (live) {
#pragma unroll
            for (int e = 0; e < 3; ++e)
                if (e < nterm) {
                    const float val = tq[e] == 0 ? R0 : (tq[e] == 1 ? R1 : T2);
                    part[((int64_t)tidx[e] * V + v) * B + d2] = tw[e] * val;
                }
            for (int t = t0 + 3; t < t1; ++t) {   // more than 3 terms: never for m = 3
                const int idx = blk_terms[t];
                const int q = entries[idx].q;
                const float val = q == 0 ? R0 : (q == 1 ? R1 : T2);
                part[((int64_t)idx * V + v) * B + d2] = entries[idx].w * val;
            }
        }
    }
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

// Rows of y for the block-major form: workgroup (v, u) adds, for each of
// the b rows of output block u, the partials of u's entries, S = 256 / b
// slices of the entry list per row (slice k takes entries k, k + S, ...,
// each in order) joined by a fixed pairwise tree; it writes the rows and the
// block's share of x_v . y_v (its b products added in order).
template <class E>
__global__ __launch_bounds__(256) void vec_rows_kernel(const float *__restrict__ part,
                                                       const int32_t *__restrict__ u_entry,
                                                       const E *__restrict__ x, int64_t rs_x, int64_t V, int64_t n,
                                                       int b, float *__restrict__ y, int64_t rs_y,
                                                       float *__restrict__ dotp)
{
    __shared__ float red[256];
    const int64_t v = blockIdx.x;
    const int u = blockIdx.y;
    const int S = 256 / b;
    const int l = threadIdx.x % b, k = threadIdx.x / b;
    float acc = 0.f;
    if (k < S) {
        // entries c, c + S, ... in order, four loads out at a time
        const int c1 = u_entry[u + 1];
        for (int c = u_entry[u] + k; c < c1; c += 4 * S) {
            float pv[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int cc = c + e * S;
                pv[e] = cc < c1 ? part[((int64_t)cc * V + v) * b + l] : 0.f;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (c + e * S < c1) acc += pv[e];
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = S / 2; h > 0; h >>= 1) {
        if (k < h) red[threadIdx.x] += red[threadIdx.x + h * b];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float dot = 0.f;
        for (int i = 0; i < b; ++i) {
            const int64_t row = (int64_t)u * b + i;
            if (row < n) {
                y[v * rs_y + row] = red[i];
                dot += ld(x, v * rs_x + row) * red[i];
            }
        }
        dotp[(int64_t)u * V + v] = dot;
    }
}

// s_v: the blocks' shares of x_v . y_v added in block order.
__global__ __launch_bounds__(256) void vec_dot_kernel(const float *__restrict__ dotp, int nbar, int64_t V,
                                                      float *__restrict__ s)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= V) return;
    float t = 0.f;
    for (int u0 = 0; u0 < nbar; u0 += 8) {   // in block order, eight loads out at a time
        float dv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) dv[e] = u0 + e < nbar ? dotp[(int64_t)(u0 + e) * V + v] : 0.f;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (u0 + e < nbar) t += dv[e];
    }
    s[v] = t;
}

template <class E, int B>
int launch_vec_blocks_b(const void *A, const void *x, int64_t rs_x, int64_t V, int64_t n, int64_t nblocks,
                        const VecEntry *d_entries, const int32_t *d_blk_begin, const int32_t *d_blk_terms,
                        const int32_t *d_u_entry, float *part, float *dotp, float *y, int64_t rs_y, float *s,
                        hipStream_t st)
{
    const int64_t nbar = (n + B - 1) / B;
    if (nblocks > INT32_MAX || V > INT32_MAX || nbar > 65535) return -1;
    hipLaunchKernelGGL((vec_block3_kernel<E, B>), dim3((unsigned)nblocks), dim3(256), 0, st, (const E *)A,
                       (const E *)x, rs_x, V, n, d_entries, d_blk_begin, d_blk_terms, part);
    hipLaunchKernelGGL(vec_rows_kernel<E>, dim3((unsigned)V, (unsigned)nbar), dim3(256), 0, st, (const float *)part,
                       d_u_entry, (const E *)x, rs_x, V, n, B, y, rs_y, dotp);
    if (s)
        hipLaunchKernelGGL(vec_dot_kernel, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, st, (const float *)dotp,
                           (int)nbar, V, s);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <class E>
int launch_vec_blocks_t(const void *A, const void *x, int64_t rs_x, int64_t V, int64_t n, int b, int64_t nblocks,
                        const VecEntry *d_entries, const int32_t *d_blk_begin, const int32_t *d_blk_terms,
                        const int32_t *d_u_entry, float *part, float *dotp, float *y, int64_t rs_y, float *s,
                        hipStream_t st)
{
    switch (b) {
    case 4:
        return launch_vec_blocks_b<E, 4>(A, x, rs_x, V, n, nblocks, d_entries, d_blk_begin, d_blk_terms, d_u_entry,
                                         part, dotp, y, rs_y, s, st);
    case 8:
        return launch_vec_blocks_b<E, 8>(A, x, rs_x, V, n, nblocks, d_entries, d_blk_begin, d_blk_terms, d_u_entry,
                                         part, dotp, y, rs_y, s, st);
    case 16:
        return launch_vec_blocks_b<E, 16>(A, x, rs_x, V, n, nblocks, d_entries, d_blk_begin, d_blk_terms, d_u_entry,
                                          part, dotp, y, rs_y, s, st);
    default: return -1;
    }
}

}  // namespace

int launch_vectors_blocks(int dtype, const void *A, const void *x, int64_t rs_x, int64_t V, int64_t n, int b,
                          int64_t nblocks, const VecEntry *d_entries, const int32_t *d_blk_begin,
                          const int32_t *d_blk_terms, const int32_t *d_u_entry, float *part, float *dotp, float *y,
                          int64_t rs_y, float *s, hipStream_t st)
{
    if (V <= 0 || nblocks <= 0) return V <= 0 ? 0 : -1;
    if (dtype == F32)
        return launch_vec_blocks_t<float>(A, x, rs_x, V, n, b, nblocks, d_entries, d_blk_begin, d_blk_terms,
                                          d_u_entry, part, dotp, y, rs_y, s, st);
    if (dtype == BF16)
        return launch_vec_blocks_t<uint16_t>(A, x, rs_x, V, n, b, nblocks, d_entries, d_blk_begin, d_blk_terms,
                                             d_u_entry, part, dotp, y, rs_y, s, st);
    return -1;
}

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
