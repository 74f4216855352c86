// In-place symmetrisation of a BCSS tensor (the post-processing step the
// paper suggests at the end of §5.4): an entry of a stored block whose block
// indices repeat is computed once per position, so mirrored entries inside
// the block can differ by rounding; each is replaced by the average over the
// block's stabiliser (the permutations of modes with equal block index).
// Blocks with distinct block indices are already the unique copy of their
// entries and are left as they are.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "common.hpp"
#include "kernels.hpp"

namespace symt {
namespace {

template <class E>
struct SymAcc {
    typedef float T;
    __device__ static float load(E v) { return (float)v; }
    __device__ static E store(float v) { return (E)v; }
};
template <>
struct SymAcc<double> {
    typedef double T;
    __device__ static double load(double v) { return v; }
    __device__ static double store(double v) { return v; }
};
template <>
struct SymAcc<uint16_t> {   // bf16 bits
    typedef float T;
    __device__ static float load(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
    __device__ static uint16_t store(float f)
    {
        uint32_t u = __float_as_uint(f);   // round to nearest, ties to even (finite values)
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (uint16_t)(u >> 16);
    }
};

// One workgroup per stored block with a repeated block index (grid-stride
// over the list of such blocks).  The orbit of entry l under
// the stabiliser is processed by the thread whose l is the smallest in the
// orbit: it sums the orbit (stabiliser order, identity first), divides by the
// stabiliser's size and writes the average back to every member.  Orbits are
// disjoint, so no two threads touch the same entry.
template <class E>
__global__ void bcss_symmetrize_kernel(E *__restrict__ bcss, int m, int b, int64_t bm, const int32_t *__restrict__ blocks,
                                       int64_t nlist, const int32_t *__restrict__ tuples,
                                       const int32_t *__restrict__ stab_start, const uint8_t *__restrict__ stab_perm)
{
    using Acc = SymAcc<E>;
    using T = typename Acc::T;
    for (int64_t x = blockIdx.x; x < nlist; x += gridDim.x) {
        const int64_t r = blocks[x];
        int mask = 0;
        for (int j = 0; j + 1 < m; ++j) mask |= (tuples[r * m + j] == tuples[r * m + j + 1] ? 1 : 0) << j;
        if (mask == 0) continue;
        const int p0 = stab_start[mask], p1 = stab_start[mask + 1];
        E *blk = bcss + r * bm;
        const int bm32 = (int)bm;   // the launcher keeps b^m below 2^31
        for (int l = threadIdx.x; l < bm32; l += blockDim.x) {
            int d[kMaxOrder];
            int q = l;
            for (int j = 0; j < m; ++j) {
                const int qn = q / b;
                d[j] = q - qn * b;
                q = qn;
            }
            auto image = [&](int p) {
                int o = 0, w = 1;
                for (int j = 0; j < m; ++j) {
                    o += d[stab_perm[p * m + j]] * w;
                    w *= b;
                }
                return o;
            };
            bool rep = true;
            for (int p = p0 + 1; p < p1 && rep; ++p) rep = image(p) >= l;
            if (!rep) continue;
            T sum = 0;
            for (int p = p0; p < p1; ++p) sum += Acc::load(blk[image(p)]);
            const E v = Acc::store(sum / (T)(p1 - p0));
            for (int p = p0; p < p1; ++p) blk[image(p)] = v;
        }
    }
}

// The same averages with the block staged in LDS (blocks of at most
// kSymLdsBytes), one workgroup per block, computed by every entry for
// itself: entry l finds its orbit representative (the smallest image of l),
// sums the representative's images in stabiliser order (so every member of
// an orbit adds the same values in the same order and gets the same bits as
// the representative in the kernel above), and writes only itself.  The
// whole block is staged before any entry is written, and no other workgroup
// touches the block, so every average is taken over the block's values as
// they were.  The block is read with coalesced 16-byte vectors (4-byte words
// when its size is not a multiple of 16 bytes).  The image of l under
// permutation p is sum_i d_i(l) * b^(p^-1(i)): shifts by p^-1(i) * log2(b)
// from a host table when b is a power of two, else weights tabulated in LDS
// once per block.  The run mask of each listed block comes from a host list
// (loaded beside the block's rank), so the only loads that wait on another
// are the block itself and the stabiliser's tables.
constexpr int kSymLdsBytes = 32768;
constexpr int kSymMaxPerms = 720;   // |S_6|
constexpr int kSymThreads = 1024;

template <class E>
__global__ __launch_bounds__(kSymThreads) void bcss_symmetrize_lds_kernel(
    E *__restrict__ bcss, int m, int b, int lb, int bm, const int32_t *__restrict__ blocks,
    const uint8_t *__restrict__ masks, int64_t nlist, const int32_t *__restrict__ stab_start,
    const uint8_t *__restrict__ stab_perm, const int32_t *__restrict__ stab_pinv)
{
    using Acc = SymAcc<E>;
    using T = typename Acc::T;
    extern __shared__ __attribute__((aligned(16))) unsigned char sym_smem[];
    __shared__ int32_t s_w[kSymMaxPerms * kMaxOrder];
    E *sb = (E *)sym_smem;
    const int bytes = bm * (int)sizeof(E);
    const bool vec16 = bytes % 16 == 0;
    for (int64_t x = blockIdx.x; x < nlist; x += gridDim.x) {
        const int64_t r = blocks[x];
        const int mask = masks[x];
        E *blk = bcss + r * (int64_t)bm;
        if (vec16) {
            for (int v = threadIdx.x; v < bytes / 16; v += blockDim.x) ((uint4 *)sym_smem)[v] = ((const uint4 *)blk)[v];
        } else {
            for (int v = threadIdx.x; v < bm; v += blockDim.x) sb[v] = blk[v];
        }
        const int p0 = stab_start[mask], p1 = stab_start[mask + 1];
        const int np = p1 - p0;   // <= kSymMaxPerms (checked by the launcher)
        // Every permutation's weights go to LDS with the block, so that the
        // loops over the permutations below read them from LDS rather than
        // waiting on a global read per permutation.
        if (lb < 0)
            for (int t = threadIdx.x; t < np * m; t += blockDim.x) {
                const int pp = t / m, j = t - pp * m;   // position j holds mode perm[j]: weight b^j for that mode
                int w = 1;
                for (int e = 0; e < j; ++e) w *= b;
                s_w[pp * kMaxOrder + stab_perm[(p0 + pp) * m + j]] = w;
            }
        else
            for (int t = threadIdx.x; t < np * m; t += blockDim.x) {
                const int pp = t / m, i = t - pp * m;   // mode i sits at position pinv(i): weight b^pinv(i)
                s_w[pp * kMaxOrder + i] = 1 << (stab_pinv[(int64_t)(p0 + pp) * kMaxOrder + i] * lb);
            }
        __syncthreads();
        auto digits = [&](int l, int *d) {
            if (lb >= 0) {   // b = 2^lb: digits are bit fields
#pragma unroll
                for (int j = 0; j < kMaxOrder; ++j) d[j] = j < m ? (l >> (j * lb)) & (b - 1) : 0;
            } else {
                int q = l;
#pragma unroll
                for (int j = 0; j < kMaxOrder; ++j) {
                    if (j < m) {
                        const int qn = q / b;
                        d[j] = q - qn * b;
                        q = qn;
                    } else {
                        d[j] = 0;
                    }
                }
            }
        };
        // Weights of permutation pp (uniform over the workgroup): b^pinv(i).
        auto weights = [&](int pp, int *w) {
#pragma unroll
            for (int i = 0; i < kMaxOrder; ++i) w[i] = i < m ? s_w[pp * kMaxOrder + i] : 0;
        };
        auto image = [&](const int *d, const int *w) {
            int o = 0;
#pragma unroll
            for (int i = 0; i < kMaxOrder; ++i) o += d[i] * w[i];
            return o;
        };
        // Four entries per thread at a time, so that every permutation's
        // weights are fetched once for four images.
        constexpr int kE = 4;
        for (int l0 = threadIdx.x; l0 < bm; l0 += kE * blockDim.x) {
            int d[kE][kMaxOrder], rep[kE];
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                rep[e] = l0 + e * (int)blockDim.x;   // identity is the stabiliser's first element
                digits(rep[e] < bm ? rep[e] : 0, d[e]);
            }
            int w[kMaxOrder];
            for (int pp = 1; pp < np; ++pp) {
                weights(pp, w);
#pragma unroll
                for (int e = 0; e < kE; ++e) rep[e] = min(rep[e], image(d[e], w));
            }
#pragma unroll
            for (int e = 0; e < kE; ++e) digits(rep[e] < bm ? rep[e] : 0, d[e]);
            T sum[kE];
#pragma unroll
            for (int e = 0; e < kE; ++e) sum[e] = 0;
            for (int pp = 0; pp < np; ++pp) {
                weights(pp, w);
#pragma unroll
                for (int e = 0; e < kE; ++e) sum[e] += Acc::load(sb[image(d[e], w)]);
            }
#pragma unroll
            for (int e = 0; e < kE; ++e) {
                const int l = l0 + e * (int)blockDim.x;
                if (l < bm) blk[l] = Acc::store(sum[e] / (T)np);
            }
        }
        __syncthreads();   // the next block reuses the staging buffer and the weights
    }
}

template <class E>
int launch_sym_t(void *bcss, int m, int b, int64_t bm, const int32_t *blocks, const uint8_t *masks, int64_t nlist,
                 const int32_t *tuples, const int32_t *stab_start, const uint8_t *stab_perm, const int32_t *stab_pinv,
                 hipStream_t s)
{
    const int64_t grid = std::min<int64_t>(std::max<int64_t>(nlist, 1), 1 << 16);
    int lb = -1;
    for (int e = 0; e < 31; ++e)
        if ((1 << e) == b) lb = e;
    const int64_t bytes = bm * (int64_t)sizeof(E);
    // 16-byte staging needs 16-byte aligned blocks: the tensor base is, and
    // so is every block when a block is a whole number of 16-byte vectors.
    const bool aligned = ((uintptr_t)bcss % 16) == 0;
    int fact = 1;
    for (int j = 2; j <= m; ++j) fact *= j;
    if (bytes <= kSymLdsBytes && fact <= kSymMaxPerms && (aligned || bytes % 16 != 0))
        hipLaunchKernelGGL(bcss_symmetrize_lds_kernel<E>, dim3((unsigned)grid), dim3(kSymThreads), (size_t)bytes, s,
                           (E *)bcss, m, b, lb, (int)bm, blocks, masks, nlist, stab_start, stab_perm, stab_pinv);
    else
        hipLaunchKernelGGL(bcss_symmetrize_kernel<E>, dim3((unsigned)grid), dim3(256), 0, s, (E *)bcss, m, b, bm, blocks,
                           nlist, tuples, stab_start, stab_perm);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int launch_symmetrize(int dtype, void *bcss, int m, int b, const int32_t *d_tuples, const int32_t *d_blocks,
                      const uint8_t *d_masks, int64_t nlist, const int32_t *d_stab_start, const uint8_t *d_stab_perm,
                      const int32_t *d_stab_pinv, hipStream_t s)
{
    int64_t bm = 1;
    for (int j = 0; j < m; ++j) bm *= b;
    if (bm > INT32_MAX) return -1;
    if (nlist <= 0) return 0;
    if (dtype == F32)
        return launch_sym_t<float>(bcss, m, b, bm, d_blocks, d_masks, nlist, d_tuples, d_stab_start, d_stab_perm,
                                     d_stab_pinv, s);
    if (dtype == BF16)
        return launch_sym_t<uint16_t>(bcss, m, b, bm, d_blocks, d_masks, nlist, d_tuples, d_stab_start, d_stab_perm,
                                        d_stab_pinv, s);
    if (dtype == F64)
        return launch_sym_t<double>(bcss, m, b, bm, d_blocks, d_masks, nlist, d_tuples, d_stab_start, d_stab_perm,
                                      d_stab_pinv, s);
    return -1;
}

}  // namespace symt
