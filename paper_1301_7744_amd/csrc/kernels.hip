// gfx950 kernels of libsttsm: BCSS pack/unpack, X panel preparation, and the
// block-contraction stage kernel on MFMA.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <utility>

#include "common.hpp"
#include "kernels.hpp"

namespace symt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ u16 f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float(((uint32_t)h) << 16); }

// ------------------------------------------------------------------ pack/unpack
// Both kernels give one workgroup a whole block (grid-stride over blocks), so
// the block's index tuple, its meta-data and its base offsets are uniform,
// and let each thread move a run of 4 consecutive entries along mode 0, the
// fastest mode of both layouts: a wave reads and writes contiguous 4-entry
// runs, and only the digits of the run's row (modes 1..m-1) are divided out.

// A run of four consecutive entries moves as one vector when both ends are
// contiguous and aligned (vec: n and b multiples of 4, pointers aligned to
// four entries; the stored side also needs stride 1 along the run).
template <class E>
using Vec4 = E __attribute__((ext_vector_type(4)));

// Stored block r (colex) of BCSS <- its sorted block of the dense tensor;
// entries beyond n are written as zero.
template <class E>
__global__ void bcss_pack_kernel(const E *__restrict__ dense, E *__restrict__ bcss, int m, int64_t n, int b,
                                 int64_t bm, int64_t nblocks, const int32_t *__restrict__ tuples, int rows,
                                 int runs, int vec)
{
    for (int64_t r = blockIdx.x; r < nblocks; r += gridDim.x) {
        int64_t base = 0, npow = 1;
        int64_t s0b = 0;
        int32_t sb[kMaxOrder];
        for (int j = 0; j < m; ++j) {
            sb[j] = tuples[r * m + j] * b;
            base += (int64_t)sb[j] * npow;
            npow *= n;
        }
        s0b = sb[0];
        const int64_t lim0 = n - s0b;   // valid entries along mode 0
        E *out = bcss + r * bm;
        for (int t = threadIdx.x; t < rows * runs; t += blockDim.x) {
            const int row = t / runs, e0 = (t - row * runs) * 4;
            int rr = row;
            int64_t off = base, np = n;
            bool ok = true;
            for (int j = 1; j < m; ++j) {
                const int lj = rr % b;
                rr /= b;
                ok = ok && (int64_t)sb[j] + lj < n;
                off += (int64_t)lj * np;
                np *= n;
            }
            if (vec && e0 + 4 <= b && (!ok || e0 + 4 <= lim0)) {
                Vec4<E> v = {E(0), E(0), E(0), E(0)};
                if (ok) v = *(const Vec4<E> *)&dense[off + e0];
                *(Vec4<E> *)&out[(int64_t)row * b + e0] = v;
                continue;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int le = e0 + e;
                if (le < b) out[(int64_t)row * b + le] = (ok && le < lim0) ? dense[off + le] : E(0);
            }
        }
    }
}

// The vector case of bcss_pack_kernel (n and b multiples of 4, aligned
// pointers): every run is either wholly inside the tensor or wholly padding,
// since n - s_0 b is a multiple of 4.  Digits of a run's row are shifts when
// b = 2^lb (lb >= 0).  Each thread takes kPackRuns runs at a time and issues
// all their loads before any store.
constexpr int kPackRuns = 4;

template <class E>
__global__ __launch_bounds__(256) void bcss_pack_vec_kernel(const E *__restrict__ dense, E *__restrict__ bcss, int m,
                                                            int64_t n, int b, int lb, int64_t bm, int64_t nblocks,
                                                            const int32_t *__restrict__ tuples, int rows, int runs)
{
    const int total = rows * runs;
    for (int64_t r = blockIdx.x; r < nblocks; r += gridDim.x) {
        int64_t base = 0, npow = 1;
        int32_t sb[kMaxOrder];
        for (int j = 0; j < m; ++j) {
            sb[j] = tuples[r * m + j] * b;
            base += (int64_t)sb[j] * npow;
            npow *= n;
        }
        const int64_t lim0 = n - sb[0];
        E *out = bcss + r * bm;
        for (int t0 = threadIdx.x; t0 < total; t0 += kPackRuns * blockDim.x) {
            Vec4<E> v[kPackRuns];
#pragma unroll
            for (int u = 0; u < kPackRuns; ++u) {
                const int t = t0 + u * (int)blockDim.x;
                v[u] = Vec4<E>{E(0), E(0), E(0), E(0)};
                if (t >= total) continue;
                int row, e0;
                if (lb >= 0) {
                    row = t >> (lb - 2);
                    e0 = (t & (runs - 1)) * 4;
                } else {
                    row = t / runs;
                    e0 = (t - row * runs) * 4;
                }
                int rr = row;
                int64_t off = base, np = n;
                bool ok = e0 < lim0;
                for (int j = 1; j < m; ++j) {
                    int lj;
                    if (lb >= 0) {
                        lj = rr & (b - 1);
                        rr >>= lb;
                    } else {
                        lj = rr % b;
                        rr /= b;
                    }
                    ok = ok && (int64_t)sb[j] + lj < n;
                    off += (int64_t)lj * np;
                    np *= n;
                }
                if (ok) v[u] = *(const Vec4<E> *)&dense[off + e0];
            }
#pragma unroll
            for (int u = 0; u < kPackRuns; ++u) {
                const int t = t0 + u * (int)blockDim.x;
                if (t < total) *(Vec4<E> *)&out[(int64_t)t * 4] = v[u];
            }
        }
    }
}

// Dense block t (dimensional order over nbar^m) <- stored block sort(t), read
// through the permuted strides of the meta-data tensor (App. B).
template <class E>
__global__ void bcss_unpack_kernel(const E *__restrict__ bcss, E *__restrict__ dense, int m, int64_t n, int b,
                                   int nbar, int64_t bm, int64_t nbm, const int64_t *__restrict__ rank,
                                   const int32_t *__restrict__ perm, const int32_t *__restrict__ pstr, int rows,
                                   int runs, int vec)
{
    for (int64_t tb = blockIdx.x; tb < nbm; tb += gridDim.x) {
        int32_t tbj[kMaxOrder], ps[kMaxOrder];
        int64_t base = 0, npow = 1, q = tb;
        const int32_t *pp = pstr + (int64_t)perm[tb] * m;
        for (int j = 0; j < m; ++j) {
            tbj[j] = (int32_t)(q % nbar) * b;
            q /= nbar;
            base += (int64_t)tbj[j] * npow;
            npow *= n;
            ps[j] = pp[j];
        }
        const E *src = bcss + rank[tb] * bm;
        const int64_t lim0 = n - tbj[0];
        for (int t = threadIdx.x; t < rows * runs; t += blockDim.x) {
            const int row = t / runs, e0 = (t - row * runs) * 4;
            int rr = row;
            int64_t off = base, np = n, so = 0;
            bool ok = true;
            for (int j = 1; j < m; ++j) {
                const int lj = rr % b;
                rr /= b;
                ok = ok && (int64_t)tbj[j] + lj < n;
                off += (int64_t)lj * np;
                so += (int64_t)lj * ps[j];
                np *= n;
            }
            if (!ok) continue;
            if (vec && ps[0] == 1 && e0 + 4 <= b && e0 + 4 <= lim0) {
                *(Vec4<E> *)&dense[off + e0] = *(const Vec4<E> *)&src[so + e0];
                continue;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int le = e0 + e;
                if (le < b && le < lim0) dense[off + le] = src[so + (int64_t)le * ps[0]];
            }
        }
    }
}

// The same with the stored block staged in LDS (blocks of at most
// kUnpackLdsBytes): the block is read once with coalesced 16-byte vectors,
// the permuted reads hit LDS, and every run goes out as one vector when the
// dense side allows it.
constexpr int kUnpackLdsBytes = 32768;

template <class E>
__global__ void bcss_unpack_lds_kernel(const E *__restrict__ bcss, E *__restrict__ dense, int m, int64_t n, int b,
                                       int nbar, int bm, int64_t nbm, const int64_t *__restrict__ rank,
                                       const int32_t *__restrict__ perm, const int32_t *__restrict__ pstr, int rows,
                                       int runs, int vec, int src16)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char unpack_smem[];
    E *sb = (E *)unpack_smem;
    const int bytes = bm * (int)sizeof(E);
    const bool vec16 = src16 && bytes % 16 == 0;   // every stored block starts 16-byte aligned
    for (int64_t tb = blockIdx.x; tb < nbm; tb += gridDim.x) {
        int32_t tbj[kMaxOrder], ps[kMaxOrder];
        int64_t base = 0, npow = 1, q = tb;
        const int32_t *pp = pstr + (int64_t)perm[tb] * m;
        for (int j = 0; j < m; ++j) {
            tbj[j] = (int32_t)(q % nbar) * b;
            q /= nbar;
            base += (int64_t)tbj[j] * npow;
            npow *= n;
            ps[j] = pp[j];
        }
        const E *src = bcss + rank[tb] * (int64_t)bm;
        const int64_t lim0 = n - tbj[0];
        __syncthreads();   // the previous block's reads of the staging buffer are done
        if (vec16) {
            for (int v = threadIdx.x; v < bytes / 16; v += blockDim.x) ((uint4 *)unpack_smem)[v] = ((const uint4 *)src)[v];
        } else {
            for (int v = threadIdx.x; v < bm; v += blockDim.x) sb[v] = src[v];
        }
        __syncthreads();
        for (int t = threadIdx.x; t < rows * runs; t += blockDim.x) {
            const int row = t / runs, e0 = (t - row * runs) * 4;
            int rr = row;
            int64_t off = base, np = n;
            int so = 0;
            bool ok = true;
            for (int j = 1; j < m; ++j) {
                const int lj = rr % b;
                rr /= b;
                ok = ok && (int64_t)tbj[j] + lj < n;
                off += (int64_t)lj * np;
                so += lj * ps[j];
                np *= n;
            }
            if (!ok) continue;
            if (vec && e0 + 4 <= b && e0 + 4 <= lim0) {
                Vec4<E> v;
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = sb[so + (e0 + e) * ps[0]];
                *(Vec4<E> *)&dense[off + e0] = v;
                continue;
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int le = e0 + e;
                if (le < b && le < lim0) dense[off + le] = sb[so + le * ps[0]];
            }
        }
    }
}

// The vector case of bcss_unpack_lds_kernel (n and b multiples of 4,
// aligned pointers).  The staged block sits in LDS at padded positions
// pad(i) = i + i/16 + i/256, so that the permuted reads, whose strides along
// a run are 1, b, b^2, ..., fall on distinct banks for b = 16 (strides 17
// and 273 words); each thread takes kPackRuns runs at a time, reads all their
// entries from LDS, then stores them; digits are shifts when b = 2^lb.
__device__ __forceinline__ int unpack_pad(int i) { return i + (i >> 4) + (i >> 8); }

template <class E>
__global__ __launch_bounds__(256) void bcss_unpack_vec_kernel(const E *__restrict__ bcss, E *__restrict__ dense,
                                                              int m, int64_t n, int b, int lb, int nbar, int bm,
                                                              int64_t nbm, const int64_t *__restrict__ rank,
                                                              const int32_t *__restrict__ perm,
                                                              const int32_t *__restrict__ pstr, int rows, int runs,
                                                              int src16)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char unpack_smem[];
    E *sb = (E *)unpack_smem;
    const bool vec16 = src16 && (bm * (int)sizeof(E)) % 16 == 0;
    const int total = rows * runs;
    for (int64_t tb = blockIdx.x; tb < nbm; tb += gridDim.x) {
        int32_t tbj[kMaxOrder], ps[kMaxOrder];
        int64_t base = 0, npow = 1, q = tb;
        const int32_t *pp = pstr + (int64_t)perm[tb] * m;
        for (int j = 0; j < m; ++j) {
            tbj[j] = (int32_t)(q % nbar) * b;
            q /= nbar;
            base += (int64_t)tbj[j] * npow;
            npow *= n;
            ps[j] = pp[j];
        }
        const E *src = bcss + rank[tb] * (int64_t)bm;
        const int64_t lim0 = n - tbj[0];
        __syncthreads();   // the previous block's reads of the staging buffer are done
        if (vec16 && sizeof(E) == 4) {
            // four vectors per thread in flight before the first is stored
            constexpr int kU = 4;
            for (int v0 = threadIdx.x; v0 < bm / 4; v0 += kU * blockDim.x) {
                uint4 w[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int v = v0 + u * (int)blockDim.x;
                    w[u] = v < bm / 4 ? ((const uint4 *)src)[v] : uint4{0u, 0u, 0u, 0u};
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int v = v0 + u * (int)blockDim.x;
                    if (v >= bm / 4) continue;
                    uint32_t *d = (uint32_t *)sb + unpack_pad(4 * v);   // the four entries stay contiguous
                    d[0] = w[u].x;
                    d[1] = w[u].y;
                    d[2] = w[u].z;
                    d[3] = w[u].w;
                }
            }
        } else if (vec16 && sizeof(E) == 2) {
            // eight entries per 16-byte vector, two vectors per thread in flight
            constexpr int kU = 2;
            for (int v0 = threadIdx.x; v0 < bm / 8; v0 += kU * blockDim.x) {
                uint4 w[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int v = v0 + u * (int)blockDim.x;
                    w[u] = v < bm / 8 ? ((const uint4 *)src)[v] : uint4{0u, 0u, 0u, 0u};
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int v = v0 + u * (int)blockDim.x;
                    if (v >= bm / 8) continue;
                    const uint32_t ww[4] = {w[u].x, w[u].y, w[u].z, w[u].w};
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        ((uint16_t *)sb)[unpack_pad(8 * v + e)] = (uint16_t)(ww[e >> 1] >> (16 * (e & 1)));
                }
            }
        } else {
            for (int v = threadIdx.x; v < bm; v += blockDim.x) sb[unpack_pad(v)] = src[v];
        }
        __syncthreads();
        for (int t0 = threadIdx.x; t0 < total; t0 += kPackRuns * blockDim.x) {
            Vec4<E> v[kPackRuns];
            int64_t dst[kPackRuns];
            bool live[kPackRuns];
#pragma unroll
            for (int u = 0; u < kPackRuns; ++u) {
                const int t = t0 + u * (int)blockDim.x;
                int row, e0;
                if (lb >= 0) {
                    row = t >> (lb - 2);
                    e0 = (t & (runs - 1)) * 4;
                } else {
                    row = t / runs;
                    e0 = (t - row * runs) * 4;
                }
                int rr = row;
                int64_t off = base, np = n;
                int so = 0;
                bool ok = t < total && e0 < lim0;
                for (int j = 1; j < m; ++j) {
                    int lj;
                    if (lb >= 0) {
                        lj = rr & (b - 1);
                        rr >>= lb;
                    } else {
                        lj = rr % b;
                        rr /= b;
                    }
                    ok = ok && (int64_t)tbj[j] + lj < n;
                    off += (int64_t)lj * np;
                    so += lj * ps[j];
                    np *= n;
                }
                live[u] = ok;
                dst[u] = off + e0;
#pragma unroll
                for (int e = 0; e < 4; ++e) v[u][e] = ok ? sb[unpack_pad(so + (e0 + e) * ps[0])] : E(0);
            }
#pragma unroll
            for (int u = 0; u < kPackRuns; ++u)
                if (live[u]) *(Vec4<E> *)&dense[dst[u]] = v[u];
        }
    }
}

template <class E>
static int launch_pack_t(const void *dense, void *bcss, int m, int64_t n, int b, int64_t bm, int64_t nblocks,
                         const int32_t *tuples, hipStream_t s)
{
    const int rows = (int)(bm / b), runs = (b + 3) / 4;
    const int64_t grid = std::min<int64_t>(std::max<int64_t>(nblocks, 1), 1 << 16);
    const uintptr_t al = 4 * sizeof(E);
    const int vec = n % 4 == 0 && b % 4 == 0 && (uintptr_t)dense % al == 0 && (uintptr_t)bcss % al == 0;
    int lb = -1;
    for (int e = 2; e < 16; ++e)
        if ((1 << e) == b) lb = e;
    if (vec)
        hipLaunchKernelGGL(bcss_pack_vec_kernel<E>, dim3((unsigned)grid), dim3(256), 0, s, (const E *)dense,
                           (E *)bcss, m, n, b, lb, bm, nblocks, tuples, rows, runs);
    else
        hipLaunchKernelGGL(bcss_pack_kernel<E>, dim3((unsigned)grid), dim3(256), 0, s, (const E *)dense, (E *)bcss, m,
                           n, b, bm, nblocks, tuples, rows, runs, vec);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <class E>
static int launch_unpack_t(const void *bcss, void *dense, int m, int64_t n, int b, int nbar, int64_t bm,
                           int64_t nbm, const int64_t *rank, const int32_t *perm, const int32_t *pstr, hipStream_t s)
{
    const int rows = (int)(bm / b), runs = (b + 3) / 4;
    const int64_t grid = std::min<int64_t>(std::max<int64_t>(nbm, 1), 1 << 16);
    const uintptr_t al = 4 * sizeof(E);
    const int vec = n % 4 == 0 && b % 4 == 0 && (uintptr_t)dense % al == 0 && (uintptr_t)bcss % al == 0;
    int lb = -1;
    for (int e = 2; e < 16; ++e)
        if ((1 << e) == b) lb = e;
    if (vec && bm * (int64_t)sizeof(E) <= kUnpackLdsBytes)
        hipLaunchKernelGGL(bcss_unpack_vec_kernel<E>, dim3((unsigned)grid), dim3(256),
                           (size_t)((bm + bm / 16 + bm / 256 + 1) * sizeof(E)), s, (const E *)bcss, (E *)dense, m, n,
                           b, lb, nbar, (int)bm, nbm, rank, perm, pstr, rows, runs,
                           (int)((uintptr_t)bcss % 16 == 0));
    else if (bm * (int64_t)sizeof(E) <= kUnpackLdsBytes)
        hipLaunchKernelGGL(bcss_unpack_lds_kernel<E>, dim3((unsigned)grid), dim3(256), (size_t)(bm * sizeof(E)), s,
                           (const E *)bcss, (E *)dense, m, n, b, nbar, (int)bm, nbm, rank, perm, pstr, rows, runs, vec,
                           (int)((uintptr_t)bcss % 16 == 0));
    else
        hipLaunchKernelGGL(bcss_unpack_kernel<E>, dim3((unsigned)grid), dim3(256), 0, s, (const E *)bcss, (E *)dense,
                           m, n, b, nbar, bm, nbm, rank, perm, pstr, rows, runs, vec);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pack(int esize, const void *dense, void *bcss, int m, int64_t n, int b, int64_t nblocks,
                const int32_t *d_tuples, hipStream_t s)
{
    int64_t bm = 1;
    for (int j = 0; j < m; ++j) bm *= b;
    if (bm / b * ((b + 3) / 4) > INT32_MAX / 2) return -1;
    if (esize == 2) return launch_pack_t<uint16_t>(dense, bcss, m, n, b, bm, nblocks, d_tuples, s);
    if (esize == 4) return launch_pack_t<uint32_t>(dense, bcss, m, n, b, bm, nblocks, d_tuples, s);
    if (esize == 8) return launch_pack_t<uint64_t>(dense, bcss, m, n, b, bm, nblocks, d_tuples, s);
    return -1;
}

int launch_unpack(int esize, const void *bcss, void *dense, int m, int64_t n, int b, int nbar,
                  const int64_t *d_rank, const int32_t *d_perm, const int32_t *d_pstr, hipStream_t s)
{
    int64_t bm = 1, nbm = 1;
    for (int j = 0; j < m; ++j) { bm *= b; nbm *= nbar; }
    if (bm / b * ((b + 3) / 4) > INT32_MAX / 2) return -1;
    if (esize == 2) return launch_unpack_t<uint16_t>(bcss, dense, m, n, b, nbar, bm, nbm, d_rank, d_perm, d_pstr, s);
    if (esize == 4) return launch_unpack_t<uint32_t>(bcss, dense, m, n, b, nbar, bm, nbm, d_rank, d_perm, d_pstr, s);
    if (esize == 8) return launch_unpack_t<uint64_t>(bcss, dense, m, n, b, nbar, bm, nbm, d_rank, d_perm, d_pstr, s);
    return -1;
}

// ------------------------------------------------------------------ hashed fill
// SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Each BCSS entry gets lo + (hi - lo) u, u = (h >> 40) 2^-24 with
// h = mix(...mix(mix(seed) ^ s_0)... ^ s_{m-1}) over its sorted global index
// s_0 <= ... <= s_{m-1}: a symmetric tensor whose unique entries are
// pseudo-random.  Entries beyond n are zero.
template <class E>
__global__ void bcss_fill_hashed_kernel(E *__restrict__ bcss, int m, int64_t n, int b, int64_t bm, int64_t total,
                                        const int32_t *__restrict__ tuples, uint64_t seed, double lo, double hi)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / bm;
        int64_t l = e - r * bm;
        int64_t idx[kMaxOrder];
        bool ok = true;
        for (int j = 0; j < m; ++j) {
            const int64_t lj = l % b;
            l /= b;
            idx[j] = (int64_t)tuples[r * m + j] * b + lj;
            ok = ok && idx[j] < n;
        }
        double v = 0.0;
        if (ok) {
            for (int j = 1; j < m; ++j) {   // insertion sort
                const int64_t x = idx[j];
                int i = j - 1;
                while (i >= 0 && idx[i] > x) { idx[i + 1] = idx[i]; --i; }
                idx[i + 1] = x;
            }
            uint64_t h = splitmix64(seed);
            for (int j = 0; j < m; ++j) h = splitmix64(h ^ (uint64_t)idx[j]);
            v = lo + (hi - lo) * ((double)(h >> 40) * (1.0 / 16777216.0));
        }
        if constexpr (sizeof(E) == 2) bcss[e] = f2bf((float)v);
        else if constexpr (sizeof(E) == 4) bcss[e] = __float_as_uint((float)v);
        else bcss[e] = (E)__double_as_longlong(v);
    }
}

int launch_fill_hashed(int esize, void *bcss, int m, int64_t n, int b, int64_t nblocks, const int32_t *d_tuples,
                       uint64_t seed, double lo, double hi, hipStream_t s)
{
    int64_t bm = 1;
    for (int j = 0; j < m; ++j) bm *= b;
    const int64_t total = bm * nblocks;
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 1 << 20));
    if (esize == 2)
        hipLaunchKernelGGL(bcss_fill_hashed_kernel<uint16_t>, dim3(blocks), dim3(256), 0, s, (uint16_t *)bcss, m, n,
                           b, bm, total, d_tuples, seed, lo, hi);
    else if (esize == 4)
        hipLaunchKernelGGL(bcss_fill_hashed_kernel<uint32_t>, dim3(blocks), dim3(256), 0, s, (uint32_t *)bcss, m, n,
                           b, bm, total, d_tuples, seed, lo, hi);
    else if (esize == 8)
        hipLaunchKernelGGL(bcss_fill_hashed_kernel<uint64_t>, dim3(blocks), dim3(256), 0, s, (uint64_t *)bcss, m, n,
                           b, bm, total, d_tuples, seed, lo, hi);
    else
        return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------------------------------ X panels
// Xp[j][i] = X(j, i) for j < p, i < n, zero elsewhere; rows of Kx entries.
// Slot 0 fp32, slot 1 bf16(x), slot 2 bf16(x - bf16(x)).
// Transposed fp32 panel: Xt[i][j] = X(j, i), Kt rows of Pt entries.
// xt[i][j] = X[j][i] (zero outside p x n): one 16 x 16 tile per workgroup
// (one entry per thread, so even a 256 x 256 panel spreads over 256
// workgroups), turned around in LDS so that X is read along i and xt written
// along j, both contiguous for a row-major X.
template <class E>
__global__ void prep_xt_kernel(const E *__restrict__ X, int64_t rs, int64_t cs, int64_t p, int64_t n,
                               int64_t Kt, int64_t Pt, float *__restrict__ xt)
{
    __shared__ float t[16][17];
    const int64_t i0 = (int64_t)blockIdx.x * 16, j0 = (int64_t)blockIdx.y * 16;
    const int c = threadIdx.x & 15, r = threadIdx.x >> 4;
    {
        const int64_t j = j0 + r, i = i0 + c;
        float v = 0.f;
        if (j < p && i < n) {
            if constexpr (sizeof(E) == 4) v = __uint_as_float(X[j * rs + i * cs]);
            else v = bf2f(X[j * rs + i * cs]);
        }
        t[r][c] = v;
    }
    __syncthreads();
    const int64_t i = i0 + r, j = j0 + c;
    if (i < Kt && j < Pt) xt[i * Pt + j] = t[c][r];
}

// Eight consecutive entries of a panel row per thread (Kx is a multiple of
// 8): one row index division per eight entries, 16-byte stores of every
// panel, and 16-byte loads of X where its row is contiguous and aligned.
template <class E>
__global__ void prep_x_kernel(const E *__restrict__ X, int64_t rs, int64_t cs, int64_t p, int64_t n,
                              int64_t Ppad, int64_t Kx, float *__restrict__ x32, u16 *__restrict__ xhi,
                              u16 *__restrict__ xlo)
{
    const int64_t total8 = Ppad * Kx / 8;
    for (int64_t e8 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e8 < total8;
         e8 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = e8 * 8, j = e / Kx, i0 = e - j * Kx;
        float v[8];
        const E *src = X + j * rs + i0 * cs;
        if (j < p && i0 + 8 <= n && cs == 1 && ((uintptr_t)src & 15) == 0) {
            if constexpr (sizeof(E) == 4) {
                const float4 a = *(const float4 *)src, b = *(const float4 *)(src + 4);
                v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w, v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
            } else {
                const uint4 w = *(const uint4 *)src;
                const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    v[2 * q] = bf2f((u16)(ww[q] & 0xFFFFu));
                    v[2 * q + 1] = bf2f((u16)(ww[q] >> 16));
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t i = i0 + q;
                v[q] = 0.f;
                if (j < p && i < n) {
                    if constexpr (sizeof(E) == 4) v[q] = __uint_as_float(X[j * rs + i * cs]);
                    else v[q] = bf2f(X[j * rs + i * cs]);
                }
            }
        }
        if (x32) {
            *(float4 *)(x32 + e) = float4{v[0], v[1], v[2], v[3]};
            *(float4 *)(x32 + e + 4) = float4{v[4], v[5], v[6], v[7]};
        }
        if (xhi || xlo) {
            uint32_t hw[4], lw[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const u16 h0 = f2bf(v[2 * q]), h1 = f2bf(v[2 * q + 1]);
                hw[q] = (uint32_t)h0 | ((uint32_t)h1 << 16);
                lw[q] = (uint32_t)f2bf(v[2 * q] - bf2f(h0)) | ((uint32_t)f2bf(v[2 * q + 1] - bf2f(h1)) << 16);
            }
            if (xhi) *(uint4 *)(xhi + e) = uint4{hw[0], hw[1], hw[2], hw[3]};
            if (xlo) *(uint4 *)(xlo + e) = uint4{lw[0], lw[1], lw[2], lw[3]};
        }
    }
}

int launch_prep_xt(int esize, const void *X, int64_t rs, int64_t cs, int64_t p, int64_t n, int64_t Kt, int64_t Pt,
                   float *xt, hipStream_t s)
{
    const int64_t gi = (Kt + 15) / 16, gj = (Pt + 15) / 16;
    if (gi < 1 || gj < 1 || gi > INT32_MAX || gj > 65535) return -1;
    const dim3 grid((unsigned)gi, (unsigned)gj);
    if (esize == 4)
        hipLaunchKernelGGL(prep_xt_kernel<uint32_t>, grid, dim3(256), 0, s, (const uint32_t *)X, rs, cs, p, n, Kt, Pt,
                           xt);
    else if (esize == 2)
        hipLaunchKernelGGL(prep_xt_kernel<uint16_t>, grid, dim3(256), 0, s, (const uint16_t *)X, rs, cs, p, n, Kt, Pt,
                           xt);
    else
        return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prep_x(int esize, const void *X, int64_t rs, int64_t cs, int64_t p, int64_t n, int64_t Ppad,
                  int64_t Kx, float *x32, uint16_t *xhi, uint16_t *xlo, hipStream_t s)
{
    if (Kx % 8 != 0) return -1;
    const int64_t total8 = Ppad * Kx / 8;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((total8 + 255) / 256, 1 << 16));
    if (esize == 4)
        hipLaunchKernelGGL(prep_x_kernel<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s, (const uint32_t *)X,
                           rs, cs, p, n, Ppad, Kx, x32, xhi, xlo);
    else if (esize == 2)
        hipLaunchKernelGGL(prep_x_kernel<uint16_t>, dim3((unsigned)blocks), dim3(256), 0, s, (const uint16_t *)X,
                           rs, cs, p, n, Ppad, Kx, x32, xhi, xlo);
    else
        return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ------------------------------------------------------------------ stage kernel
//
// One workgroup (4 waves) computes an MT x NT tile of one row group's GEMM
//   Out[mm][nn] = sum_k In[mm][k] * X[nn][k],
// where mm runs over the entries of an input block without the contracted
// mode k, nn = jbar*bC + jj over the output C-block index of mode k, and
// k = ibar*bA + lk over the contracted mode.  In[mm][k] is entry (mm, lk) of
// the logical input block (s, ibar), read from the stored block sort(s, ibar)
// through the strides of insertion position q: the permutation is applied
// while staging, so no permuted copy is ever formed.
//
// Both operands are staged in LDS as [row][k] with k contiguous (row stride
// KT + pad), double buffered, with the next chunk's global loads in flight
// while the MFMAs consume the current one.
template <int CMP>
struct CmpTraits;
template <>
struct CmpTraits<CMP_FP32> {
    static constexpr int KT = 16, LROW = 20, VK = 4;   // floats per row, k per vector
    typedef float L;
};
template <>
struct CmpTraits<CMP_BF16> {
    static constexpr int KT = 32, LROW = 40, VK = 8;   // bf16 per row
    typedef u16 L;
};
template <>
struct CmpTraits<CMP_X3> {
    static constexpr int KT = 32, LROW = 40, VK = 8;
    typedef u16 L;
};

// Input blocks per row group whose table the generic tile keeps in LDS
// (larger groups read it from global memory).
constexpr int kGenericTabBlocks = 256;

// LDS of the generic tile.
template <int CMP, int MT, int NT>
struct GenericSmem {
    using L = typename CmpTraits<CMP>::L;
    static constexpr int NL = CMP == CMP_X3 ? 2 : 1;   // LDS planes (hi, lo)
    static constexpr int LROW = CmpTraits<CMP>::LROW;
    __attribute__((aligned(16))) L s_in[NL][2][MT * LROW];
    __attribute__((aligned(16))) L s_x[NL][2][NT * LROW];
    int32_t s_mpart[kMaxOrder][MT];   // input offset of row mm, per insertion position
    int32_t s_opart[MT];              // output offset of row mm (-1: beyond Mblk)
    int64_t s_npart[NT];              // output offset of column nn (-1: beyond N)
    int32_t s_sqk[kMaxOrder];         // stride of the contracted mode, per insertion position
    int64_t s_ioff[kGenericTabBlocks];   // the row group's input table (nbar <= kGenericTabBlocks)
    int32_t s_iq[kGenericTabBlocks];
};

// One MT x NT tile of one row group (see the comment above); used by the
// per-level kernel and by the grouped persistent kernel of the server.
template <int CMP, int MT, int NT, int WM, int WN, bool B_IS_IN>
__device__ __forceinline__ void generic_tile(const StageArgs &a, const Task task, GenericSmem<CMP, MT, NT> &sm)
{
    using Tr = CmpTraits<CMP>;
    constexpr int KT = Tr::KT, LROW = Tr::LROW, VK = Tr::VK;
    constexpr bool SPLIT = CMP == CMP_X3;
    constexpr int NL = SPLIT ? 2 : 1;            // LDS planes (hi, lo)
    constexpr int WTM = MT / WM, WTN = NT / WN;  // wave tile
    constexpr int TM = WTM / 32, TN = WTN / 32;  // 32x32 subtiles per wave
    static_assert(WM * WN == 4 && TM >= 1 && TN >= 1, "tile shape");
    constexpr int IN_VECS = MT * KT / VK;        // vectors of VK k-values per In chunk
    constexpr int X_VECS = NT * KT / VK;
    constexpr int IN_PER_T = (IN_VECS + 255) / 256;
    constexpr int X_PER_T = (X_VECS + 255) / 256;

    auto &s_in = sm.s_in;
    auto &s_x = sm.s_x;
    auto &s_mpart = sm.s_mpart;
    auto &s_opart = sm.s_opart;
    auto &s_npart = sm.s_npart;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const GroupDesc g = a.groups[task.group];
    const int m0 = task.mt * MT, n0 = task.nt * NT;
    const int Nvalid = g.jcount * a.bC;

    // Row and column offset tables of this tile.
    for (int mm = tid; mm < MT; mm += 256) {
        const int mg = m0 + mm;
        if (mg < a.Mblk) {
            int r = mg;
            int dig[kMaxOrder];
            for (int i = 0; i < a.m - 1; ++i) { dig[i] = r % a.mrad[i]; r /= a.mrad[i]; }
            int op = 0;
            for (int i = 0; i < a.m - 1; ++i) op += dig[i] * a.os[a.mmode[i]];
            s_opart[mm] = op;
            for (int q = 0; q <= a.k; ++q) {
                int ip = 0;
                for (int i = 0; i < a.m - 1; ++i) ip += dig[i] * a.sq[q][a.mmode[i]];
                s_mpart[q][mm] = ip;
            }
        } else {
            s_opart[mm] = -1;
            for (int q = 0; q <= a.k; ++q) s_mpart[q][mm] = -1;
        }
    }
    for (int nn = tid; nn < NT; nn += 256) {
        const int ng = n0 + nn;
        if (ng < Nvalid) {
            const int jb = ng / a.bC, jj = ng - jb * a.bC;
            s_npart[nn] = g.out_base + (int64_t)jb * g.out_jstride + (int64_t)jj * a.os[a.k];
        } else {
            s_npart[nn] = -1;
        }
    }
    if (tid <= a.k) sm.s_sqk[tid] = a.sq[tid][a.k];
    const bool tab_lds = a.nbar <= kGenericTabBlocks;
    if (tab_lds)
        for (int i = tid; i < a.nbar; i += 256) {
            const InEntry ie = a.in_tab[g.in_row + i];
            sm.s_ioff[i] = ie.off;
            sm.s_iq[i] = ie.q;
        }

    // Per-thread staging assignment (fixed across chunks).
    // In: vector v -> row mm = v % MT, k-vector kv = v / MT.
    // X : vector v -> row nn = v / (KT/VK), kv = v % (KT/VK).
    float in_f[IN_PER_T][VK];   // staged input values (fp32; bf16 inputs widened)
    f32x4 x_f32[X_PER_T];       // staged X (fp32 compute)
    u16x8 x_hi[X_PER_T], x_lo[X_PER_T];

    // FP32 and split contractions always read fp32 input (the plan checks),
    // so only the bf16 kernel carries the bf16-input load paths.
    const bool in_f32 = CMP == CMP_BF16 ? a.in_f32 != 0 : true;
    const float *in32 = (const float *)a.in;
    const u16 *in16 = (const u16 *)a.in;
    // The row group's input table in global memory (typed so: a read that
    // may come from LDS or from here would otherwise become one flat load,
    // which counts on both wait counters).
    typedef __attribute__((address_space(1))) const InEntry gInEntry;
    gInEntry *row = (gInEntry *)a.in_tab + g.in_row;

    __syncthreads();

    int in_mm[IN_PER_T], in_kv[IN_PER_T];   // row and k vector of each staged input vector
    auto load_chunk = [&](int c) {
        const int blk0 = (c / a.chunks_per_blk) * a.chunk_blocks;
        const int lk0 = (c % a.chunks_per_blk) * a.chunk_k;
        // valid k values of this chunk (a prefix of 0..KT-1)
        int kvalid;
        if (a.chunk_blocks > 1) kvalid = min(a.chunk_blocks, a.nbar - blk0) * a.bA;
        else kvalid = min(a.chunk_k, a.bA - lk0);
        const int kstart = blk0 * a.bA + lk0;
        if (a.chunk_blocks == 1) {
            // The chunk lies inside one input block: one table entry, one
            // permutation and one stride of the contracted mode for all of
            // it.  Threads run along k when the contracted mode is stored
            // fastest, else along the rows, so that neighbouring threads
            // read neighbouring entries either way; whole aligned vectors
            // along k are read as 16-byte loads.
            int64_t ioff;
            int iq;
            if (tab_lds) {
                ioff = sm.s_ioff[blk0];
                iq = sm.s_iq[blk0];
            } else {
                ioff = row[blk0].off;
                iq = row[blk0].q;
            }
            const int sk = sm.s_sqk[iq];
            const bool kfast = sk == 1;
#pragma unroll
            for (int t = 0; t < IN_PER_T; ++t) {
                const int v = tid + t * 256;
                const int mm = kfast ? v / (KT / VK) : v % MT;
                const int kv = kfast ? v % (KT / VK) : v / MT;
                in_mm[t] = mm;
                in_kv[t] = kv;
#pragma unroll
                for (int e = 0; e < VK; ++e) in_f[t][e] = 0.f;
                if (v < IN_VECS && s_mpart[0][mm] >= 0) {
                    const int64_t off = ioff + s_mpart[iq][mm] + (int64_t)(lk0 + kv * VK) * sk;
                    const bool whole = kfast && kv * VK + VK <= kvalid;
                    if (whole && in_f32 && ((uintptr_t)(in32 + off) & 15) == 0) {
#pragma unroll
                        for (int h = 0; h < VK / 4; ++h) {
                            const f32x4 w = *(const f32x4 *)(in32 + off + 4 * h);
#pragma unroll
                            for (int e = 0; e < 4; ++e) in_f[t][4 * h + e] = w[e];
                        }
                    } else if (VK == 8 && whole && !in_f32 && ((uintptr_t)(in16 + off) & 15) == 0) {
                        const u16x8 w = *(const u16x8 *)(in16 + off);
#pragma unroll
                        for (int e = 0; e < VK; ++e) in_f[t][e] = bf2f(w[e & 7]);
                    } else {
#pragma unroll
                        for (int e = 0; e < VK; ++e)
                            if (kv * VK + e < kvalid) {
                                const int64_t o = off + (int64_t)e * sk;
                                in_f[t][e] = in_f32 ? in32[o] : bf2f(in16[o]);
                            }
                    }
                }
            }
        } else if (a.bA % VK == 0) {
            // Several whole blocks per chunk, bA a multiple of VK: a
            // vector's VK k values lie in one block, so it takes one table
            // entry, and one 16-byte load where the contracted mode is
            // stored fastest.  kvalid is a multiple of bA, so a vector is
            // either wholly valid or wholly past the end.
#pragma unroll
            for (int t = 0; t < IN_PER_T; ++t) {
                const int v = tid + t * 256;
                const int mm = v % MT, kv = v / MT;
                in_mm[t] = mm;
                in_kv[t] = kv;
#pragma unroll
                for (int e = 0; e < VK; ++e) in_f[t][e] = 0.f;
                const int kk0 = kv * VK;
                if (v < IN_VECS && s_mpart[0][mm] >= 0 && kk0 < kvalid) {
                    const int gi = kk0 / a.chunk_k;
                    const int lk = lk0 + (kk0 - gi * a.chunk_k);
                    int64_t ioff;
                    int iq;
                    if (tab_lds) {
                        ioff = sm.s_ioff[blk0 + gi];
                        iq = sm.s_iq[blk0 + gi];
                    } else {
                        ioff = row[blk0 + gi].off;
                        iq = row[blk0 + gi].q;
                    }
                    const int sk = sm.s_sqk[iq];
                    const int64_t off = ioff + s_mpart[iq][mm] + (int64_t)lk * sk;
                    if (sk == 1 && in_f32 && ((uintptr_t)(in32 + off) & 15) == 0) {
#pragma unroll
                        for (int h = 0; h < VK / 4; ++h) {
                            const f32x4 w = *(const f32x4 *)(in32 + off + 4 * h);
#pragma unroll
                            for (int e = 0; e < 4; ++e) in_f[t][4 * h + e] = w[e];
                        }
                    } else if (VK == 8 && sk == 1 && !in_f32 && ((uintptr_t)(in16 + off) & 15) == 0) {
                        const u16x8 w = *(const u16x8 *)(in16 + off);
#pragma unroll
                        for (int e = 0; e < VK; ++e) in_f[t][e] = bf2f(w[e & 7]);
                    } else {
#pragma unroll
                        for (int e = 0; e < VK; ++e) {
                            const int64_t o = off + (int64_t)e * sk;
                            in_f[t][e] = in_f32 ? in32[o] : bf2f(in16[o]);
                        }
                    }
                }
            }
        } else if (a.bA % 4 == 0) {
            // Several whole blocks per chunk, bA a multiple of 4 but not of
            // VK (bf16 chunks of b = 4 blocks): each group of 4 k values of
            // a vector lies in one block and takes one table entry, and one
            // 16- or 8-byte load where the contracted mode is stored
            // fastest.  kvalid is a multiple of bA, so a group is either
            // wholly valid or wholly past the end.
#pragma unroll
            for (int t = 0; t < IN_PER_T; ++t) {
                const int v = tid + t * 256;
                const int mm = v % MT, kv = v / MT;
                in_mm[t] = mm;
                in_kv[t] = kv;
#pragma unroll
                for (int e = 0; e < VK; ++e) in_f[t][e] = 0.f;
                if (v < IN_VECS && s_mpart[0][mm] >= 0) {
#pragma unroll
                    for (int h = 0; h < VK / 4; ++h) {
                        const int kk0 = kv * VK + 4 * h;
                        if (kk0 < kvalid) {
                            const int gi = kk0 / a.chunk_k;
                            const int lk = lk0 + (kk0 - gi * a.chunk_k);
                            int64_t ioff;
                            int iq;
                            if (tab_lds) {
                                ioff = sm.s_ioff[blk0 + gi];
                                iq = sm.s_iq[blk0 + gi];
                            } else {
                                ioff = row[blk0 + gi].off;
                                iq = row[blk0 + gi].q;
                            }
                            const int sk = sm.s_sqk[iq];
                            const int64_t off = ioff + s_mpart[iq][mm] + (int64_t)lk * sk;
                            if (sk == 1 && in_f32 && ((uintptr_t)(in32 + off) & 15) == 0) {
                                const f32x4 w = *(const f32x4 *)(in32 + off);
#pragma unroll
                                for (int e = 0; e < 4; ++e) in_f[t][4 * h + e] = w[e];
                            } else if (sk == 1 && !in_f32 && ((uintptr_t)(in16 + off) & 7) == 0) {
                                const u16x4 w = *(const u16x4 *)(in16 + off);
#pragma unroll
                                for (int e = 0; e < 4; ++e) in_f[t][4 * h + e] = bf2f(w[e]);
                            } else {
#pragma unroll
                                for (int e = 0; e < 4; ++e) {
                                    const int64_t o = off + (int64_t)e * sk;
                                    in_f[t][4 * h + e] = in_f32 ? in32[o] : bf2f(in16[o]);
                                }
                            }
                        }
                    }
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < IN_PER_T; ++t) {
                const int v = tid + t * 256;
                const int mm = v % MT, kv = v / MT;
                in_mm[t] = mm;
                in_kv[t] = kv;
#pragma unroll
                for (int e = 0; e < VK; ++e) in_f[t][e] = 0.f;
                if (v < IN_VECS && s_mpart[0][mm] >= 0) {
#pragma unroll
                    for (int e = 0; e < VK; ++e) {
                        const int kk = kv * VK + e;
                        if (kk < kvalid) {
                            const int gi = kk / a.chunk_k;
                            const int lk = lk0 + (kk - gi * a.chunk_k);
                            int64_t ioff;
                            int iq;
                            if (tab_lds) {
                                ioff = sm.s_ioff[blk0 + gi];
                                iq = sm.s_iq[blk0 + gi];
                            } else {
                                ioff = row[blk0 + gi].off;
                                iq = row[blk0 + gi].q;
                            }
                            const int64_t off = ioff + s_mpart[iq][mm] + (int64_t)lk * sm.s_sqk[iq];
                            in_f[t][e] = in_f32 ? in32[off] : bf2f(in16[off]);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < X_PER_T; ++t) {
            const int v = tid + t * 256;
            const int nn = v / (KT / VK), kv = v % (KT / VK);
            const int ng = n0 + nn;
            const bool rowok = v < X_VECS && ng < Nvalid;
            const int64_t base = (int64_t)ng * a.Kx + kstart + kv * VK;
            const bool xwhole = kv * VK + VK <= kvalid;
            if constexpr (CMP == CMP_FP32) {
                const float *xp = (const float *)a.xp;
                f32x4 val = {0.f, 0.f, 0.f, 0.f};
                if (rowok) {
                    if (xwhole && ((uintptr_t)(xp + base) & 15) == 0) {
                        val = *(const f32x4 *)(xp + base);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (kv * 4 + e < kvalid) val[e] = xp[base + e];
                    }
                }
                x_f32[t] = val;
            } else {
                const u16 *xh = (const u16 *)a.xp;
                const u16 *xl = (const u16 *)a.xp_lo;
                u16x8 h = {0, 0, 0, 0, 0, 0, 0, 0}, l = {0, 0, 0, 0, 0, 0, 0, 0};
                if (rowok) {
                    if (xwhole && ((uintptr_t)(xh + base) & 15) == 0 &&
                        (!SPLIT || ((uintptr_t)(xl + base) & 15) == 0)) {
                        h = *(const u16x8 *)(xh + base);
                        if constexpr (SPLIT) l = *(const u16x8 *)(xl + base);
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            if (kv * 8 + e < kvalid) {
                                h[e] = xh[base + e];
                                if constexpr (SPLIT) l[e] = xl[base + e];
                            }
                        }
                    }
                }
                x_hi[t] = h;
                if constexpr (SPLIT) x_lo[t] = l;
            }
        }
    };

    auto store_chunk = [&](int buf) {
#pragma unroll
        for (int t = 0; t < IN_PER_T; ++t) {
            const int v = tid + t * 256;
            if (v >= IN_VECS) break;
            const int mm = in_mm[t], kv = in_kv[t];
            if constexpr (CMP == CMP_FP32) {
                f32x4 val = {in_f[t][0], in_f[t][1], in_f[t][2], in_f[t][3]};
                *(f32x4 *)&s_in[0][buf][mm * LROW + kv * 4] = val;
            } else {
                u16x8 h, l;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float f = in_f[t][e];
                    const u16 hb = f2bf(f);
                    h[e] = hb;
                    if constexpr (SPLIT) l[e] = f2bf(f - bf2f(hb));
                }
                *(u16x8 *)&s_in[0][buf][mm * LROW + kv * 8] = h;
                if constexpr (SPLIT) *(u16x8 *)&s_in[NL - 1][buf][mm * LROW + kv * 8] = l;
            }
        }
#pragma unroll
        for (int t = 0; t < X_PER_T; ++t) {
            const int v = tid + t * 256;
            if (v >= X_VECS) break;
            const int nn = v / (KT / VK), kv = v % (KT / VK);
            if constexpr (CMP == CMP_FP32) {
                *(f32x4 *)&s_x[0][buf][nn * LROW + kv * 4] = x_f32[t];
            } else {
                *(u16x8 *)&s_x[0][buf][nn * LROW + kv * 8] = x_hi[t];
                if constexpr (SPLIT) *(u16x8 *)&s_x[NL - 1][buf][nn * LROW + kv * 8] = x_lo[t];
            }
        }
    };

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int r32 = lane & 31, half = lane >> 5;
    load_chunk(0);
    for (int c = 0; c < a.nchunks; ++c) {
        const int buf = c & 1;
        store_chunk(buf);
        __syncthreads();
        if (c + 1 < a.nchunks) load_chunk(c + 1);
        if constexpr (CMP == CMP_FP32) {
#pragma unroll
            for (int kg = 0; kg < KT / 8; ++kg) {
                f32x4 va[TM], vb[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    va[i] = *(const f32x4 *)&s_in[0][buf][(wm * WTM + i * 32 + r32) * LROW + kg * 8 + half * 4];
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    vb[j] = *(const f32x4 *)&s_x[0][buf][(wn * WTN + j * 32 + r32) * LROW + kg * 8 + half * 4];
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j) {
                            if constexpr (B_IS_IN)
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(vb[j][t], va[i][t], acc[i][j], 0, 0, 0);
                            else
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(va[i][t], vb[j][t], acc[i][j], 0, 0, 0);
                        }
            }
        } else {
#pragma unroll
            for (int kg = 0; kg < KT / 16; ++kg) {
                bf16x8 ha[TM], hb[TN], la[TM], lb[TN];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int o = (wm * WTM + i * 32 + r32) * LROW + kg * 16 + half * 8;
                    ha[i] = __builtin_bit_cast(bf16x8, *(const u16x8 *)&s_in[0][buf][o]);
                    if constexpr (SPLIT) la[i] = __builtin_bit_cast(bf16x8, *(const u16x8 *)&s_in[NL - 1][buf][o]);
                }
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    const int o = (wn * WTN + j * 32 + r32) * LROW + kg * 16 + half * 8;
                    hb[j] = __builtin_bit_cast(bf16x8, *(const u16x8 *)&s_x[0][buf][o]);
                    if constexpr (SPLIT) lb[j] = __builtin_bit_cast(bf16x8, *(const u16x8 *)&s_x[NL - 1][buf][o]);
                }
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        if constexpr (B_IS_IN) {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hb[j], ha[i], acc[i][j], 0, 0, 0);
                            if constexpr (SPLIT) {
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lb[j], ha[i], acc[i][j], 0, 0, 0);
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(hb[j], la[i], acc[i][j], 0, 0, 0);
                            }
                        } else {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha[i], hb[j], acc[i][j], 0, 0, 0);
                            if constexpr (SPLIT) {
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ha[i], lb[j], acc[i][j], 0, 0, 0);
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(la[i], hb[j], acc[i][j], 0, 0, 0);
                            }
                        }
                    }
            }
        }
    }

    // Epilogue: D[row][col] of a 32x32 subtile sits in lane col = lane%32,
    // register r at row 8*(r/4) + 4*(lane/32) + r%4.
    float *out32 = (float *)a.out;
    u16 *out16 = (u16 *)a.out;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int rowi = 8 * (r >> 2) + 4 * half + (r & 3);
                int mm, nn;
                if constexpr (B_IS_IN) {
                    mm = wm * WTM + i * 32 + r32;
                    nn = wn * WTN + j * 32 + rowi;
                } else {
                    mm = wm * WTM + i * 32 + rowi;
                    nn = wn * WTN + j * 32 + r32;
                }
                const int op = s_opart[mm];
                const int64_t np = s_npart[nn];
                if (op >= 0 && np >= 0) {
                    const int64_t o = np + op;
                    if (a.out_f32) out32[o] = a.accumulate ? out32[o] + acc[i][j][r] : acc[i][j][r];
                    else out16[o] = f2bf(acc[i][j][r]);
                }
            }
}

// bf16 tiles of up to 128 rows: at most 128 VGPRs, so that four workgroups
// fit per CU as for FP32 (the tile is latency-bound: m6_n24_b4 bf16 ran at
// three per CU with 138); 256-row tiles are held to two by their LDS.
template <int CMP, int MT, int NT, int WM, int WN, bool B_IS_IN, bool FIRST>
__global__ __launch_bounds__(256, CMP == CMP_BF16 && MT <= 128 ? 4 : 1) void stage_kernel(const StageArgs a)
{
    __shared__ GenericSmem<CMP, MT, NT> sm;
    generic_tile<CMP, MT, NT, WM, WN, B_IS_IN>(a, a.tasks[blockIdx.x], sm);
}

// Grouped persistent kernel: one launch runs the tasks of many (request,
// level) stages, each task naming its stage's arguments.  Workgroups take
// tasks from a shared queue (an atomic counter) until it is empty; tasks of
// one launch never depend on each other, so no workgroup ever waits.
template <int CMP, int MT, int NT, int WM, int WN>
__global__ __launch_bounds__(256) void grouped_kernel(const StageArgs *__restrict__ stages,
                                                      const GroupedTask *__restrict__ tasks, int ntasks,
                                                      int *__restrict__ queue_head)
{
    __shared__ GenericSmem<CMP, MT, NT> sm;
    __shared__ int s_t;
    for (;;) {
        if (threadIdx.x == 0) s_t = atomicAdd(queue_head, 1);
        __syncthreads();
        const int t = s_t;
        __syncthreads();   // every thread has read s_t before it is reused
        if (t >= ntasks) break;
        const GroupedTask gt = tasks[t];
        const StageArgs &a = stages[gt.stage];
        const Task task{gt.group, gt.mt, gt.nt};
        if (a.k != 0) generic_tile<CMP, MT, NT, WM, WN, true>(a, task, sm);
        else generic_tile<CMP, MT, NT, WM, WN, false>(a, task, sm);
        __syncthreads();   // LDS is reused by the next task
    }
}

int launch_grouped(int compute, const StageArgs *d_stages, const GroupedTask *d_tasks, int ntasks, int *d_head,
                   int grid, hipStream_t s)
{
    if (ntasks <= 0) return 0;
    const dim3 g((unsigned)std::max(1, std::min(grid, ntasks))), b(256);
    if (compute == CMP_FP32)
        hipLaunchKernelGGL((grouped_kernel<CMP_FP32, kGroupedMT, kGroupedNT, 2, 2>), g, b, 0, s, d_stages, d_tasks,
                           ntasks, d_head);
    else if (compute == CMP_BF16)
        hipLaunchKernelGGL((grouped_kernel<CMP_BF16, kGroupedMT, kGroupedNT, 2, 2>), g, b, 0, s, d_stages, d_tasks,
                           ntasks, d_head);
    else if (compute == CMP_X3)
        hipLaunchKernelGGL((grouped_kernel<CMP_X3, kGroupedMT, kGroupedNT, 2, 2>), g, b, 0, s, d_stages, d_tasks,
                           ntasks, d_head);
    else
        return -1;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// FIRST marks the level that reads A; it is a separate instantiation so that
// profilers report the first contraction on its own.
template <int CMP, bool B_IS_IN, bool FIRST>
static int launch_stage_cmp(const StageArgs &a, int MT, int NT, hipStream_t s)
{
    const dim3 grid((unsigned)a.ntasks), block(256);
    if (NT == 32) {   // narrow groups (few output columns): four waves along the rows
        switch (MT) {
        case 256: hipLaunchKernelGGL((stage_kernel<CMP, 256, 32, 4, 1, B_IS_IN, FIRST>), grid, block, 0, s, a); break;
        case 128: hipLaunchKernelGGL((stage_kernel<CMP, 128, 32, 4, 1, B_IS_IN, FIRST>), grid, block, 0, s, a); break;
        default: return -1;
        }
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    switch (MT) {
    case 256: hipLaunchKernelGGL((stage_kernel<CMP, 256, 64, 4, 1, B_IS_IN, FIRST>), grid, block, 0, s, a); break;
    case 128: hipLaunchKernelGGL((stage_kernel<CMP, 128, 64, 2, 2, B_IS_IN, FIRST>), grid, block, 0, s, a); break;
    case 64: hipLaunchKernelGGL((stage_kernel<CMP, 64, 64, 2, 2, B_IS_IN, FIRST>), grid, block, 0, s, a); break;
    case 32: hipLaunchKernelGGL((stage_kernel<CMP, 32, 128, 1, 4, B_IS_IN, FIRST>), grid, block, 0, s, a); break;
    default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int CMP>
static int launch_stage_c(const StageArgs &a, int MT, int NT, bool first, hipStream_t s)
{
    const bool b_in = a.k != 0;   // output contiguous along the block rows unless mode 0 is contracted
    if (first)
        return b_in ? launch_stage_cmp<CMP, true, true>(a, MT, NT, s) : launch_stage_cmp<CMP, false, true>(a, MT, NT, s);
    return b_in ? launch_stage_cmp<CMP, true, false>(a, MT, NT, s) : launch_stage_cmp<CMP, false, false>(a, MT, NT, s);
}

int launch_stage(const StageArgs &a, int compute, int MT, int NT, bool first, hipStream_t s)
{
    if (a.ntasks <= 0) return 0;
    if (compute == CMP_FP32) return launch_stage_c<CMP_FP32>(a, MT, NT, first, s);
    if (compute == CMP_BF16) return launch_stage_c<CMP_BF16>(a, MT, NT, first, s);
    if (compute == CMP_X3) {   // the split form only ever runs the first level
        if (!first) return -1;
        return a.k != 0 ? launch_stage_cmp<CMP_X3, true, true>(a, MT, NT, s)
                        : launch_stage_cmp<CMP_X3, false, true>(a, MT, NT, s);
    }
    return -1;
}

// ------------------------------------------------------------------ fast stage kernel
//
// Same tile contract as stage_kernel, specialised to the shapes the measured
// workloads take: an input block has exactly 256 entries per value of the
// contracted index and bA divides 16, so one K chunk of 16 is G = 16/bA whole
// input blocks.  A tile covers either the whole block row (MT = 256) or, for
// levels below the first, half of it split along mode m-1: that mode lies
// outside the symmetric group, is never permuted and is the slowest in
// storage, so the half is contiguous in every stored block.
//
// Each stored block (or half) is read with contiguous float4 loads in
// storage order (coalesced for every permutation) and scattered into LDS in
// the canonical [k][m] layout: reading a non-stored block costs nothing but
// a different set of LDS strides, chosen per block by its insertion position
// q (the same for the whole workgroup).  Rows of MT + 4 floats keep the
// scatter and the MFMA operand reads free of bank conflicts.  X comes from a
// transposed, zero-padded panel [k][n], so its loads need no bounds checks.
// A chunk's global loads go out PD chunks ahead of its MFMAs into one of PD
// register sets; with PD = 1 a chunk is written to LDS between two MFMA
// phases, with PD >= 2 in the middle of the previous chunk's MFMAs (the
// other LDS buffer).  The block table entries a load needs are read one
// chunk before it, so nothing waits on LDS inside the MFMA loop.  Every thread
// holds its LDS scatter address for each insertion position q < M, and picks
// one with a wave-uniform select: staging reads no kernel argument and no
// table in the loop.  The order M is a template parameter so that every digit
// loop unrolls.
constexpr int kFastMaxBlocks = 512;   // input blocks per group the LDS table holds

// f(integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time.
template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Is...>)
{
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <int M, int MT, int NT, int KT, int PD, bool B_IS_IN, bool FIRST>
__global__ __launch_bounds__(256, 2) void stage_fast_f32(const StageArgs a)
{
    constexpr int RS = MT + 4, XS = NT + 4;
    // Last level (mode 0 contracted, B_IS_IN false): the contracted mode is
    // stored fastest in every block, so chunks are staged [row][k] (row
    // stride RSK) with 16-byte writes, and each lane reads its 8 k values
    // of a chunk with two 16-byte reads; the k pair t of the MFMA takes
    // k = t (lanes 0-31) and t + 8 (lanes 32-63), X the same.
    constexpr bool KMK = !B_IS_IN;
    constexpr int RSK = KT + 4;
    // The four waves split the tile along M and each covers every column,
    // so a tile with fewer valid columns shortens all four waves alike (each
    // wave runs on its own SIMD: no SIMD idles while another has work).
    constexpr int WTM = MT / 4, TM = WTM / 32, TN = NT / 32;
    constexpr int NF = MT * KT / 1024;                 // float4 of In per thread per chunk
    constexpr int XV = NT * KT / 4;                    // float4 of X per chunk
    constexpr int XF = (XV + 255) / 256;               // ... per thread
    static_assert(TM >= 1 && TN >= 1 && NF >= 1, "tile");
    static_assert(KMK || 2 * KT * RS >= 4 * 1024, "epilogue staging fits the input buffers");
    __shared__ __attribute__((aligned(16))) float s_in[2][KMK ? MT * RSK : KT * RS];
    __shared__ __attribute__((aligned(16))) float s_x[2][KT * XS];
    __shared__ int32_t s_opart[MT];
    __shared__ int64_t s_npart[NT];
    __shared__ int64_t s_ioff[kFastMaxBlocks];
    __shared__ int32_t s_iq[kFastMaxBlocks];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave;
    const Task task = a.tasks[blockIdx.x];
    const GroupDesc g = a.groups[task.group];
    const int n0 = task.nt * NT + task.noff;
    const int ncol = task.ncol;   // valid columns from n0 (<= NT)
    const int k = a.k, bA = a.bA, nbar = a.nbar, G = a.chunk_blocks;
    const int sub4 = MT * bA / 4;                      // float4 per block part (>= 256)
    const float *in = (const float *)a.in;
    const float *xt = (const float *)a.xp;
    const int64_t xs = a.xt_stride;
    const bool xdir = a.x_direct != 0;
    const int64_t xrs = a.x_rs;
    const int xp_rows = a.x_p, xp_cols = a.x_n;

    for (int i = tid; i < nbar; i += 256) {
        const InEntry ie = a.in_tab[g.in_row + i];
        s_ioff[i] = ie.off;
        s_iq[i] = ie.q;
    }
    for (int mm = tid; mm < MT; mm += 256) s_opart[mm] = a.fopart[task.mt * MT + mm];
    for (int nn = tid; nn < NT; nn += 256) {
        const int ng = n0 + nn;
        if (nn < ncol) {
            const int jb = ng / a.bC, jj = ng - jb * a.bC;
            s_npart[nn] = g.out_base + (int64_t)jb * g.out_jstride + (int64_t)jj * a.osk;
        } else {
            s_npart[nn] = -1;
        }
    }
    // Offset of this thread's float4 inside the block, and its chunk block
    // (uniform: a block part holds >= 256 float4).
    int gq[NF], o4[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const int F = tid + 256 * f;
        gq[f] = (256 * f) / sub4;
        o4[f] = task.mt * MT * bA + 4 * (F - gq[f] * sub4);
    }
    // LDS address of this thread's float4 for every insertion position q
    // (rows of this M tile start at 0), from its stored digits (host table,
    // per M tile).  A register vector: the wave-uniform q indexes it without
    // going through memory.
    static_assert(M <= 8, "order");
    using AdVec = typename std::conditional<M <= 4, i32x4, i32x8>::type;
    AdVec adq[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        adq[f] = AdVec{};
        int dg[M];
#pragma unroll
        for (int i = 0; i < M; ++i) dg[i] = a.fdig[((task.mt * NF + f) * M + i) * 256 + tid];
        if constexpr (KMK) {
            int row = -task.mt * MT;   // stored positions 1.. hold the row modes (q = 0)
#pragma unroll
            for (int i = 1; i < M; ++i) row += dg[i] * a.lds[0][i];
            adq[f][0] = row * RSK + gq[f] * bA + dg[0];
        } else {
#pragma unroll
            for (int q = 0; q < M; ++q) {
                int ad = gq[f] * bA * RS - task.mt * MT;
#pragma unroll
                for (int i = 0; i < M; ++i) ad += dg[i] * a.lds[q][i];
                adq[f][q] = ad;
            }
        }
    }
    __syncthreads();

    // Table entries (block offset, q) of the chunk to be loaded next; a
    // block past nbar (a partial last chunk, or a chunk past the last) reads
    // the zero block, staged like a block with q = k.
    const int64_t zoff = a.zero_blk - in;
    // All of a thread's float4 of a chunk lie in one block when a block part
    // holds every float4 of the chunk (bA = KT): one table entry, one q.
    const bool one_block = gq[NF - 1] == 0;
    int64_t toff[NF];
    int tq[NF];
    auto read_tab = [&](int c) {
        if (one_block) {
            const int ib = c * G;
            const int ibc = ib < nbar ? ib : nbar - 1;
            const int64_t o = s_ioff[ibc];
            const int q = s_iq[ibc];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                toff[f] = ib < nbar ? o : zoff;
                tq[f] = ib < nbar ? q : k;
            }
            return;
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int ib = c * G + gq[f];
            const int ibc = ib < nbar ? ib : nbar - 1;
            const int64_t o = s_ioff[ibc];
            const int q = s_iq[ibc];
            toff[f] = ib < nbar ? o : zoff;
            tq[f] = ib < nbar ? q : k;
        }
    };
    // PD register sets of loaded chunks: chunk c is loaded into set c % PD,
    // PD chunks before its MFMAs.  With PD = 2 the loads past the last chunk
    // re-read it (never stored) so that every load is unconditional and the
    // wait before a store covers only the older set.
    using I0 = std::integral_constant<int, 0>;
    f32x4 rin[PD][NF], rx[PD][XF];
    int rq[PD][NF];
    const int nch = a.nchunks;
    auto load_chunk = [&](auto S, int c) {
        constexpr int st = decltype(S)::value;
        const int cx = c < nch ? c : nch - 1;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            rq[st][f] = tq[f];
            rin[st][f] = *(const f32x4 *)(in + toff[f] + o4[f]);
        }
#pragma unroll
        for (int f = 0; f < XF; ++f) {
            const int v = tid + 256 * f;
            if (xdir) {
                // X itself: column n0 + xn of the tile is row n0 + xn of X,
                // four consecutive k of it per float4 (zero past p and n)
                const int xn = v / (KT / 4), xk = (v % (KT / 4)) * 4;
                const int row = n0 + xn, kk = cx * KT + xk;
                const bool ok = v < XV && row < xp_rows && kk < xp_cols;
                rx[st][f] = *(const f32x4 *)(xt + (ok ? (int64_t)row * xrs + kk : 0));
                if (!ok) rx[st][f] = f32x4{0.f, 0.f, 0.f, 0.f};
            } else {
                const int xk = v / (NT / 4), xn = (v % (NT / 4)) * 4;
                const int xc = xn < ncol ? xn : 0;   // columns past the tile are never used: stay in bounds
                if (v < XV) rx[st][f] = *(const f32x4 *)(xt + (int64_t)(cx * KT + xk) * xs + n0 + xc);
            }
        }
        read_tab(c + 1);
    };
    auto store_chunk = [&](int buf, auto S) {
        constexpr int st = decltype(S)::value;
        float *si = s_in[buf];
        if (one_block) {
            const int qs = __builtin_amdgcn_readfirstlane(rq[st][0]);
            if (KMK || qs != 0) {
#pragma unroll
                for (int f = 0; f < NF; ++f) *(f32x4 *)&si[adq[f][qs]] = rin[st][f];
            } else {
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const int ad = adq[f][0];
                    si[ad] = rin[st][f][0];
                    si[ad + RS] = rin[st][f][1];
                    si[ad + 2 * RS] = rin[st][f][2];
                    si[ad + 3 * RS] = rin[st][f][3];
                }
            }
        } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const int qs = __builtin_amdgcn_readfirstlane(rq[st][f]);   // the same for the whole workgroup
            const int ad = adq[f][qs];
            const f32x4 v = rin[st][f];
            // stored position 0 is the contracted mode (LDS stride RS) when
            // q = 0, else mode 0 (stride 1: the float4 stays one LDS row)
            if (KMK || qs != 0) {
                *(f32x4 *)&si[ad] = v;
            } else {
                si[ad] = v[0];
                si[ad + RS] = v[1];
                si[ad + 2 * RS] = v[2];
                si[ad + 3 * RS] = v[3];
            }
        }
        }
#pragma unroll
        for (int f = 0; f < XF; ++f) {
            const int v = tid + 256 * f;
            if (xdir) {   // four k rows of one column
                const int xn = v / (KT / 4), xk = (v % (KT / 4)) * 4;
                if (v < XV) {
                    s_x[buf][xk * XS + xn] = rx[st][f][0];
                    s_x[buf][(xk + 1) * XS + xn] = rx[st][f][1];
                    s_x[buf][(xk + 2) * XS + xn] = rx[st][f][2];
                    s_x[buf][(xk + 3) * XS + xn] = rx[st][f][3];
                }
            } else {
                const int xk = v / (NT / 4), xn = (v % (NT / 4)) * 4;
                if (v < XV) *(f32x4 *)&s_x[buf][xk * XS + xn] = rx[st][f];
            }
        }
    };

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int r32 = lane & 31, half = lane >> 5;
    const int arow = wm * WTM + r32;         // this lane's M row in subtile 0
    const int xcol = r32;                    // this lane's N column in subtile 0

    // MFMAs of one chunk with the operands of the next k pair read from LDS
    // before the current MFMAs issue; the global loads of chunk c + PD go
    // out after the first MFMA group, behind work already queued on the pipe.
    auto mfma_chunk = [&](int buf, int c, auto S, auto O) {
        const float *si = s_in[buf];
        const float *sx = s_x[buf];
        float va[2][TM], vb[2][TN];
        f32x4 vk[TM][KT / 8];   // KMK: this lane's k values t + 8 * half, t = 0 .. KT/2 - 1
        auto rd = [&](int t, int sl) {
            const int kk = KMK ? t + (KT / 2) * half : 2 * t + half;
            if constexpr (!KMK) {
#pragma unroll
                for (int i = 0; i < TM; ++i) va[sl][i] = si[kk * RS + arow + 32 * i];
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) vb[sl][j] = sx[kk * XS + xcol + 32 * j];
        };
        auto mf = [&](int sl, int t) {
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
                    if (j > 0 && 32 * j >= ncol) continue;   // 32-column subtile past the tile
                    if constexpr (B_IS_IN)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(vb[sl][j], va[sl][i], acc[i][j], 0, 0, 0);
                    else if constexpr (KMK)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(vk[i][t / 4][t % 4], vb[sl][j], acc[i][j], 0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(va[sl][i], vb[sl][j], acc[i][j], 0, 0, 0);
                }
        };
        const bool live = c < nch;   // c = nch: the padding half of the last pair
        if (live) {
            if constexpr (KMK) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int h = 0; h < KT / 8; ++h)
                        vk[i][h] = *(const f32x4 *)&si[(arow + 32 * i) * RSK + (KT / 2) * half + 4 * h];
            }
            rd(0, 0);
        }
#pragma unroll
        for (int t = 0; t < KT / 2; ++t) {
            if (live) {
                if (t + 1 < KT / 2) rd(t + 1, (t + 1) & 1);
                mf(t & 1, t);
            }
            if (t == 0) {
                if constexpr (PD == 1) {
                    if (c + 1 < nch) load_chunk(S, c + 1);
                } else {
                    load_chunk(S, c + PD);
                }
            }
            // PD >= 2: chunk c + 1 (set O, loaded PD - 1 chunks ago) goes
            // into the other LDS buffer while this wave's MFMAs drain; that
            // buffer was last read before the barrier that opened this chunk.
            if constexpr (PD >= 2)
                if (t == KT / 4) store_chunk(buf ^ 1, O);
        }
    };

    read_tab(0);
    if constexpr (PD == 1) {
        load_chunk(I0{}, 0);
        for (int c = 0; c < nch; ++c) {
            store_chunk(c & 1, I0{});
            __syncthreads();
            mfma_chunk(c & 1, c, I0{}, I0{});
        }
    } else {
        static_for<PD>([&](auto I) { load_chunk(I, (int)decltype(I)::value); });
        store_chunk(0, I0{});
        __syncthreads();
        // Chunks go in groups of PD; past the last chunk a group runs no
        // MFMA, so that no load, store or barrier sits behind a branch
        // (chunks past the last are staged and never read).
        for (int c = 0; c < nch; c += PD) {
            static_for<PD>([&](auto I) {
                constexpr int i = decltype(I)::value;
                mfma_chunk((c + i) & 1, c + i, I, std::integral_constant<int, (i + 1) % PD>{});
                __syncthreads();
            });
        }
    }

    float *out = (float *)a.out;
    if constexpr (B_IS_IN) {
        // Output rows (mm) run along mode 0 of the output block, stride 1 in
        // groups of four (mode 0 is not contracted here and its extent is a
        // multiple of 4).  Each wave turns a 32 x 32 subtile around in LDS
        // ([nn][mm], its own 4 KB of the staging buffer) so that every lane
        // stores four consecutive entries with one 16-byte write.
        __syncthreads();   // every wave is past its last read of the staging buffers
        float *so = &s_in[0][0] + wave * 1024;
        const int rr = lane >> 3, c4 = 4 * (lane & 7);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if (j > 0 && 32 * j >= ncol) continue;
#pragma unroll
                for (int r = 0; r < 16; ++r) so[(8 * (r >> 2) + 4 * half + (r & 3)) * 32 + r32] = acc[i][j][r];
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int p4 = 0; p4 < 4; ++p4) {
                    const int nl = rr + 8 * p4;
                    const f32x4 v = *(const f32x4 *)&so[nl * 32 + c4];
                    const int64_t np = s_npart[j * 32 + nl];
                    if (np >= 0) *(f32x4 *)&out[np + s_opart[wm * WTM + i * 32 + c4]] = v;
                }
                __builtin_amdgcn_wave_barrier();
            }
    } else {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if (j > 0 && 32 * j >= ncol) continue;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int mm = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                    const int64_t np = s_npart[j * 32 + r32];
                    if (np >= 0) out[np + s_opart[mm]] = acc[i][j][r];
                }
            }
    }
}

template <int M, int MT, int NT, int KT, int PD>
static void launch_fast_t(const StageArgs &a, bool first, hipStream_t s)
{
    const dim3 grid((unsigned)a.ntasks), block(256);
    if (a.k != 0) {
        if (first) hipLaunchKernelGGL((stage_fast_f32<M, MT, NT, KT, PD, true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((stage_fast_f32<M, MT, NT, KT, PD, true, false>), grid, block, 0, s, a);
    } else {
        if (first) hipLaunchKernelGGL((stage_fast_f32<M, MT, NT, KT, PD, false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((stage_fast_f32<M, MT, NT, KT, PD, false, false>), grid, block, 0, s, a);
    }
}

// Tile shapes of the block-copy kernel (MT x NT, K chunk KT, prefetch depth PD).
#define STTSM_FAST_TILES(X) X(256, 64, 16, 1) X(256, 128, 16, 1) X(256, 32, 16, 1) X(128, 64, 16, 1) \
    X(128, 128, 16, 1) X(128, 64, 32, 1) X(256, 64, 16, 2) X(128, 128, 16, 2) X(128, 64, 16, 2) X(128, 128, 16, 3) \
    X(128, 64, 16, 3) X(128, 64, 16, 4) X(128, 32, 16, 1) X(128, 32, 16, 2)

template <int M>
static int launch_fast_m(const StageArgs &a, int MT, int NT, int KT, int PD, bool first, hipStream_t s)
{
#define STTSM_TRY(mt, nt, kt, pd) \
    if (MT == mt && NT == nt && KT == kt && PD == pd) { launch_fast_t<M, mt, nt, kt, pd>(a, first, s); return 0; }
    STTSM_FAST_TILES(STTSM_TRY)
#undef STTSM_TRY
    return -1;
}

bool fast_supported(int m, int nbar) { return (m == 3 || m == 5) && nbar >= 1 && nbar <= kFastMaxBlocks; }

bool fast_tile_supported(int MT, int NT, int KT, int PD)
{
#define STTSM_HAS(mt, nt, kt, pd) if (MT == mt && NT == nt && KT == kt && PD == pd) return true;
    STTSM_FAST_TILES(STTSM_HAS)
#undef STTSM_HAS
    return false;
}

int launch_stage_fast(const StageArgs &a, int MT, int NT, int KT, int PD, bool first, hipStream_t s)
{
    if (a.ntasks <= 0) return 0;
    if (!fast_supported(a.m, a.nbar)) return -1;
    const int rc = a.m == 3 ? launch_fast_m<3>(a, MT, NT, KT, PD, first, s) : launch_fast_m<5>(a, MT, NT, KT, PD, first, s);
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace symt
