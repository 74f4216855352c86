// In-place symmetrisation of a BCSS tensor (the post-processing step the
// paper suggests at the end of §5.4): an entry of a stored block whose block
// indices repeat is computed once per position, so mirrored entries inside
// the block can differ by rounding; each is replaced by the average over the
// block's stabiliser (the permutations of modes with equal block index).
// Blocks with distinct block indices are already the unique copy of their
// entries and are left as they are.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// One workgroup per stored block (grid-stride).  The orbit of entry l under
// the stabiliser is processed by the thread whose l is the smallest in the
// orbit: it sums the orbit (stabiliser order, identity first), divides by the
// stabiliser's size and writes the average back to every member.  Orbits are
// disjoint, so no two threads touch the same entry.
template <class E>
__global__ void bcss_symmetrize_kernel(E *__restrict__ bcss, int m, int b, int64_t bm, int64_t nblocks,
                                       const int32_t *__restrict__ tuples, const int32_t *__restrict__ stab_start,
                                       const uint8_t *__restrict__ stab_perm)
{
    using Acc = SymAcc<E>;
    using T = typename Acc::T;
    for (int64_t r = blockIdx.x; r < nblocks; r += gridDim.x) {
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

template <class E>
int launch_sym_t(void *bcss, int m, int b, int64_t bm, int64_t nblocks, const int32_t *tuples,
                 const int32_t *stab_start, const uint8_t *stab_perm, hipStream_t s)
{
    const int64_t grid = std::min<int64_t>(std::max<int64_t>(nblocks, 1), 1 << 16);
    hipLaunchKernelGGL(bcss_symmetrize_kernel<E>, dim3((unsigned)grid), dim3(256), 0, s, (E *)bcss, m, b, bm, nblocks,
                       tuples, stab_start, stab_perm);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

int launch_symmetrize(int dtype, void *bcss, int m, int b, int64_t nblocks, const int32_t *d_tuples,
                      const int32_t *d_stab_start, const uint8_t *d_stab_perm, hipStream_t s)
{
    int64_t bm = 1;
    for (int j = 0; j < m; ++j) bm *= b;
    if (bm > INT32_MAX) return -1;
    if (nblocks <= 0) return 0;
    if (dtype == F32) return launch_sym_t<float>(bcss, m, b, bm, nblocks, d_tuples, d_stab_start, d_stab_perm, s);
    if (dtype == BF16) return launch_sym_t<uint16_t>(bcss, m, b, bm, nblocks, d_tuples, d_stab_start, d_stab_perm, s);
    if (dtype == F64) return launch_sym_t<double>(bcss, m, b, bm, nblocks, d_tuples, d_stab_start, d_stab_perm, s);
    return -1;
}

}  // namespace symt
