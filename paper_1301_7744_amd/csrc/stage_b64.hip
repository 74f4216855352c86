// bf16 stage kernel for order 2 with 64 x 64 blocks (bA = bC = 64): one
// level of the algorithm-by-blocks for m = 2 (the figure of §4 for
// C := X A X^T; Fig. mD with m = 2), bf16 operands, fp32 MFMA accumulation
// (v_mfma_f32_32x32x16_bf16).
//
// A row group's GEMM here has 64 rows (one block row), K = nbar * 64 and
// N = jcount * 64 columns; with blocks this large the level is a plain
// dense contraction, so a workgroup takes a 256-row tile made of four
// consecutive row groups (one wave pair each) and NT columns:
//   Out[row][nn] = sum_kk In[row][kk] * X[nn][kk].
// Every K chunk is one whole stored block per row group (8 KB, read as
// contiguous 16-byte vectors in stored order); a block whose contracted mode
// is stored fastest is staged [row][kk], the other orientation [kk][row]
// (the two permutations of §5.3 for m = 2), and MFMA operands come from the
// first with plain 16-byte reads and from the second with ds_read_b64_tr_b16
// (transposing 4 x 4 groups of 16-bit entries on the way out).  X comes from
// the zero-padded bf16 panel [Ppad][Kx] into LDS [nn][kk].
//
// Eight waves: wave w computes rows 64 (w % 4) .. + 63 (its row group) and
// columns NT/2 (w / 4) .. + NT/2 - 1.  Two K chunks are in flight in
// registers while the MFMAs consume the chunk staged in LDS (double
// buffered; one barrier per chunk).  The tile's input-table entries are
// copied to LDS once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace symt {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kB = 64;              // block size (entries per mode)
constexpr int kRowGroups = 4;       // row groups per tile (MT = 256)
constexpr int kStr = kB + 8;        // LDS row stride (bf16) of every staged panel
constexpr int kRegion = kB * kStr;  // one row group's staged block
constexpr int kMaxNbar = 128;       // K <= 8192

template <int NT>
struct B64Smem {
    __attribute__((aligned(16))) u16 a[2][kRowGroups][kRegion];
    __attribute__((aligned(16))) u16 x[2][NT * kStr];
    int64_t off[kRowGroups][kMaxNbar];   // element offset of each input block
    uint8_t kfast[kRowGroups][kMaxNbar]; // 1: contracted mode stored fastest ([row][kk])
};

__device__ __forceinline__ u16 to_bf16(float f)
{
    return __builtin_bit_cast(u16, (__bf16)f);   // round to nearest even (v_cvt)
}

// ROWS_LANE: the output is contiguous along the rows (the M index), so the
// MFMA takes X as its first operand and each lane holds one row; otherwise
// it is contiguous along the columns and each lane holds one column.
template <int K, int NT, bool ROWS_LANE>
__global__ __launch_bounds__(512, 1) void stage_b64_bf16(const StageArgs a)
{
    constexpr int TN = NT / 64;       // 32-column subtiles per wave
    constexpr int XV = NT * 8 / 512;  // X vectors per thread per chunk
    __shared__ B64Smem<NT> sm;
    const Task tk = a.tasks[blockIdx.x];
    const int g0 = tk.group, ngr = tk.mt, n0 = tk.nt * NT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rg = wave & 3, chalf = wave >> 2;
    const int r32 = lane & 31, half = lane >> 5;
    const int grp = lane >> 4, gl = lane & 15;
    const int nbar = a.nbar;
    const u16 *in = (const u16 *)a.in;
    const u16 *xp = (const u16 *)a.xp;
    const int64_t Kx = a.Kx, Ppad = a.Ppad;
    // Which stored position holds the contracted mode, per insertion position.
    const bool kf0 = a.sq[0][K] == 1, kf1 = a.sq[1][K] == 1;

    for (int e = tid; e < kRowGroups * nbar; e += 512) {
        const int r = e / nbar, ib = e - r * nbar;
        int64_t off = 0;
        uint8_t kf = 1;
        if (r < ngr) {
            const InEntry ie = a.in_tab[a.groups[g0 + r].in_row + ib];
            off = ie.off;
            kf = (ie.q == 0 ? kf0 : kf1) ? 1 : 0;
        }
        sm.off[r][ib] = off;
        sm.kfast[r][ib] = kf;
    }
    const bool wave_on = rg < ngr;
    const GroupDesc gd = a.groups[g0 + (wave_on ? rg : 0)];
    const int Nvalid = wave_on ? gd.jcount * kB : 0;
    const int wcol0 = n0 + chalf * (NT / 2);   // first column of this wave
    __syncthreads();

    u32x4 ra[2][kRowGroups], rx[2][XV];
    // Chunk c (clamped to a valid chunk) into register set s: every load is
    // unconditional, so the waits are per register set.
    auto gload = [&](int c, int s) {
#pragma unroll
        for (int r = 0; r < kRowGroups; ++r) {
            const int64_t off = sm.off[r < ngr ? r : 0][c];
            ra[s][r] = *(const u32x4 *)(in + off + (int64_t)tid * 8);
        }
#pragma unroll
        for (int f = 0; f < XV; ++f) {
            const int v = tid + 512 * f;
            const int64_t row = n0 + (v >> 3);
            const int64_t go = (row < Ppad ? row : 0) * Kx + (int64_t)c * kB + (v & 7) * 8;
            rx[s][f] = *(const u32x4 *)(xp + go);
            if (row >= Ppad) rx[s][f] = u32x4{0u, 0u, 0u, 0u};
        }
    };
    // The block's 64 stored rows of 64 entries each go to LDS rows of kStr:
    // [row][kk] when the contracted mode is stored fastest, else [kk][row];
    // compute reads it by that orientation.
    auto lstore = [&](int s, int buf) {
#pragma unroll
        for (int r = 0; r < kRowGroups; ++r) {
            if (r >= ngr) continue;
            *(u32x4 *)&sm.a[buf][r][(tid >> 3) * kStr + (tid & 7) * 8] = ra[s][r];
        }
#pragma unroll
        for (int f = 0; f < XV; ++f) {
            const int v = tid + 512 * f;
            *(u32x4 *)&sm.x[buf][(v >> 3) * kStr + (v & 7) * 8] = rx[s][f];
        }
    };

    f32x16 acc[2][TN];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    auto compute = [&](int buf, int c) {
        if (!wave_on) return;
        const u16 *A = sm.a[buf][rg];
        const u16 *X = sm.x[buf];
        const bool kf = __builtin_amdgcn_readfirstlane(sm.kfast[rg][c]) != 0;   // uniform over the wave
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            bf16x8 va[2], vb[TN];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const int rb = 32 * i;
                if (kf) {
                    va[i] = __builtin_bit_cast(bf16x8, *(const u16x8 *)&A[(rb + r32) * kStr + ks * 16 + 8 * half]);
                } else {
                    const int kk0 = ks * 16 + 8 * (grp >> 1);
                    const int rbase = rb + 16 * (grp & 1);
                    const int o = (kk0 + (gl >> 2)) * kStr + rbase + 4 * (gl & 3);
                    typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
                    const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(A + o));
                    const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(A + o + 4 * kStr));
                    va[i] = __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
                }
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int col = chalf * (NT / 2) + 32 * j + r32;
                vb[j] = __builtin_bit_cast(bf16x8, *(const u16x8 *)&X[col * kStr + ks * 16 + 8 * half]);
            }
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if (wcol0 + 32 * j >= Nvalid) continue;   // no valid column in this subtile
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    if constexpr (ROWS_LANE)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vb[j], va[i], acc[i][j], 0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va[i], vb[j], acc[i][j], 0, 0, 0);
                }
            }
        }
    };

    const int nch = nbar;
    gload(0, 0);
    gload(nch > 1 ? 1 : 0, 1);
    __builtin_amdgcn_sched_barrier(0);
    lstore(0, 0);
    __syncthreads();
    for (int c = 0; c < nch; c += 2) {
        gload(c + 2 < nch ? c + 2 : nch - 1, 0);
        __builtin_amdgcn_sched_barrier(0);
        compute(0, c);
        if (c + 1 < nch) lstore(1, 1);
        __syncthreads();
        if (c + 1 >= nch) break;
        gload(c + 3 < nch ? c + 3 : nch - 1, 1);
        __builtin_amdgcn_sched_barrier(0);
        compute(1, c + 1);
        if (c + 2 < nch) lstore(0, 0);
        __syncthreads();
    }

    // Epilogue: entry (row mm, column ng) of the row group goes to
    // out_base + (ng / 64) out_jstride + (ng % 64) osk + mm mos[0].
    if (!wave_on) return;
    const int64_t ob = gd.out_base, ojs = gd.out_jstride, osk = a.osk, mos0 = a.mos[0];
    const bool f32out = a.out_f32 != 0;
    if (ROWS_LANE && !f32out) {
        // bf16 output contiguous along the rows (mos[0] = 1): each 64 x 32
        // subtile goes through LDS as [col][row] and out as 16-byte stores of
        // 8 consecutive rows (the loop above ended on a barrier, so the
        // staging buffers are free; every wave has a region of its own).
        u16 *so = &sm.a[0][0][0] + wave * (32 * kStr);
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            if (wcol0 + 32 * j >= Nvalid) continue;
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    so[(8 * (r >> 2) + 4 * half + (r & 3)) * kStr + 32 * i + r32] = to_bf16(acc[i][j][r]);
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int v = lane + 64 * h;
                const int col = v >> 3, rc = (v & 7) * 8;
                const int ng = wcol0 + 32 * j + col;
                const u32x4 w = *(const u32x4 *)&so[col * kStr + rc];
                if (ng < Nvalid)
                    *(u32x4 *)((u16 *)a.out + ob + (int64_t)(ng / kB) * ojs + (int64_t)(ng % kB) * osk + rc) = w;
            }
            __builtin_amdgcn_wave_barrier();
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < TN; ++j) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int inner = 8 * (r >> 2) + 4 * half + (r & 3);
                const int mm = ROWS_LANE ? 32 * i + r32 : 32 * i + inner;
                const int ng = wcol0 + 32 * j + (ROWS_LANE ? inner : r32);
                if (ng >= Nvalid) continue;
                const int64_t o = ob + (int64_t)(ng / kB) * ojs + (int64_t)(ng % kB) * osk + (int64_t)mm * mos0;
                if (f32out) ((float *)a.out)[o] = acc[i][j][r];
                else ((u16 *)a.out)[o] = to_bf16(acc[i][j][r]);
            }
    }
}

template <int K, int NT>
int launch_nt(const StageArgs &a, bool rows_lane, hipStream_t s)
{
    const dim3 g((unsigned)a.ntasks), b(512);
    if (rows_lane) hipLaunchKernelGGL((stage_b64_bf16<K, NT, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((stage_b64_bf16<K, NT, false>), g, b, 0, s, a);
    return 0;
}

template <int K>
int launch_k(const StageArgs &a, int NT, bool rows_lane, hipStream_t s)
{
    switch (NT) {
    case 256: return launch_nt<K, 256>(a, rows_lane, s);
    case 192: return launch_nt<K, 192>(a, rows_lane, s);
    case 128: return launch_nt<K, 128>(a, rows_lane, s);
    default: return -1;
    }
}

}  // namespace

bool b64_bf16_supported(int m, int bA, int bC, int nbar, bool bf16_input)
{
    return m == 2 && bA == kB && bC == kB && nbar >= 1 && nbar <= kMaxNbar && bf16_input;
}

int launch_stage_b64(const StageArgs &a, int NT, hipStream_t s)
{
    if (a.ntasks <= 0) return 0;
    if (!b64_bf16_supported(a.m, a.bA, a.bC, a.nbar, a.in_f32 == 0) || (a.k != 0 && a.k != 1)) return -1;
    // rows contiguous in the output: each lane holds one row
    const bool rows_lane = a.mos[0] == 1;
    const int rc = a.k == 0 ? launch_k<0>(a, NT, rows_lane, s) : launch_k<1>(a, NT, rows_lane, s);
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace symt
