// Block-copy bf16 stage kernel for gfx950: one level of the algorithm-by-blocks
// (Fig. mD) with bf16 operands, fp32 MFMA accumulation
// (v_mfma_f32_32x32x16_bf16), for order M in {3, 4} and square blocks of
// B in {8, 16} entries per mode (bA = bC = B).
//
// Tile contract (the same as the other stage kernels): one workgroup of four
// waves computes an MT x NT tile of one row group's GEMM
//   Out[row][nn] = sum_kk In[row][kk] * X[nn][kk],
// rows = entries of an input block without the contracted mode K,
// kk = ibar*B + lk over the contracted mode, nn over the group's output
// columns.  Here a tile's rows are the two lowest non-contracted modes in
// full (MT = B*B); the remaining non-contracted modes are fixed per M tile.
//
// Staging: every input block is read from HBM as contiguous 16-byte vectors
// in its stored order (coalesced for every permutation) and written to LDS in
// one canonical layout.  Which logical mode sits at which stored position is
// fixed by the block's insertion position Q (the permutation of §5.3 / App. B)
// and is a compile-time case here: the kernel switches once per block on Q,
// uniformly across the wave, so each case's address arithmetic is shifts and
// adds on constants.  For levels below the last (K > 0) LDS holds [kk][row]
// (row fastest) and the MFMA operands are read with ds_read_b64_tr_b16, which
// transposes 4x4 groups of 16-bit entries on the way out; at the last level
// (K = 0, where mode 0 is always the contracted one) LDS holds [row][kk] and
// operands are plain 16-byte reads.  X comes from the zero-padded bf16 panel
// [Ppad][Kx] into LDS [nn][kk].
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

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two fp32 -> bf16, round to nearest, ties to even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t to_bf16x2(float a, float b)
{
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{a, b}), bf16x2));
}

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Stored position of logical mode l inside an input block whose contracted
// mode K was inserted at position Q (modes 0..K are the sorted ones).
constexpr int stored_pos(int l, int K, int Q)
{
    return l == K ? Q : (l > K ? l : (l < Q ? l : l + 1));
}
// j-th non-contracted logical mode.
constexpr int mmode_of(int j, int K) { return j < K ? j : j + 1; }

constexpr int kBf16MaxBlocks = 512;   // input blocks per group the LDS table holds

template <int M, int B, int K, int NT, int KT>
struct Bf16Cfg {
    static constexpr int MT = B * B;
    static constexpr bool KM = K == 0;                  // LDS [row][kk] (else [kk][row])
    // b = 16 below the last level: each 16-wide k step of a chunk is one
    // whole block, staged in a region of its own; a block whose contracted
    // mode is stored fastest (q = 0) is staged there as [row][kk], any other
    // as [kk][row], so no entry is ever written transposed.
    static constexpr bool DUAL = !KM && B == 16;
    static constexpr int RS = MT + 16;                  // [kk][row] row stride (bf16)
    static constexpr int RSK = DUAL ? B + 8 : KT + 8;   // [row][kk] row stride (of one block's region if DUAL)
    static constexpr int REG = B * RS > MT * RSK ? B * RS : MT * RSK;   // one block's region (DUAL)
    static constexpr int XS = KT + 8;                   // X [nn][kk] row stride
    // waves along M: 4 for 32-wide column tiles, else 2 (1 for 64-row tiles)
    static constexpr int WM = NT <= 32 ? 4 : (MT >= 128 ? 2 : 1), WN = 4 / WM;
    static constexpr int WTM = MT / WM, WTN = NT / WN;
    static constexpr int TM = WTM / 32, TN = WTN / 32;
    static constexpr int G = KT / B;                    // whole blocks per K chunk
    static constexpr int IN_ELEMS = KM ? MT * RSK : (DUAL ? G * REG : KT * RS);
    static constexpr int PART = B * B * B / 8;          // 16-byte vectors of one block's tile part
    static constexpr int VEC = G * PART;                // ... per chunk
    static constexpr int NV = (VEC + 255) / 256;        // per thread
    static constexpr int XV = NT * KT / 8;              // X vectors per chunk
    static constexpr int NXV = (XV + 255) / 256;
    static_assert(KT % B == 0 && KT % 16 == 0, "chunk");
    static_assert(TM >= 1 && TN >= 1, "tile");
    static_assert(PART % 64 == 0, "a block part spans whole waves");
    static_assert(!DUAL || PART % 256 == 0, "DUAL: a thread's f-th vector lies in block 256 f / PART");
};

constexpr int kOutRow = 40;   // row stride (bf16) of a wave's 32 x 32 output staging tile

template <int M, int B, int K, int NT, int KT>
struct Bf16Smem {
    using C = Bf16Cfg<M, B, K, NT, KT>;
    union {
        struct {
            __attribute__((aligned(16))) u16 s_in[2][C::IN_ELEMS];
            __attribute__((aligned(16))) u16 s_x[2][NT * C::XS];
        };
        // epilogue: one 32 x 32 output subtile per wave, [nn][mm]
        __attribute__((aligned(16))) u16 s_out[4][32 * kOutRow];
    };
    int64_t s_ioff[kBf16MaxBlocks];
    int32_t s_iq[kBf16MaxBlocks];
};

// Where a thread's vector lands, for one insertion position Q: element offset
// inside the stored block (goff), LDS offset (loff) in the chunk buffer, and
// whether its 8 entries run along the contracted mode (transposed write into
// a [kk][row] buffer).  d0, d1, d2 are the vector's digits at the three
// stored positions the tile part spans in full (ascending; d0 counts entries,
// a multiple of 8); fixed_digits are the digits of the non-contracted modes
// beyond the first two, fixed by the M tile.
template <int M, int B, int K, int Q, int RS, int RSK, bool KM>
__device__ __forceinline__ void place(int d0, int d1, int d2, const int *fixed_digits, int kbase, int *goff,
                                      int *loff, bool *along_k)
{
    constexpr int m0 = mmode_of(0, K), m1 = mmode_of(1, K);
    constexpr int pk = stored_pos(K, K, Q), p0 = stored_pos(m0, K, Q), p1 = stored_pos(m1, K, Q);
    // The three full positions in ascending order.
    constexpr int lo = pk < p0 ? (pk < p1 ? pk : p1) : (p0 < p1 ? p0 : p1);
    constexpr int hi = pk > p0 ? (pk > p1 ? pk : p1) : (p0 > p1 ? p0 : p1);
    constexpr int mid = pk + p0 + p1 - lo - hi;
    static_assert(lo == 0, "stored position 0 is always spanned in full");
    int g = d0 + d1 * ipow(B, mid) + d2 * ipow(B, hi);
#pragma unroll
    for (int j = 2; j < M - 1; ++j) {
        const int p = stored_pos(mmode_of(j, K), K, Q);
        g += fixed_digits[j - 2] * ipow(B, p);
    }
    *goff = g;
    // Digits per logical role.
    auto digit_at = [&](int pos) { return pos == 0 ? d0 : (pos == mid ? d1 : d2); };
    const int dk = digit_at(pk), r0 = digit_at(p0), r1 = digit_at(p1);
    const int row = r0 + B * r1;
    if constexpr (KM) *loff = row * RSK + kbase + dk;
    else *loff = (kbase + dk) * RS + row;
    *along_k = !KM && pk == 0;
}

// Global-memory view of a 16-byte vector: the grouped form reads its input
// and X pointers from the stage table, where the compiler cannot see their
// address space; flat loads would count on both wait counters and every
// prefetched chunk would be waited for at once.
typedef __attribute__((address_space(1))) const u32x4 gu32x4;
typedef __attribute__((address_space(1))) const GroupDesc gGroupDesc;
typedef __attribute__((address_space(1))) const InEntry gInEntry;
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) u16 gu16;
typedef __attribute__((address_space(1))) u32x4 gu32x4w;

template <int M, int B, int K, int NT, int KT, int PD>
__device__ __forceinline__ void bf16_tile(const StageArgs &a, const Task task, Bf16Smem<M, B, K, NT, KT> &sm)
{
    using C = Bf16Cfg<M, B, K, NT, KT>;
    constexpr int RS = C::RS, RSK = C::RSK, XS = C::XS;
    constexpr int WM = C::WM, WTM = C::WTM, WTN = C::WTN, TM = C::TM, TN = C::TN;
    constexpr int G = C::G, PART = C::PART, NV = C::NV, NXV = C::NXV, XV = C::XV;
    constexpr bool B_IS_IN = K != 0;   // output rows run along the block rows unless mode 0 is contracted

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    gGroupDesc &gd = ((gGroupDesc *)a.groups)[task.group];
    const int n0 = task.nt * NT;
    const int Nvalid = gd.jcount * B;
    const int nbar = a.nbar;
    const int nch = (nbar + G - 1) / G;
    const u16 *in = (const u16 *)a.in;
    const u16 *xp = (const u16 *)a.xp;
    const int64_t Kx = a.Kx, Kpad = a.Kpad, Ppad = a.Ppad;

    // Digits of the fixed non-contracted modes of this M tile.
    int fixed[M > 3 ? M - 3 : 1];
    {
        int r = task.mt;
#pragma unroll
        for (int j = 0; j < M - 3; ++j) {
            fixed[j] = r % B;
            r /= B;
        }
    }
    for (int i = tid; i < nbar; i += 256) {
        gInEntry *ie = (gInEntry *)a.in_tab + gd.in_row + i;
        sm.s_ioff[i] = ie->off;
        sm.s_iq[i] = ie->q;
    }
    // This thread's vectors: block g of the chunk and digits in the part.
    // Threads beyond the chunk's vector count (only when it is not a
    // multiple of 256) load a duplicate of the last vector and store nothing,
    // so that every load is unconditional: the compiler can then wait for
    // exactly the oldest register stage instead of every load in flight.
    int vg[NV], vd0[NV], vd1[NV], vd2[NV];
    bool vok[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) {
        const int v0 = tid + 256 * f;
        vok[f] = C::VEC % 256 == 0 || v0 < C::VEC;
        const int v = vok[f] ? v0 : C::VEC - 1;
        vg[f] = v / PART;
        const int w = v % PART;
        vd0[f] = 8 * (w % (B / 8));
        const int w1 = w / (B / 8);
        vd1[f] = w1 % B;
        vd2[f] = w1 / B;
    }
    __syncthreads();

    // PD register stages of global loads: chunk c lives in stage c % PD
    // from its load until its store to LDS.
    u32x4 rin[PD][NV], rx[PD][NXV];
    int rl[PD][NV];
    bool rk[PD][NV], rv[PD][NV], rxv[PD][NXV];
    bool rkm[PD][G];   // DUAL: block g of the chunk is staged [row][kk]
    auto load_chunk = [&](int c, int u) {
#pragma unroll
        for (int f = 0; f < NV; ++f) {
            const int ib = c * G + vg[f];
            // ib is uniform across the wave (a block part spans whole
            // waves); a block beyond nbar is read as block 0 and stored as
            // zeros in block 0's layout, which covers the same LDS entries
            const bool valid = ib < nbar;
            const int ibc = valid ? ib : 0;
            const int q = __builtin_amdgcn_readfirstlane(sm.s_iq[ibc]);
            int goff = 0, loff = 0;
            bool ak = false;
            const int kb = C::DUAL ? 0 : vg[f] * B;   // DUAL: offset inside the block's region
            switch (q) {
#define STTSM_Q(QQ) \
    case QQ: \
        if constexpr (QQ <= K) \
            place<M, B, K, QQ, RS, RSK, C::KM || (C::DUAL && QQ == 0)>(vd0[f], vd1[f], vd2[f], fixed, kb, &goff, &loff, &ak); \
        break;
                STTSM_Q(0) STTSM_Q(1) STTSM_Q(2) STTSM_Q(3)
#undef STTSM_Q
            default: break;
            }
            if constexpr (C::DUAL) loff += vg[f] * C::REG;
            rl[u][f] = loff;
            rk[u][f] = ak;
            rv[u][f] = valid;
            if constexpr (C::DUAL)
                if ((256 * f) % PART == 0) rkm[u][(256 * f) / PART] = q == 0;
            rin[u][f] = *(const gu32x4 *)(in + sm.s_ioff[ibc] + goff);
        }
#pragma unroll
        for (int f = 0; f < NXV; ++f) {
            const int v0 = tid + 256 * f;
            const int v = XV % 256 == 0 || v0 < XV ? v0 : XV - 1;
            const int row = v / (KT / 8), kv = (v % (KT / 8)) * 8;
            const int64_t ng = n0 + row, kg = (int64_t)c * KT + kv;
            const bool ok = ng < Ppad && kg < Kpad;
            rxv[u][f] = ok;
            rx[u][f] = *(const gu32x4 *)(xp + (ok ? ng * Kx + kg : 0));
        }
    };
    auto store_chunk = [&](int buf, int u) {
        u16 *si = sm.s_in[buf];
        const u32x4 zero = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int f = 0; f < NV; ++f) {
            if (!vok[f]) continue;
            const u32x4 w = rv[u][f] ? rin[u][f] : zero;
            if constexpr (!C::KM) {
                if (rk[u][f]) {   // 8 entries along kk: one per LDS row
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        si[rl[u][f] + (2 * e) * RS] = (u16)(w[e] & 0xFFFFu);
                        si[rl[u][f] + (2 * e + 1) * RS] = (u16)(w[e] >> 16);
                    }
                    continue;
                }
            }
            *(u32x4 *)&si[rl[u][f]] = w;
        }
#pragma unroll
        for (int f = 0; f < NXV; ++f) {
            const int v = tid + 256 * f;
            if (XV % 256 != 0 && v >= XV) continue;
            const int row = v / (KT / 8), kv = (v % (KT / 8)) * 8;
            *(u32x4 *)&sm.s_x[buf][row * XS + kv] = rxv[u][f] ? rx[u][f] : zero;
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
    const int grp = lane >> 4, gl = lane & 15;   // 16-lane group, lane inside it
    const bool wave_live = n0 + wn * WTN < Nvalid;

    // MFMAs of chunk c; after its first k step, the loads of chunk c + PD go
    // out into the register stage u that chunk c has just left.
    auto mfma_chunk = [&](int buf, int c, int u) {
        const u16 *si = sm.s_in[buf];
        const u16 *sx = sm.s_x[buf];
        bool kmv[KT / 16];   // read before stage u is reloaded
#pragma unroll
        for (int s = 0; s < KT / 16; ++s) kmv[s] = C::KM || (C::DUAL && rkm[u][s]);
#pragma unroll
        for (int s = 0; s < KT / 16; ++s) {
            bf16x8 va[TM], vb[TN];
            // k step s: block s's region (DUAL), else columns 16 s .. 16 s + 15
            const int sbase = C::DUAL ? s * C::REG : 0, sk = C::DUAL ? 0 : 16 * s;
            if (wave_live) {
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const int rb = wm * WTM + 32 * i;
                    if (kmv[s]) {
                        va[i] = __builtin_bit_cast(bf16x8,
                                                   *(const u16x8 *)&si[sbase + (rb + r32) * RSK + sk + 8 * half]);
                    } else {
                        // Lane 4t + u of a 16-lane group points at row kk0 + t,
                        // entries rbase + 4u .. +3; the transposing read hands
                        // lane i of the group entries (rbase + i, kk0 .. kk0+3).
                        const int kk0 = sk + 8 * (grp >> 1);
                        const int rbase = rb + 16 * (grp & 1);
                        const int o = sbase + (kk0 + (gl >> 2)) * RS + rbase + 4 * (gl & 3);
                        typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
                        const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(si + o));
                        const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(si + o + 4 * RS));
                        va[i] = __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
                    }
                }
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    vb[j] = __builtin_bit_cast(bf16x8,
                                               *(const u16x8 *)&sx[(wn * WTN + 32 * j + r32) * XS + 16 * s + 8 * half]);
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j) {
                        if constexpr (B_IS_IN)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vb[j], va[i], acc[i][j], 0, 0, 0);
                        else
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va[i], vb[j], acc[i][j], 0, 0, 0);
                    }
            }
            if (s == 0) load_chunk(c + PD, u);
        }
    };

    // Every load is issued unconditionally (chunks past the end read valid
    // addresses and are masked to zero), and the chunk loop runs a multiple
    // of PD times, so that the loads in flight are the same on every path
    // and each store waits only for its own stage.  The extra chunks add
    // zeros.
    const int nch_pad = (nch + PD - 1) / PD * PD;
    // The stages go out oldest first: the scheduler must not reorder them,
    // or the first store would wait for every load in flight, and with it
    // the loop (whose waits are merged at its head) on every pass.
#pragma unroll
    for (int u = 0; u < PD; ++u) {
        load_chunk(u, u);
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int c0 = 0; c0 < nch_pad; c0 += PD) {
#pragma unroll
        for (int u = 0; u < PD; ++u) {
            const int c = c0 + u;
            store_chunk(c & 1, u);
            __syncthreads();
            mfma_chunk(c & 1, c, u);
        }
    }

    // Epilogue.  Output row mm of the tile (digits r0 = mm % B, r1 = mm / B
    // of the two lowest non-contracted modes, the rest fixed by the M tile)
    // sits at opart(mm) inside an output block; column ng of the group at
    // npart(ng) = out_base + (ng / B) out_jstride + (ng % B) osk.
    int64_t fixed_off = 0;
#pragma unroll
    for (int j = 0; j < M - 3; ++j) fixed_off += (int64_t)fixed[j] * a.mos[j + 2];
    auto opart = [&](int mm) { return (int64_t)(mm % B) * a.mos[0] + (int64_t)(mm / B) * a.mos[1] + fixed_off; };
    auto npart = [&](int ng) {
        return gd.out_base + (int64_t)(ng / B) * gd.out_jstride + (int64_t)(ng % B) * a.osk;
    };
    // D[r][lane%32] of a 32x32 subtile: register r holds row 8(r/4) + 4(lane/32) + r%4.
    if constexpr (K == 0) {
        // C in fp32.  Lanes run along the output columns, whose C-block mode
        // is mode 0 (stride 1): each store covers 2 x 128 contiguous bytes.
        if (wave_live) {
            gfloat *out = (gfloat *)a.out;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int ng = n0 + wn * WTN + j * 32 + r32;
                if (ng < Nvalid) {
                    gfloat *oj = out + npart(ng);
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int mm = wm * WTM + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                            oj[opart(mm)] = acc[i][j][r];
                        }
                }
            }
        }
    } else {
        // bf16 temporary.  Lanes run along the tile rows (block mode 0,
        // stride 1); each wave stages one 32 x 32 subtile at a time in LDS as
        // [column][row] and writes it back as 16-byte row runs.
        __syncthreads();   // every wave is done with the staging buffers
        u16 *so = sm.s_out[wave];
        gu16 *out = (gu16 *)a.out;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
#pragma unroll
                for (int r = 0; r < 16; r += 2) {
                    const uint32_t h = to_bf16x2(acc[i][j][r], acc[i][j][r + 1]);
                    const int row = 8 * (r >> 2) + 4 * half + (r & 3);
                    so[row * kOutRow + r32] = (u16)(h & 0xFFFFu);
                    so[(row + 1) * kOutRow + r32] = (u16)(h >> 16);
                }
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int v = lane + 64 * h;            // 128 runs of 8 entries
                    const int col = v >> 2, run = (v & 3) * 8;
                    const u32x4 w = *(const u32x4 *)&so[col * kOutRow + run];
                    const int ng = n0 + wn * WTN + j * 32 + col;
                    const int mm = wm * WTM + i * 32 + run;
                    if (wave_live && ng < Nvalid) *(gu32x4w *)(out + npart(ng) + opart(mm)) = w;
                }
                __builtin_amdgcn_wave_barrier();
            }
    }
}

template <int M, int B, int K, int NT, int KT, int PD>
__global__ __launch_bounds__(256, 2) void stage_fast_bf16(const StageArgs a)
{
    __shared__ Bf16Smem<M, B, K, NT, KT> sm;
    bf16_tile<M, B, K, NT, KT, PD>(a, a.tasks[blockIdx.x], sm);
}

// Grouped persistent form for the server: every task names its stage; all
// stages of one launch share (M, B, K).  Workgroups pull tasks from one
// atomic counter until the queue is empty; tasks never wait on each other.
template <int M, int B, int K, int NT, int KT, int PD>
__global__ __launch_bounds__(256, 2) void grouped_fast_bf16(const StageArgs *__restrict__ stages,
                                                            const GroupedTask *__restrict__ tasks, int ntasks,
                                                            int *__restrict__ queue_head)
{
    __shared__ Bf16Smem<M, B, K, NT, KT> sm;
    __shared__ int s_t;
    for (;;) {
        if (threadIdx.x == 0) s_t = atomicAdd(queue_head, 1);
        __syncthreads();
        const int t = s_t;
        __syncthreads();
        if (t >= ntasks) break;
        const GroupedTask gt = tasks[t];
        bf16_tile<M, B, K, NT, KT, PD>(stages[gt.stage], Task{gt.group, gt.mt, gt.nt}, sm);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// X-resident form for b = 16 (the tile contract of stage_fast_bf16 with one
// block per K chunk; every output entry gets the same MFMA sequence on the
// same operands, hence the same bits).  Differences:
//  - the tile's XNT rows of the X panel (all Kpad <= 256 k values) are
//    staged in LDS at the start of a task, so the chunk loop stages only the
//    input block;
//  - each task has one record (the input blocks' offsets and permutations,
//    the output placement), loaded one task ahead, instead of a chain of
//    task -> row group -> input table reads;
//  - every thread computes, once per M tile, the global and LDS offsets of
//    its two 16-byte vectors for each insertion position q, packed into
//    64-bit registers, so a chunk costs a shift, the load and the store;
//  - the workgroups are persistent over the plan's task order (task t on
//    workgroup t mod gridDim.x);
//  - each wave computes 64 rows x XNT columns (2 x XNT/32 MFMA tiles).
// Measured at m3_n256_b16: 96-column tiles (at most 512 tasks per level,
// one per resident workgroup) take the step from 64.5 to 57.4 us; 64 columns
// match the chunk-staged kernel, 128 columns (one workgroup per CU) are
// slower.  Kept below 64 KB of LDS: workgroups whose per-thread arrays the
// compiler had moved into LDS (70.8 KB) spent 8-9 us before their first
// instruction past the prologue's barrier.
constexpr int kXresMaxK = 256;             // largest Kpad the resident X slice holds
constexpr int kXresXS = kXresMaxK + 8;     // its row stride (bf16)

template <int M, int K, int XNT>
struct XresSmem {
    using C = Bf16Cfg<M, 16, K, 64, 16>;
    __attribute__((aligned(16))) u16 s_x[XNT * kXresXS];
    union {
        __attribute__((aligned(16))) u16 s_in[2][C::IN_ELEMS];
        __attribute__((aligned(16))) u16 s_out[4][32 * kOutRow];
    };
    int64_t s_rec[sizeof(XresRec) / 8];   // the current task's record
};

constexpr int kXresRecWords = (int)(sizeof(XresRec) / 8);
static_assert(sizeof(XresRec) % 8 == 0 && kXresRecWords <= 64, "a record is a few 8-byte words");

// The X-resident tile loop.  GROUPED = false: the tasks of one stage `a1`,
// task t on workgroup t mod gridDim.x, each record loaded one task ahead.
// GROUPED = true (the server): tasks of many stages of one (M, K), each
// naming its stage, row group and tile (GroupedTask), task t on workgroup
// t mod gridDim.x; the stage's values are read per task and its record is
// assembled from the stage's tables (no record table is uploaded).
template <int M, int K, int PD, int XNT, bool GROUPED>
__device__ __forceinline__ void xres_run(const StageArgs &a1, const StageArgs *__restrict__ stages,
                                         const GroupedTask *__restrict__ gtasks, int ngtasks,
                                         int *__restrict__ queue_head, XresSmem<M, K, XNT> &sm, int *s_task)
{
    constexpr int B = 16, NT = XNT, KT = 16;
    using C = Bf16Cfg<M, B, K, 64, KT>;
    constexpr int RS = C::RS, RSK = C::RSK, PART = C::PART, NV = C::NV;
    constexpr int TM = 2, TN = NT / 32;     // wave w: rows 64 w .. 64 w + 63, all NT columns
    constexpr bool B_IS_IN = K != 0;
    constexpr int NQ = K + 1;               // insertion positions of the contracted mode
    constexpr int XVT = NT * kXresMaxK / 8 / 256;   // X-slice vectors per thread (at most)
    static_assert(C::G == 1 && C::VEC == 512 && NV == 2 && PART == 512, "one whole block part per chunk");
    static_assert(C::DUAL || C::KM, "per-block regions or [row][kk]");
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int r32 = lane & 31, half = lane >> 5;
    const int grp = lane >> 4, gl = lane & 15;
    // Values of the stage (per launch, or per task when grouped).
    const u16 *in = (const u16 *)a1.in;
    const u16 *xp = (const u16 *)a1.xp;
    int nbar = a1.nbar;
    int nch_pad = (nbar + PD - 1) / PD * PD;
    int64_t Kx = a1.Kx, Ppad = a1.Ppad;
    int kvec = a1.Kpad / 8;                 // 16-byte vectors per X row
    int xv_count = NT * kvec;

    // Digits of this thread's two vectors in the block part (fixed).
    int vd0[NV], vd1[NV], vd2[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) {
        const int w = tid + 256 * f;
        vd0[f] = 8 * (w % (B / 8));
        const int w1 = w / (B / 8);
        vd1[f] = w1 % B;
        vd2[f] = w1 / B;
    }
    // X-slice vector v = tid + 256 f: its row and k offset (fixed per stage).
    int xrow[XVT], xk[XVT];
    auto x_slots = [&]() {
#pragma unroll
        for (int f = 0; f < XVT; ++f) {
            const int v = tid + 256 * f;
            xrow[f] = v / kvec;
            xk[f] = (v - xrow[f] * kvec) * 8;
        }
    };
    if constexpr (!GROUPED) x_slots();
    // Per vector, its global and LDS offsets for insertion position q
    // (16 bits each: goff < b^m <= 65536, loff < 2^13), packed in 64-bit
    // words at bit 16 q: plain registers, selected with a uniform shift
    // (arrays indexed per q would be placed in memory).
    static_assert(M <= 4 && C::IN_ELEMS <= 65536, "offsets fit in 16 bits");
    uint64_t gpk0 = 0, gpk1 = 0, lpk0 = 0, lpk1 = 0;
    int cur_mt = -1;
    int fixed[M > 3 ? M - 3 : 1] = {};

    // Record words, loaded one task ahead: every thread loads word
    // tid % words (so the load is not behind a branch), the first `words`
    // threads store theirs.
    const int rw = tid % kXresRecWords;
    const int64_t *recw = (const int64_t *)a1.xrec;
    int64_t next_word = 0;
    // Grouped: task t on workgroup t mod gridDim.x as well; the next task's
    // record is assembled from its stage's tables (row group, input table),
    // loaded one task ahead: the row group's fields by every thread, input
    // block tid's offset and insertion position by thread tid < nbar.
    int nx_stage = 0, nx_q = 0, nx_jc = 0, nx_n0 = 0, nx_mt = 0;
    int64_t nx_off = 0, nx_ob = 0, nx_ojs = 0;
    auto grouped_prefetch = [&](int tn) {
        const GroupedTask gt = gtasks[tn];
        nx_stage = __builtin_amdgcn_readfirstlane(gt.stage);
        const StageArgs &sa = stages[nx_stage];
        // (fields read through global-space pointers: the table pointers
        // come from memory, and flat loads would count on the LDS counter)
        gGroupDesc *g = (gGroupDesc *)sa.groups + gt.group;
        nx_ob = g->out_base;
        nx_ojs = g->out_jstride;
        nx_jc = g->jcount;
        nx_n0 = gt.nt * NT;
        nx_mt = gt.mt;
        if (tid < sa.nbar) {
            gInEntry *e = (gInEntry *)sa.in_tab + g->in_row + tid;
            nx_off = e->off;
            nx_q = e->q;
        }
    };
    if constexpr (!GROUPED)
        next_word = blockIdx.x < (unsigned)a1.ntasks ? recw[(int64_t)blockIdx.x * kXresRecWords + rw] : 0;
    else if (blockIdx.x < (unsigned)ngtasks)
        grouped_prefetch(blockIdx.x);

    for (int t = blockIdx.x;; t += gridDim.x) {
        int stage = 0;
        if constexpr (GROUPED) {
            if (t >= ngtasks) break;
            stage = nx_stage;
            XresRec *r = (XresRec *)sm.s_rec;
            if (tid < 16) r->off[tid] = nx_off;
            if (tid < 64) {   // wave 0: the insertion positions, two bits each
                const uint64_t b0 = __builtin_amdgcn_ballot_w64(tid < 16 && (nx_q & 1));
                const uint64_t b1 = __builtin_amdgcn_ballot_w64(tid < 16 && (nx_q & 2));
                if (tid == 0) {
                    uint32_t qb = 0;
                    for (int i = 0; i < 16; ++i)
                        qb |= (uint32_t)(((b0 >> i) & 1u) | (((b1 >> i) & 1u) << 1)) << (2 * i);
                    r->q_bits = (int32_t)qb;
                    r->out_base = nx_ob;
                    r->out_jstride = nx_ojs;
                    r->n0 = nx_n0;
                    r->mt = nx_mt;
                    r->jcount = nx_jc;
                }
            }
            const StageArgs &sa = stages[stage];
            in = (const u16 *)sa.in;
            xp = (const u16 *)sa.xp;
            nbar = sa.nbar;
            nch_pad = (nbar + PD - 1) / PD * PD;
            Kx = sa.Kx;
            Ppad = sa.Ppad;
            kvec = sa.Kpad / 8;
            xv_count = NT * kvec;
            x_slots();
            __syncthreads();
            const int tn = t + gridDim.x;
            grouped_prefetch(tn < ngtasks ? tn : t);
        } else {
            if (t >= a1.ntasks) break;
            if (tid < kXresRecWords) sm.s_rec[tid] = next_word;
            __syncthreads();
            const int tn = t + gridDim.x;
            next_word = recw[(int64_t)(tn < a1.ntasks ? tn : t) * kXresRecWords + rw];
        }
        const StageArgs &a = GROUPED ? stages[stage] : a1;
        const XresRec *rec = (const XresRec *)sm.s_rec;
        const int n0 = __builtin_amdgcn_readfirstlane(rec->n0);
        const int mt = __builtin_amdgcn_readfirstlane(rec->mt);
        const int Nvalid = __builtin_amdgcn_readfirstlane(rec->jcount) * B;
        const uint32_t q_bits = __builtin_amdgcn_readfirstlane(rec->q_bits);

        // X rows n0 .. n0 + 63 (zero past Ppad), k 0 .. Kpad - 1: every
        // load first, then the stores.
        u32x4 xr[XVT];
#pragma unroll
        for (int f = 0; f < XVT; ++f) {
            const int64_t ng = n0 + xrow[f];
            const bool ok = tid + 256 * f < xv_count && ng < Ppad;
            xr[f] = *(const gu32x4 *)(xp + (ok ? ng * Kx + xk[f] : 0));
            if (!ok) xr[f] = u32x4{0u, 0u, 0u, 0u};
        }
        __builtin_amdgcn_sched_barrier(0);

        if (mt != cur_mt) {
            int r = mt;
#pragma unroll
            for (int j = 0; j < M - 3; ++j) {
                fixed[j] = r % B;
                r /= B;
            }
            auto offsets = [&](int f, uint64_t *gp, uint64_t *lp) {
                uint64_t g = 0, l = 0;
                bool ak = false;
                int go = 0, lo = 0;
#define STTSM_XQ(QQ) \
    if constexpr (QQ < NQ) { \
        place<M, B, K, QQ, RS, RSK, C::KM || QQ == 0>(vd0[f], vd1[f], vd2[f], fixed, 0, &go, &lo, &ak); \
        g |= (uint64_t)(uint32_t)go << (16 * QQ); \
        l |= (uint64_t)(uint32_t)lo << (16 * QQ); \
    }
                STTSM_XQ(0) STTSM_XQ(1) STTSM_XQ(2) STTSM_XQ(3)
#undef STTSM_XQ
                *gp = g;
                *lp = l;
            };
            offsets(0, &gpk0, &lpk0);
            offsets(1, &gpk1, &lpk1);
            cur_mt = mt;
        }

        // The task's input-block offsets, one per lane (lane i holds block
        // i's): a chunk's offset is a readlane, with no LDS access on the
        // path from one chunk's barrier to the next chunk's loads.
        const int64_t lane_off = rec->off[lane & 15];
        const uint32_t off_lo = (uint32_t)lane_off, off_hi = (uint32_t)((uint64_t)lane_off >> 32);

        u32x4 rin[PD][NV];
        int rl[PD][NV];
        bool rv[PD], rq0[PD];
        auto load_chunk = [&](int c, int u) {
            const bool valid = c < nbar;
            const int ib = valid ? c : 0;
            const int q = (int)((q_bits >> (2 * ib)) & 3u);
            const uint32_t olo = __builtin_amdgcn_readlane(off_lo, ib);
            const uint32_t ohi = __builtin_amdgcn_readlane(off_hi, ib);
            const u16 *blk = in + (int64_t)(((uint64_t)ohi << 32) | olo);
            rv[u] = valid;
            rq0[u] = q == 0;
            const uint32_t sh = 16u * (uint32_t)q;
            const int go0 = (int)((gpk0 >> sh) & 0xFFFFu), go1 = (int)((gpk1 >> sh) & 0xFFFFu);
            rl[u][0] = (int)((lpk0 >> sh) & 0xFFFFu);
            rl[u][1] = (int)((lpk1 >> sh) & 0xFFFFu);
            rin[u][0] = *(const gu32x4 *)(blk + go0);
            rin[u][1] = *(const gu32x4 *)(blk + go1);
        };
        auto store_chunk = [&](int buf, int u) {
            u16 *si = sm.s_in[buf];
            const u32x4 zero = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int f = 0; f < NV; ++f) *(u32x4 *)&si[rl[u][f]] = rv[u] ? rin[u][f] : zero;
        };

        // The stages go out oldest first (see bf16_tile), after the X slice.
#pragma unroll
        for (int u = 0; u < PD; ++u) {
            load_chunk(u, u);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int f = 0; f < XVT; ++f)
            if (tid + 256 * f < xv_count) *(u32x4 *)&sm.s_x[xrow[f] * kXresXS + xk[f]] = xr[f];

        f32x16 acc[TM][TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

        // Operands of chunk c (block part from buffer buf, X slice columns
        // c KT .. c KT + KT - 1), then its MFMAs.
        auto read_ops = [&](int buf, int c, bool km, bf16x8 *va, bf16x8 *vb) {
            const u16 *si = sm.s_in[buf];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const int rb = wave * 64 + 32 * i;
                if (C::KM || km) {
                    va[i] = __builtin_bit_cast(bf16x8, *(const u16x8 *)&si[(rb + r32) * RSK + 8 * half]);
                } else {
                    const int kk0 = 8 * (grp >> 1);
                    const int rbase = rb + 16 * (grp & 1);
                    const int o = (kk0 + (gl >> 2)) * RS + rbase + 4 * (gl & 3);
                    typedef __attribute__((address_space(3))) s16x4 lds_s16x4;
                    const s16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(si + o));
                    const s16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(si + o + 4 * RS));
                    va[i] = __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
                }
            }
#pragma unroll
            for (int j = 0; j < TN; ++j)
                vb[j] = __builtin_bit_cast(bf16x8, *(const u16x8 *)&sm.s_x[(32 * j + r32) * kXresXS + c * KT + 8 * half]);
        };
        auto mma = [&](const bf16x8 *va, const bf16x8 *vb) {
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                if (j > 0 && n0 + 32 * j >= Nvalid) continue;   // no valid column in this subtile
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    if constexpr (B_IS_IN)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vb[j], va[i], acc[i][j], 0, 0, 0);
                    else
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va[i], vb[j], acc[i][j], 0, 0, 0);
                }
            }
        };

        // Chunk c lives in register stage c mod PD and LDS buffer c mod 2.
        // Iteration c reads chunk c's operands, stores chunk c + 1 into the
        // other buffer and sends chunk c + 1 + PD's loads into the stage
        // just freed, runs chunk c's MFMAs, then meets the barrier that
        // publishes chunk c + 1 (and frees buffer c mod 2 for chunk c + 2).
        // Loads and stores go out unconditionally (chunks past nbar read
        // block 0 and store zeros; the last iteration's store lands in a
        // buffer nothing reads before the epilogue's barrier), so that every
        // wait is for the stage PD iterations old; chunks past nbar skip
        // their MFMAs (the X slice holds nothing past Kpad).
        static_assert(PD % 2 == 0, "the buffer of chunk c is fixed per unrolled step");
        store_chunk(0, 0);
        bool km_cur = rq0[0];
        load_chunk(PD, 0);
        __syncthreads();
        for (int c0 = 0; c0 < nch_pad; c0 += PD) {
#pragma unroll
            for (int u = 0; u < PD; ++u) {
                const int c = c0 + u;
                const int un = (u + 1) % PD;
                bf16x8 va[TM], vb[TN];
                if (c < nbar) read_ops(u & 1, c, km_cur, va, vb);
                const bool km_next = rq0[un];
                store_chunk((u + 1) & 1, un);
                load_chunk(c + 1 + PD, un);
                if (c < nbar) mma(va, vb);
                km_cur = km_next;
                __syncthreads();
            }
        }

        // Epilogue (as in bf16_tile).
        const int64_t out_base = rec->out_base, out_jstride = rec->out_jstride;
        int64_t fixed_off = 0;
#pragma unroll
        for (int j = 0; j < M - 3; ++j) fixed_off += (int64_t)fixed[j] * a.mos[j + 2];
        auto opart = [&](int mm) { return (int64_t)(mm % B) * a.mos[0] + (int64_t)(mm / B) * a.mos[1] + fixed_off; };
        auto npart = [&](int ng) { return out_base + (int64_t)(ng / B) * out_jstride + (int64_t)(ng % B) * a.osk; };
        if constexpr (K == 0) {
            gfloat *out = (gfloat *)a.out;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int ng = n0 + j * 32 + r32;
                if (ng < Nvalid) {
                    gfloat *oj = out + npart(ng);
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int mm = wave * 64 + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                            oj[opart(mm)] = acc[i][j][r];
                        }
                }
            }
        } else {
            __syncthreads();   // every wave is done with s_in, which s_out overlays
            u16 *so = sm.s_out[wave];
            gu16 *out = (gu16 *)a.out;
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) {
#pragma unroll
                    for (int r = 0; r < 16; r += 2) {
                        const uint32_t h = to_bf16x2(acc[i][j][r], acc[i][j][r + 1]);
                        const int row = 8 * (r >> 2) + 4 * half + (r & 3);
                        so[row * kOutRow + r32] = (u16)(h & 0xFFFFu);
                        so[(row + 1) * kOutRow + r32] = (u16)(h >> 16);
                    }
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int v = lane + 64 * h;
                        const int col = v >> 2, run = (v & 3) * 8;
                        const u32x4 w = *(const u32x4 *)&so[col * kOutRow + run];
                        const int ng = n0 + j * 32 + col;
                        const int mm = wave * 64 + i * 32 + run;
                        if (ng < Nvalid) *(gu32x4w *)(out + npart(ng) + opart(mm)) = w;
                    }
                    __builtin_amdgcn_wave_barrier();
                }
        }
        __syncthreads();   // before the next task's record, X slice and staging
    }
}

template <int M, int K, int PD, int XNT>
__global__ __launch_bounds__(256, XNT == 128 ? 1 : 2) void stage_xres_bf16(const StageArgs a)
{
    __shared__ XresSmem<M, K, XNT> sm;
    xres_run<M, K, PD, XNT, false>(a, nullptr, nullptr, 0, nullptr, sm, nullptr);
}

// Grouped persistent form for the server: every task names its stage, row
// group and tile; all stages of one launch share (M, K) and the tile.
template <int M, int K, int PD, int XNT>
__global__ __launch_bounds__(256, XNT == 128 ? 1 : 2) void grouped_xres_bf16(const StageArgs *__restrict__ stages,
                                                                             const GroupedTask *__restrict__ tasks,
                                                                             int ntasks, int *__restrict__ queue_head)
{
    __shared__ XresSmem<M, K, XNT> sm;
    xres_run<M, K, PD, XNT, true>(stages[0], stages, tasks, ntasks, queue_head, sm, nullptr);
}


// Default tile (NT, KT, PD) per block size; the grouped kernel always uses it.
template <int B>
struct Bf16Default {
    static constexpr int NT = B == 16 ? 64 : 128, KT = 16, PD = 2;
};

// Other per-level tiles (NT, KT, PD), selectable for measurement.
#define STTSM_BF16_TILES_16(X) X(128, 32, 1) X(64, 32, 1) X(64, 32, 2) X(64, 16, 1) X(64, 16, 3) X(128, 16, 2) X(32, 16, 1)
#define STTSM_BF16_TILES_8(X) X(256, 32, 1) X(128, 32, 1) X(128, 32, 2) X(128, 16, 3)

template <int M, int B, int K>
int launch_one(const StageArgs &a, int NT, int KT, int PD, const StageArgs *d_stages, const GroupedTask *d_tasks,
               int ntasks, int *d_head, int grid, hipStream_t s)
{
    using D = Bf16Default<B>;
    if (d_stages) {
        if (NT != D::NT || KT != D::KT || PD != D::PD) return -1;
        const dim3 g((unsigned)std::max(1, std::min(grid, ntasks))), b(256);
        hipLaunchKernelGGL((grouped_fast_bf16<M, B, K, D::NT, D::KT, D::PD>), g, b, 0, s, d_stages, d_tasks, ntasks,
                           d_head);
        return 0;
    }
    const dim3 g((unsigned)a.ntasks), b(256);
    if (NT == D::NT && KT == D::KT && PD == D::PD) {
        hipLaunchKernelGGL((stage_fast_bf16<M, B, K, D::NT, D::KT, D::PD>), g, b, 0, s, a);
        return 0;
    }
#define STTSM_TRY(nt, kt, pd) \
    if (NT == nt && KT == kt && PD == pd) { \
        hipLaunchKernelGGL((stage_fast_bf16<M, B, K, nt, kt, pd>), g, b, 0, s, a); \
        return 0; \
    }
    if constexpr (B == 16) { STTSM_BF16_TILES_16(STTSM_TRY) }
    else { STTSM_BF16_TILES_8(STTSM_TRY) }
#undef STTSM_TRY
    return -1;
}

template <int M, int B>
int launch_mb(int K, const StageArgs &a, int NT, int KT, int PD, const StageArgs *d_stages,
              const GroupedTask *d_tasks, int ntasks, int *d_head, int grid, hipStream_t s)
{
    switch (K) {
    case 0: return launch_one<M, B, 0>(a, NT, KT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
    case 1: return launch_one<M, B, 1>(a, NT, KT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
    case 2: return launch_one<M, B, 2>(a, NT, KT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
    case 3:
        if constexpr (M > 3) return launch_one<M, B, 3>(a, NT, KT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
        return -1;
    default: return -1;
    }
}

int launch_bf16_any(int M, int B, int K, const StageArgs &a, int NT, int KT, int PD, const StageArgs *d_stages,
                    const GroupedTask *d_tasks, int ntasks, int *d_head, int grid, hipStream_t s)
{
    int rc = -1;
    if (M == 3 && B == 8) rc = launch_mb<3, 8>(K, a, NT, KT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
    else if (M == 3 && B == 16) rc = launch_mb<3, 16>(K, a, NT, KT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
    else if (M == 4 && B == 8) rc = launch_mb<4, 8>(K, a, NT, KT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
    else if (M == 4 && B == 16) rc = launch_mb<4, 16>(K, a, NT, KT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

bool bf16_fast_supported(int m, int bA, int bC, int nbar)
{
    return (m == 3 || m == 4) && bA == bC && (bA == 8 || bA == 16) && nbar >= 1 && nbar <= kBf16MaxBlocks;
}

void bf16_fast_tile(int b, int *MT, int *NT, int *KT, int *PD)
{
    *MT = b * b;
    if (b == 16) {
        *NT = Bf16Default<16>::NT, *KT = Bf16Default<16>::KT, *PD = Bf16Default<16>::PD;
    } else {
        *NT = Bf16Default<8>::NT, *KT = Bf16Default<8>::KT, *PD = Bf16Default<8>::PD;
    }
}

bool bf16_tile_supported(int b, int NT, int KT, int PD)
{
#define STTSM_HAS(nt, kt, pd) if (NT == nt && KT == kt && PD == pd) return true;
    if (b == 16) {
        if (NT == Bf16Default<16>::NT && KT == Bf16Default<16>::KT && PD == Bf16Default<16>::PD) return true;
        STTSM_BF16_TILES_16(STTSM_HAS)
    } else if (b == 8) {
        if (NT == Bf16Default<8>::NT && KT == Bf16Default<8>::KT && PD == Bf16Default<8>::PD) return true;
        STTSM_BF16_TILES_8(STTSM_HAS)
    }
#undef STTSM_HAS
    return false;
}

bool bf16_xres_supported(int b, int Kpad, bool bf16_input)
{
    return b == 16 && Kpad >= 16 && Kpad <= kXresMaxK && bf16_input;
}

namespace {

// Compute units of the current device (cached per device).
int current_cus()
{
    static int cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cache[dev]) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cache[dev] = c;
    }
    return cache[dev];
}

template <int M, int K>
int launch_xres_k(const StageArgs &a, int NT, int PD, hipStream_t s)
{
    if (!a.xrec) return -1;
    // resident workgroups per CU: two with 64- and 96-column tiles, one with 128
    const int per_cu = NT == 128 ? 1 : 2;
    const dim3 g((unsigned)std::max(1, std::min(a.ntasks, per_cu * current_cus()))), b(256);
    if (NT == 64 && PD == 2) hipLaunchKernelGGL((stage_xres_bf16<M, K, 2, 64>), g, b, 0, s, a);
    else if (NT == 64 && PD == 4) hipLaunchKernelGGL((stage_xres_bf16<M, K, 4, 64>), g, b, 0, s, a);
    else if (NT == 96 && PD == 2) hipLaunchKernelGGL((stage_xres_bf16<M, K, 2, 96>), g, b, 0, s, a);
    else if (NT == 96 && PD == 4) hipLaunchKernelGGL((stage_xres_bf16<M, K, 4, 96>), g, b, 0, s, a);
    else if (NT == 128 && PD == 2) hipLaunchKernelGGL((stage_xres_bf16<M, K, 2, 128>), g, b, 0, s, a);
    else if (NT == 128 && PD == 4) hipLaunchKernelGGL((stage_xres_bf16<M, K, 4, 128>), g, b, 0, s, a);
    else return -1;
    return 0;
}

template <int M, int K>
int launch_grouped_xres_k(int NT, int PD, const StageArgs *d_stages, const GroupedTask *d_tasks, int ntasks,
                          int *d_head, int grid, hipStream_t s)
{
    const int per_cu = NT == 128 ? 1 : 2;
    const dim3 g((unsigned)std::max(1, std::min(std::min(grid, per_cu * current_cus()), ntasks))), b(256);
#define STTSM_GX(nt, pd) \
    if (NT == nt && PD == pd) { \
        hipLaunchKernelGGL((grouped_xres_bf16<M, K, pd, nt>), g, b, 0, s, d_stages, d_tasks, ntasks, d_head); \
        return 0; \
    }
    STTSM_GX(64, 2) STTSM_GX(64, 4) STTSM_GX(96, 2) STTSM_GX(96, 4) STTSM_GX(128, 2) STTSM_GX(128, 4)
#undef STTSM_GX
    return -1;
}

int launch_xres(const StageArgs &a, int NT, int PD, hipStream_t s)
{
    if (a.m == 3) {
        switch (a.k) {
        case 0: return launch_xres_k<3, 0>(a, NT, PD, s);
        case 1: return launch_xres_k<3, 1>(a, NT, PD, s);
        case 2: return launch_xres_k<3, 2>(a, NT, PD, s);
        default: return -1;
        }
    }
    if (a.m == 4) {
        switch (a.k) {
        case 0: return launch_xres_k<4, 0>(a, NT, PD, s);
        case 1: return launch_xres_k<4, 1>(a, NT, PD, s);
        case 2: return launch_xres_k<4, 2>(a, NT, PD, s);
        case 3: return launch_xres_k<4, 3>(a, NT, PD, s);
        default: return -1;
        }
    }
    return -1;
}

}  // namespace

int launch_stage_bf16(const StageArgs &a, int NT, int KT, int PD, bool xres, hipStream_t s)
{
    if (a.ntasks <= 0) return 0;
    if (!bf16_fast_supported(a.m, a.bA, a.bC, a.nbar)) return -1;
    if (xres) {
        if (!bf16_xres_supported(a.bA, a.Kpad, a.in_f32 == 0) || (NT != 64 && NT != 96 && NT != 128) || KT != 16)
            return -1;
        const int rc = launch_xres(a, NT, PD, s);
        if (rc) return rc;
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
    return launch_bf16_any(a.m, a.bA, a.k, a, NT, KT, PD, nullptr, nullptr, 0, nullptr, 0, s);
}

int launch_grouped_xres(int m, int k, int NT, int PD, const StageArgs *d_stages, const GroupedTask *d_tasks,
                        int ntasks, int *d_head, int grid, hipStream_t s)
{
    if (ntasks <= 0) return 0;
    int rc = -1;
    if (m == 3) {
        if (k == 0) rc = launch_grouped_xres_k<3, 0>(NT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
        else if (k == 1) rc = launch_grouped_xres_k<3, 1>(NT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
        else if (k == 2) rc = launch_grouped_xres_k<3, 2>(NT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
    } else if (m == 4) {
        if (k == 0) rc = launch_grouped_xres_k<4, 0>(NT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
        else if (k == 1) rc = launch_grouped_xres_k<4, 1>(NT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
        else if (k == 2) rc = launch_grouped_xres_k<4, 2>(NT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
        else if (k == 3) rc = launch_grouped_xres_k<4, 3>(NT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
    }
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_grouped_bf16(int m, int b, int k, const StageArgs *d_stages, const GroupedTask *d_tasks, int ntasks,
                        int *d_head, int grid, hipStream_t s)
{
    if (ntasks <= 0) return 0;
    StageArgs dummy{};
    int MT, NT, KT, PD;
    bf16_fast_tile(b, &MT, &NT, &KT, &PD);
    return launch_bf16_any(m, b, k, dummy, NT, KT, PD, d_stages, d_tasks, ntasks, d_head, grid, s);
}

}  // namespace symt
