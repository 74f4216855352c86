// Internal types shared by the host plan and the gfx950 kernels of libsttsm.
#pragma once
#include <stdint.h>

namespace symt {

constexpr int kMaxOrder = 8;

enum Dtype : int32_t { F32 = 0, BF16 = 1, F64 = 2 };
enum Prec : int32_t { PREC_FP32 = 0, PREC_BF16 = 1, PREC_X3_FP32 = 2, PREC_X3_BF16 = 3 };

// How one stage reads its operand and multiplies.
enum Compute : int32_t {
    CMP_FP32 = 0,   // fp32 operands, v_mfma_f32_32x32x2_f32
    CMP_BF16 = 1,   // bf16 operands (input converted on load if fp32), v_mfma_f32_32x32x16_bf16
    CMP_X3 = 2      // fp32 input split hi/lo into bf16, three bf16 products
};

// One row group of a stage: a fixed sorted prefix s of the symmetric modes
// and a fixed tuple J' of the trailing C-block indices.  Its GEMM has
// M = entries of one input block without the contracted mode, K = nbar*bA,
// N = jcount*bC (output C-block index jbar = 0..jcount-1 in the contracted
// mode).  Output block for jbar sits at out_base + jbar*out_jstride elements.
struct GroupDesc {
    int64_t out_base;
    int64_t out_jstride;
    int32_t jcount;
    int32_t in_row;   // first entry of this group's row in the input table
};

// Input block ibar of a group: element offset of the stored block sort(s, ibar)
// and the insertion position q of ibar into s (the block's mode permutation).
struct InEntry {
    int64_t off;
    int32_t q;
    int32_t pad_;
};

struct Task {
    int32_t group;
    int16_t mt;     // M tile index
    int16_t nt;     // N tile index
    int16_t noff;   // block-copy FP32 kernel: first column nt*NT + noff ...
    int16_t ncol;   // ... and ncol valid columns (a tile may be split in two)
};

// Task of the grouped persistent kernel: a tile of one (request, level) stage.
struct GroupedTask {
    int32_t stage;   // index into the launch's StageArgs array
    int32_t group;
    int16_t mt, nt;
};

// Tile of the grouped kernel (generic staging, 2x2 waves of 32x32).
constexpr int kGroupedMT = 64;
constexpr int kGroupedNT = 64;

// One term of the vector product y = A x^(m-1): stored block `r` with the
// free index at stored position q (the first position holding block index
// u = s[q]), counted `w` times (the number of block tuples with leading
// index u whose sorted form is s).  s holds the block's sorted indices.
struct VecEntry {
    int32_t r;
    int32_t q;
    float w;
    int32_t s[kMaxOrder];
};

// One task of the X-resident bf16 kernel with everything its prologue
// needs in one record: the element offsets of the group's nbar <= 16 input
// blocks, their insertion positions (2 bits each), the N tile's first
// column, the M tile, and the group's output placement.
struct XresRec {
    int64_t off[16];
    int64_t out_base;
    int64_t out_jstride;
    int32_t q_bits;
    int32_t n0;
    int32_t mt;
    int32_t jcount;
};

// Launch-wide parameters of one stage (kernel argument, passed by value).
struct StageArgs {
    const void *in;          // input tensor (A in BCSS, or T^(k+1))
    void *out;               // output tensor (T^(k), or C in BCSS)
    const void *xp;          // padded X, [Ppad][Kpad] (fp32 or bf16 by compute form)
    const void *xp_lo;       // split: low part of X (bf16), else null
    const GroupDesc *groups;
    const InEntry *in_tab;
    const Task *tasks;
    int32_t ntasks;
    int32_t m;               // order
    int32_t k;               // contracted mode
    int32_t nbar;            // number of A blocks per mode
    int32_t bA, bC;
    int32_t Kpad;            // nbar*bA
    int32_t Ppad;            // pbar*bC
    int32_t Kx;              // row stride of the X panels (Kpad rounded up to 8)
    int32_t Mblk;            // entries of an input block without mode k
    int32_t in_f32;          // 1: input stored fp32, 0: bf16
    int32_t out_f32;         // 1: output stored fp32, 0: bf16
    int32_t chunk_blocks;    // G: whole input blocks per K chunk (bA < KT), else 1
    int32_t chunk_k;         // k values per block per chunk (min(bA, KT))
    int32_t chunks_per_blk;  // ceil(bA / chunk_k)
    int32_t nchunks;         // total K chunks
    // Mixed-radix digits of the M index: for i < m-1, the i-th non-contracted
    // mode (modes in increasing order, skipping k) has radix mrad[i];
    // mmode[i] is that mode.
    int32_t mrad[kMaxOrder];
    int32_t mmode[kMaxOrder];
    // Stride of logical mode j inside a stored input block, for insertion
    // position q (0..k): sq[q][j].
    int32_t sq[kMaxOrder][kMaxOrder];
    // Strides of the output block (dimensional order).
    int32_t os[kMaxOrder];
    // Block-copy staging (stage_fast kernels): extents and strides of the
    // stored input block, and for insertion position q the LDS stride of the
    // logical mode found at stored position i: lds[q][i].
    int32_t ext_in[kMaxOrder];
    int32_t gs[kMaxOrder];
    int32_t lds[kMaxOrder][kMaxOrder];
    int32_t xt_stride;       // row stride of the transposed X panel [Kt][xt_stride]
    int32_t mos[kMaxOrder];  // os[mmode[i]]: output stride of the i-th M digit
    int32_t osk;             // os[k]: output stride of the contracted (now C-block) mode
    // Block-copy kernel tables (per launch): stored digits of each thread's
    // float4, fdig[((mt*NF + f)*m + i)*256 + t], and output offset of each
    // block row, fopart[row].
    const int32_t *fdig;
    const int32_t *fopart;
    // Block-copy FP32 kernel: one zero input block, read in place of the
    // blocks past nbar that a last, partial K chunk covers.
    const float *zero_blk;
    // Generic kernel with an fp32 output: 1 adds the tile's sums to what the
    // output holds (the rank-update form's passes after the first), 0 stores.
    int32_t accumulate;
    // X-resident bf16 kernel: one record per task, in task order.
    const XresRec *xrec;
    // FP32 block-copy kernel: 1 when xp is the caller's fp32 X itself
    // (rows of x_rs entries, x_p rows of x_n entries, x_n a multiple of 4,
    // 16-byte aligned) instead of the transposed panel, staged transposed
    // into LDS with zeros past p and n.
    int32_t x_direct;
    int32_t x_p, x_n;
    int64_t x_rs;
};


}  // namespace symt
