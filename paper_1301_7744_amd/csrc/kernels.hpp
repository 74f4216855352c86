// Launchers of the gfx950 kernels (defined in kernels.hip, stage_bf16.hip, symmetrize.hip and vectors.hip).  Each returns 0,
// or -1 when the launch could not be made.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace symt {

int launch_pack(int esize, const void *dense, void *bcss, int m, int64_t n, int b, int64_t nblocks,
                const int32_t *d_tuples, hipStream_t s);
int launch_unpack(int esize, const void *bcss, void *dense, int m, int64_t n, int b, int nbar,
                  const int64_t *d_rank, const int32_t *d_perm, const int32_t *d_pstr, hipStream_t s);
int launch_fill_hashed(int esize, void *bcss, int m, int64_t n, int b, int64_t nblocks, const int32_t *d_tuples,
                       uint64_t seed, double lo, double hi, hipStream_t s);
int launch_prep_x(int esize, const void *X, int64_t rs, int64_t cs, int64_t p, int64_t n, int64_t Ppad,
                  int64_t Kx, float *x32, uint16_t *xhi, uint16_t *xlo, hipStream_t s);
int launch_stage(const StageArgs &a, int compute, int MT, int NT, bool first, hipStream_t s);
int launch_stage_fast(const StageArgs &a, int MT, int NT, int KT, int PD, bool first, hipStream_t s);
bool fast_tile_supported(int MT, int NT, int KT, int PD);
// Grouped persistent launch over a task queue (*d_head must be 0).
int launch_grouped(int compute, const StageArgs *d_stages, const GroupedTask *d_tasks, int ntasks, int *d_head,
                   int grid, hipStream_t s);
// Whether the block-copy kernel is instantiated for order m and nbar blocks.
bool fast_supported(int m, int nbar);
// Block-copy bf16 stage kernel (stage_bf16.hip): supported shapes, its tile,
// the per-level launch, and the grouped persistent launch over tasks whose
// stages all share (m, b, k).
bool bf16_fast_supported(int m, int bA, int bC, int nbar);
void bf16_fast_tile(int b, int *MT, int *NT, int *KT, int *PD);   // the default tile
bool bf16_tile_supported(int b, int NT, int KT, int PD);
int launch_stage_bf16(const StageArgs &a, int NT, int KT, int PD, bool xres, hipStream_t s);
// Grouped persistent X-resident form (the server): tasks as for the other
// grouped kernels; all stages share (m, k, NT, PD); the stages' xrec is not
// read (each record is assembled from the row group and input tables).
int launch_grouped_xres(int m, int k, int NT, int PD, const StageArgs *d_stages, const GroupedTask *d_tasks,
                        int ntasks, int *d_head, int grid, hipStream_t s);
// bf16 kernel for m = 2 with 64 x 64 blocks (stage_b64.hip): 256-row tiles of
// four row groups, NT in {128, 192, 256} columns, eight waves.
bool b64_bf16_supported(int m, int bA, int bC, int nbar, bool bf16_input);
int launch_stage_b64(const StageArgs &a, int NT, hipStream_t s);
// Whether the X-resident bf16 form applies: b = 16, Kpad <= 256, bf16 input.
bool bf16_xres_supported(int b, int Kpad, bool bf16_input);
int launch_grouped_bf16(int m, int b, int k, const StageArgs *d_stages, const GroupedTask *d_tasks, int ntasks,
                        int *d_head, int grid, hipStream_t s);
// In-place symmetrisation of the blocks with repeated indices (symmetrize.hip).
int launch_symmetrize(int dtype, void *bcss, int m, int b, const int32_t *d_tuples, const int32_t *d_blocks,
                      const uint8_t *d_masks, int64_t nlist, const int32_t *d_stab_start, const uint8_t *d_stab_perm,
                      const int32_t *d_stab_pinv, hipStream_t s);
// Batched vector products y_v = A x_v^(m-1), s_v = x_v . y_v (vectors.hip);
// part holds nchunks * V * b floats.
int launch_vectors(int dtype, const void *A, const void *x, int64_t rs_x, int64_t V, int m, int64_t n, int b,
                   const VecEntry *d_entries, const int32_t *d_chunk_begin, const int32_t *d_u_chunk, int nchunks,
                   float *part, float *y, int64_t rs_y, float *s, hipStream_t st);
// Block-major form for m = 3, b in {4, 8, 16}: one workgroup per stored
// block (nblocks); part holds nentries * V * b floats, dotp nbar * V.
int launch_vectors_blocks(int dtype, const void *A, const void *x, int64_t rs_x, int64_t V, int64_t n, int b,
                          int64_t nblocks, const VecEntry *d_entries, const int32_t *d_blk_begin,
                          const int32_t *d_blk_terms, const int32_t *d_u_entry, float *part, float *dotp, float *y,
                          int64_t rs_y, float *s, hipStream_t st);
int launch_prep_xt(int esize, const void *X, int64_t rs, int64_t cs, int64_t p, int64_t n, int64_t Kt, int64_t Pt,
                   float *xt, hipStream_t s);

}  // namespace symt
