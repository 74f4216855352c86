// Host-side plan for BCSS sttsm: block ranks, the meta-data tensor, per-stage
// row groups, input-block tables and task lists, and the workspace layout.
// Built once per shape and precision, uploaded to the device once, cached.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "common.hpp"

namespace symt {

// binom(n, k) exactly; -1 on overflow or n < 0.
int64_t binom(int64_t n, int64_t k);
// Colex rank of a sorted tuple: sum_i binom(s_i + i, i + 1).
int64_t colex_rank(const int32_t *s, int len);
// All sorted len-tuples over [0, N) in colex order, flattened (len ints each).
std::vector<int32_t> sorted_tuples(int len, int N);

// Tile shape of one stage launch.
struct TileCfg {
    int MT, NT, WM, WN;
    int KT = 16;   // K chunk of the block-copy kernel
    int PD = 1;    // its prefetch depth (register sets of staged loads)
    bool xres = false;   // bf16 block-copy, b = 16: the X-resident persistent form
};

struct StagePlan {
    int d = 0;          // loop level (0 forms T^(m-1))
    int k = 0;          // contracted mode
    int compute = CMP_FP32;
    bool fast = false;  // block-copy staging kernel (whole 256-row blocks, bA | 16)
    bool fast_bf16 = false;   // block-copy bf16 kernel (m in {3, 4}, bA = bC in {8, 16})
    bool b64 = false;         // bf16 kernel for m = 2, bA = bC = 64 (tasks of four row groups)
    TileCfg tile{};
    StageArgs args{};   // everything but in/out/xp pointers
    std::vector<GroupDesc> groups;
    std::vector<InEntry> in_tab;
    std::vector<Task> tasks;
    std::vector<int32_t> fdig, fopart;   // block-copy kernel tables (see StageArgs)
    std::vector<XresRec> xrec;           // X-resident bf16 kernel: per task record
    // Device copies (owned by the plan).
    GroupDesc *d_groups = nullptr;
    InEntry *d_in_tab = nullptr;
    Task *d_tasks = nullptr;
    int32_t *d_fdig = nullptr, *d_fopart = nullptr;
    XresRec *d_xrec = nullptr;
    std::vector<float> zero;   // block-copy FP32 kernel: one zero input block
    float *d_zero = nullptr;
    // Where the operands live: -1 means the caller's A (input) or C (output),
    // otherwise a byte offset into the workspace.
    int64_t in_ws = -1, out_ws = -1;
    int xp_slot = 0, xp_lo_slot = -1;  // which padded-X panel (see Plan::xp_off)
    int64_t flops = 0;
    int64_t out_elems = 0;
};

// Byte offsets of one stage's tables inside Plan::tab_blob (-1: empty).
struct TabOff {
    int64_t groups = -1, in_tab = -1, tasks = -1, fdig = -1, fopart = -1, zero = -1, xrec = -1;
};

struct Plan {
    int m = 0;
    int64_t n = 0, p = 0;
    int bA = 0, bC = 0;
    int nbar = 0, pbar = 0;
    int prec = 0, in_dtype = 0;
    int64_t Kpad = 0, Ppad = 0, Kx = 0;   // Kx: row stride of the X panels
    int64_t Kt = 0, Pt = 0;               // transposed fp32 panel: Kt rows of Pt entries
    // X panels in the workspace: slot 0 fp32, slot 1 bf16 (rounded), slot 2
    // bf16 lo, all [Ppad][Kx]; slot 3 fp32 transposed [Kt][Pt]; all zero-padded.
    int64_t xp_off[4] = {-1, -1, -1, -1};
    // Temporaries T^(k), k = 1..m-1.
    int64_t temp_off[kMaxOrder] = {};
    int temp_dtype[kMaxOrder] = {};
    int64_t temp_jtuples[kMaxOrder] = {};
    int64_t temp_prefixes[kMaxOrder] = {};
    int64_t temp_block[kMaxOrder] = {};
    size_t ws_bytes = 0;
    int64_t flops = 0;
    std::vector<StagePlan> stages;
    // Host-only plans (plan_get_host): every stage's tables packed into one
    // buffer, each table 256-byte aligned, for a device region the caller
    // provides; tab_off[d] gives stage d's offsets.
    std::vector<unsigned char> tab_blob;
    std::vector<TabOff> tab_off;
};

struct PlanKey {
    int m;
    int64_t n, p;
    int bA, bC, prec, in_dtype;
    bool generic_only = false;   // force the generic staging kernel (testing)
    bool grouped = false;        // tiles of the grouped kernel (serving)
    // X-resident levels: per-task records and the XCD locality order of the
    // tasks (the server's grouped X-resident kernel reads neither).
    bool xres_records = true;
    // The measurement overrides of the tile choice in force when the plan was
    // built (STTSM_FAST_TILE, STTSM_BF16_TILE, STTSM_NARROW_MT,
    // STTSM_WIDE_MT), so that a plan is never reused under other overrides.
    std::string overrides;
    bool operator<(const PlanKey &o) const;
};

// Builds (first call) or returns the cached plan; uploads device tables.
// Returns nullptr and fills *err on failure.
const Plan *plan_get(const PlanKey &key, std::string *err);
// Host-only plan, built once per (device, key) and cached, with its tables
// packed into tab_blob; allocates no device memory.  The stages' table
// pointers in args are null: a launch rebases them onto a device copy of
// tab_blob.
const Plan *plan_get_host(const PlanKey &key, std::string *err);
// Host part only (no device upload); for size queries.  Caller owns result.
// cus: compute units of the device the plan runs on (the block-copy FP32
// stages split tail tiles so that no CU gets more than one half tile extra).
bool plan_build_host(const PlanKey &key, Plan *out, std::string *err, int cus = 256);

// Rank-update form of the operation (the second algorithmic variant of §8,
// stated there for m = 2 as C = sum_i X_i (A_i X^T)): with Y = A x_1 X ...
// x_{m-1} X (every mode but mode 0; its row i is row i of A times X in the
// other modes), C = sum over the block rows i of Y of X_{:,i} x_0 Y_i.  The
// block rows are taken in passes of `rows`: a pass forms its rows of Y (the
// last temporary level restricted to the pass's prefixes) into a buffer of
// one pass, then adds their rank-(rows * bA) update to C (the last level over
// the pass's K range; the first pass stores, later passes add, in pass
// order).  Levels above run as in the chain.  Every level uses the generic
// staging kernel.
struct RankPass {
    StagePlan row;       // level m-2 restricted to the pass's prefixes, writing the pass buffer
    StagePlan upd;       // level m-1 over the pass's rows only
    int64_t k_begin = 0; // first contracted index of the pass (pass start * bA)
};
struct RankPlan {
    const Plan *chain = nullptr;   // generic-kernel chain plan: X panels and levels 0..m-3
    int rows = 0;                  // block rows per pass
    std::vector<RankPass> passes;
    int64_t buf_off = 0;           // the pass buffer in the workspace
    int64_t buf_elems = 0;
    size_t ws_bytes = 0;
};
// Host part from a host-built chain plan (generic kernels, m >= 2), for size
// queries; rank_plan_get builds it over the cached chain plan and uploads its
// tables.  rows >= nbar gives one pass.
bool rank_plan_build_host(const Plan &chain, int rows, RankPlan *out, std::string *err);
const RankPlan *rank_plan_get(const PlanKey &key, int rows, std::string *err);

// Meta-data tensor of App. B for an order-m BCSS with nbar blocks per mode:
// for every block t (dimensional order over nbar^m) the rank of sort(t) and a
// permutation id; perm_strides[id*m + j] is the stride, inside the stored
// block of extent b, of logical mode j.
struct MetaTable {
    int m = 0, nbar = 0, b = 0;
    std::vector<int64_t> rank;       // nbar^m
    std::vector<int32_t> perm;       // nbar^m
    std::vector<int32_t> perm_strides;
    std::vector<int32_t> tuples;     // sorted block tuples in colex order, m each
    std::vector<int32_t> rep_blocks; // colex ranks of the tuples with a repeated index
    std::vector<uint8_t> rep_masks;  // their run masks (bit j: s_j == s_{j+1})
    int64_t *d_rank = nullptr;
    int32_t *d_rep_blocks = nullptr;
    uint8_t *d_rep_masks = nullptr;
    int32_t *d_perm = nullptr;
    int32_t *d_perm_strides = nullptr;
    int32_t *d_tuples = nullptr;
};
const MetaTable *meta_get(int m, int nbar, int b, std::string *err);

// Stabilisers of sorted block tuples of order m: a sorted tuple's equal
// entries form runs of consecutive positions; bit j of its run mask is set
// when s_j == s_{j+1}.  The permutations of the m positions that map every
// run onto itself (the tuple's stabiliser) for mask x are
// perm[start[x]*m .. start[x+1]*m), m positions each, identity first.
// Work list of the batched vector product for an order-m BCSS with nbar
// blocks per mode: for every output block row u (0..nbar-1) the terms
// (stored block, free position, weight) that add to y's rows u*b..u*b+b-1,
// cut into chunks of at most kVecChunk terms; chunks of one u are
// consecutive, u_chunk[u]..u_chunk[u+1].
constexpr int kVecChunk = 4;
struct VecPlan {
    int m = 0, nbar = 0, b = 0;
    std::vector<VecEntry> entries;
    std::vector<int32_t> chunk_begin;   // per chunk: first entry; plus a final end
    std::vector<int32_t> chunk_u;       // per chunk: its output block row
    std::vector<int32_t> u_chunk;       // nbar + 1
    int64_t terms = 0;                  // sum over entries of b^m (multiply-adds per vector)
    VecEntry *d_entries = nullptr;
    int32_t *d_chunk_begin = nullptr, *d_chunk_u = nullptr, *d_u_chunk = nullptr;
    // Block-major form (m = 3, b in {4, 8, 16}): one workgroup per stored
    // block serves every vector and every term of the block, so A is read
    // once per batch.  Block r's terms are entries blk_terms[blk_begin[r] ..
    // blk_begin[r + 1]); output block row u sums entries u_entry[u] ..
    // u_entry[u + 1] (entries are grouped by u), one partial per entry.
    bool block_major = false;
    std::vector<int32_t> blk_begin, blk_terms, u_entry;
    int32_t *d_blk_begin = nullptr, *d_blk_terms = nullptr, *d_u_entry = nullptr;
};
// Built on the host (and uploaded when upload is true), cached per device.
const VecPlan *vec_plan_get(int m, int nbar, int b, bool upload, std::string *err);

struct StabTable {
    int m = 0;
    std::vector<int32_t> start;   // 2^(m-1) + 1
    std::vector<uint8_t> perm;
    // pinv[p * kMaxOrder + i]: the position permutation p puts mode i at
    // (perm[p * m + pinv] == i); entries past m are 0.
    std::vector<int32_t> pinv;
    int32_t *d_start = nullptr;
    uint8_t *d_perm = nullptr;
    int32_t *d_pinv = nullptr;
};
const StabTable *stab_get(int m, std::string *err);

}  // namespace symt
