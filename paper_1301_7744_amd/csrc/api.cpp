// C ABI of libsttsm (declared in include/sttsm.h).
#include "../../include/sttsm.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "abi_util.hpp"
#include "kernels.hpp"
#include "plan.hpp"

using namespace symt;

namespace symt {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int dtype_size(int dt)
{
    switch (dt) {
    case STTSM_F32: return 4;
    case STTSM_BF16: return 2;
    case STTSM_F64: return 8;
    default: return 0;
    }
}

bool layout_ok(const bcss_layout *L, std::string *why)
{
    if (!L) { *why = "null layout"; return false; }
    if (L->m < 1 || L->m > kMaxOrder) { *why = "order m must be 1..8"; return false; }
    if (L->n < 1) { *why = "n must be >= 1"; return false; }
    if (L->b < 1) { *why = "block size b must be >= 1"; return false; }
    if (!dtype_size(L->dtype)) { *why = "unknown dtype"; return false; }
    if ((L->n + L->b - 1) / L->b > (1 << 20)) { *why = "too many blocks per mode"; return false; }
    return true;
}

}  // namespace symt

namespace {

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Optional per-level timing: a pool of event pairs recorded around each
// level's launch on the caller's stream, read back on request.
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> ev;      // 2 per slot
    std::vector<int> level;          // level per used slot
    size_t used = 0;
    int64_t dropped = 0;
};
Profiler g_prof;

// Returns the index of a free slot, or -1 (profiling off or pool exhausted).
long prof_slot(int lvl)
{
    std::lock_guard<std::mutex> lock(g_prof.mu);
    if (!g_prof.on) return -1;
    if (g_prof.used >= g_prof.level.size()) {
        ++g_prof.dropped;
        return -1;
    }
    g_prof.level[g_prof.used] = lvl;
    return (long)g_prof.used++;
}

}  // namespace

namespace symt {

// Validates an sttsm problem and returns its plan key.
int make_key(const bcss_layout *A, const bcss_layout *C, int32_t prec, PlanKey *key)
{
    std::string why;
    if (!layout_ok(A, &why)) return fail(STTSM_EINVAL, "A: " + why);
    if (!layout_ok(C, &why)) return fail(STTSM_EINVAL, "C: " + why);
    if (A->m != C->m) return fail(STTSM_EINVAL, "A and C must have the same order");
    if (C->dtype != STTSM_F32) return fail(STTSM_EINVAL, "C must be F32");
    if (prec < STTSM_PREC_FP32 || prec > STTSM_PREC_BF16X3_FIRST_BF16) return fail(STTSM_EINVAL, "unknown precision");
    if (prec == STTSM_PREC_BF16) {
        if (A->dtype != STTSM_F32 && A->dtype != STTSM_BF16) return fail(STTSM_EINVAL, "BF16 form needs F32 or BF16 A");
    } else if (A->dtype != STTSM_F32) {
        return fail(STTSM_EINVAL, "this precision form needs F32 A and X");
    }
    key->m = A->m;
    key->n = A->n;
    key->p = C->n;
    key->bA = A->b;
    key->bC = C->b;
    key->prec = prec;
    key->in_dtype = A->dtype == STTSM_F32 ? F32 : BF16;
    const char *gen = getenv("STTSM_GENERIC_KERNELS");
    key->generic_only = gen && gen[0] == '1';
    key->overrides.clear();
    for (const char *name : {"STTSM_FAST_TILE", "STTSM_BF16_TILE", "STTSM_NARROW_MT", "STTSM_WIDE_MT",
                             "STTSM_BF16_XRES"}) {
        const char *v = getenv(name);
        if (v && *v) key->overrides += std::string(name) + "=" + v + ";";
    }
    return STTSM_OK;
}

}  // namespace symt

extern "C" {

const char *sttsm_last_error(void) { return g_err.c_str(); }

const char *sttsm_version(void) { return "sttsm 0.1 (gfx950)"; }

int64_t bcss_num_blocks(int32_t m, int64_t nbar)
{
    if (m < 1 || nbar < 1) return -1;
    return binom(nbar + m - 1, m);
}

int64_t bcss_num_elems(const bcss_layout *L)
{
    std::string why;
    if (!layout_ok(L, &why)) return -1;
    const int64_t nb = bcss_num_blocks(L->m, (L->n + L->b - 1) / L->b);
    if (nb < 0) return -1;
    __int128 e = nb;
    for (int j = 0; j < L->m; ++j) {
        e *= L->b;
        if (e > ((__int128)1 << 62)) return -1;
    }
    return (int64_t)e;
}

int bcss_pack(const bcss_layout *L, const void *dense, void *bcss, void *stream)
{
    std::string why;
    if (!layout_ok(L, &why)) return fail(STTSM_EINVAL, why);
    if (!dense || !bcss) return fail(STTSM_EINVAL, "null buffer");
    const int64_t ne = bcss_num_elems(L);
    if (ne < 0) return fail(STTSM_EINVAL, "BCSS size overflows");
    const int nbar = (int)((L->n + L->b - 1) / L->b);
    const MetaTable *T = meta_get(L->m, nbar, L->b, &why);
    if (!T) return fail(STTSM_ENOMEM, why);
    if (launch_pack(dtype_size(L->dtype), dense, bcss, L->m, L->n, L->b, bcss_num_blocks(L->m, nbar),
                    T->d_tuples, as_stream(stream)))
        return fail(STTSM_EHIP, std::string("pack launch failed: ") + hipGetErrorString(hipGetLastError()));
    return STTSM_OK;
}

int bcss_unpack(const bcss_layout *L, const void *bcss, void *dense, void *stream)
{
    std::string why;
    if (!layout_ok(L, &why)) return fail(STTSM_EINVAL, why);
    if (!dense || !bcss) return fail(STTSM_EINVAL, "null buffer");
    const int nbar = (int)((L->n + L->b - 1) / L->b);
    const MetaTable *T = meta_get(L->m, nbar, L->b, &why);
    if (!T) return fail(STTSM_ENOMEM, why);
    if (launch_unpack(dtype_size(L->dtype), bcss, dense, L->m, L->n, L->b, nbar, T->d_rank, T->d_perm,
                      T->d_perm_strides, as_stream(stream)))
        return fail(STTSM_EHIP, std::string("unpack launch failed: ") + hipGetErrorString(hipGetLastError()));
    return STTSM_OK;
}

size_t sttsm_vectors_workspace_bytes(const bcss_layout *A, int64_t V)
{
    std::string why;
    if (!layout_ok(A, &why) || A->m < 2 || V < 1) return 0;
    const int nbar = (int)((A->n + A->b - 1) / A->b);
    const VecPlan *P = vec_plan_get(A->m, nbar, A->b, false, &why);
    if (!P) return 0;
    if (P->block_major)   // partials per entry, then per-block shares of the dot products
        return ((P->entries.size() * (size_t)V * (size_t)A->b * sizeof(float) + 255) / 256 * 256) +
               (size_t)nbar * (size_t)V * sizeof(float);
    return std::max<size_t>(256, (size_t)P->chunk_u.size() * (size_t)V * (size_t)A->b * sizeof(float));
}

int64_t sttsm_vectors_flops(const bcss_layout *A, int64_t V)
{
    std::string why;
    if (!layout_ok(A, &why) || A->m < 2 || V < 1) return -1;
    const int nbar = (int)((A->n + A->b - 1) / A->b);
    const VecPlan *P = vec_plan_get(A->m, nbar, A->b, false, &why);
    if (!P) return -1;
    return 2 * P->terms * V;
}

int sttsm_vectors(const bcss_layout *A, const void *A_dev, const void *x_dev, int64_t V, int64_t rs_x, float *y_dev,
                  int64_t rs_y, float *s_dev, void *ws, size_t ws_bytes, void *stream)
{
    std::string why;
    if (!layout_ok(A, &why)) return fail(STTSM_EINVAL, why);
    if (A->m < 2) return fail(STTSM_EINVAL, "vector products need m >= 2");
    if (A->dtype != STTSM_F32 && A->dtype != STTSM_BF16) return fail(STTSM_EINVAL, "A must be F32 or BF16");
    if (V < 1) return fail(STTSM_EINVAL, "need at least one vector");
    if (!A_dev || !x_dev || !y_dev || !ws) return fail(STTSM_EINVAL, "null buffer");
    if (rs_x < A->n || rs_y < A->n) return fail(STTSM_EINVAL, "row strides must be >= n");
    const int nbar = (int)((A->n + A->b - 1) / A->b);
    const VecPlan *P = vec_plan_get(A->m, nbar, A->b, true, &why);
    if (!P) return fail(STTSM_ENOMEM, why);
    if (ws_bytes < sttsm_vectors_workspace_bytes(A, V)) return fail(STTSM_EINVAL, "workspace too small");
    const int lrc =
        P->block_major
            ? launch_vectors_blocks(A->dtype, A_dev, x_dev, rs_x, V, A->n, A->b, (int64_t)P->blk_begin.size() - 1,
                                    P->d_entries, P->d_blk_begin, P->d_blk_terms, P->d_u_entry, (float *)ws,
                                    (float *)((char *)ws + (P->entries.size() * (size_t)V * (size_t)A->b *
                                                                sizeof(float) + 255) / 256 * 256),
                                    y_dev, rs_y, s_dev, as_stream(stream))
            : launch_vectors(A->dtype, A_dev, x_dev, rs_x, V, A->m, A->n, A->b, P->d_entries, P->d_chunk_begin,
                             P->d_u_chunk, (int)P->chunk_u.size(), (float *)ws, y_dev, rs_y, s_dev,
                             as_stream(stream));
    if (lrc)
        return fail(STTSM_EHIP, std::string("vector launch failed: ") + hipGetErrorString(hipGetLastError()));
    return STTSM_OK;
}

int bcss_symmetrize(const bcss_layout *L, void *bcss, void *stream)
{
    std::string why;
    if (!layout_ok(L, &why)) return fail(STTSM_EINVAL, why);
    if (!bcss) return fail(STTSM_EINVAL, "null buffer");
    const int64_t ne = bcss_num_elems(L);
    if (ne < 0) return fail(STTSM_EINVAL, "BCSS size overflows");
    const int nbar = (int)((L->n + L->b - 1) / L->b);
    const MetaTable *T = meta_get(L->m, nbar, L->b, &why);
    if (!T) return fail(STTSM_ENOMEM, why);
    const StabTable *S = stab_get(L->m, &why);
    if (!S) return fail(STTSM_ENOMEM, why);
    if (launch_symmetrize(L->dtype, bcss, L->m, L->b, T->d_tuples, T->d_rep_blocks, T->d_rep_masks,
                          (int64_t)T->rep_blocks.size(),
                          S->d_start, S->d_perm, S->d_pinv, as_stream(stream)))
        return fail(STTSM_EHIP, std::string("symmetrize launch failed: ") + hipGetErrorString(hipGetLastError()));
    return STTSM_OK;
}

int bcss_fill_hashed(const bcss_layout *L, uint64_t seed, double lo, double hi, void *bcss, void *stream)
{
    std::string why;
    if (!layout_ok(L, &why)) return fail(STTSM_EINVAL, why);
    if (!bcss) return fail(STTSM_EINVAL, "null buffer");
    if (bcss_num_elems(L) < 0) return fail(STTSM_EINVAL, "BCSS size overflows");
    const int nbar = (int)((L->n + L->b - 1) / L->b);
    const MetaTable *T = meta_get(L->m, nbar, L->b, &why);
    if (!T) return fail(STTSM_ENOMEM, why);
    if (launch_fill_hashed(dtype_size(L->dtype), bcss, L->m, L->n, L->b, bcss_num_blocks(L->m, nbar), T->d_tuples,
                           seed, lo, hi, as_stream(stream)))
        return fail(STTSM_EHIP, std::string("fill launch failed: ") + hipGetErrorString(hipGetLastError()));
    return STTSM_OK;
}

int64_t sttsm_flops(const bcss_layout *A, const bcss_layout *C)
{
    std::string why;
    if (!layout_ok(A, &why) || !layout_ok(C, &why) || A->m != C->m) return -1;
    const int64_t nbar = (A->n + A->b - 1) / A->b, pbar = (C->n + C->b - 1) / C->b;
    const int m = A->m;
    __int128 total = 0;
    for (int d = 0; d < m; ++d) {
        const int64_t jt = binom(pbar + d, d + 1), pf = binom(nbar + m - d - 2, m - d - 1);
        if (jt < 0 || pf < 0) return -1;
        __int128 t = (__int128)jt * pf;
        for (int i = 0; i < m - d; ++i) t *= A->b;
        for (int i = 0; i < d + 1; ++i) t *= C->b;
        total += t;
        if (total > ((__int128)1 << 60)) return -1;
    }
    total *= 2 * nbar;
    return (int64_t)total;
}

size_t sttsm_workspace_bytes(const bcss_layout *A, const bcss_layout *C, int32_t prec)
{
    PlanKey key;
    if (make_key(A, C, prec, &key) != STTSM_OK) return 0;
    Plan P;
    std::string why;
    if (!plan_build_host(key, &P, &why)) {
        g_err = why;
        return 0;
    }
    return P.ws_bytes;
}

int sttsm_workspace_temp(const bcss_layout *A, const bcss_layout *C, int32_t prec, int32_t k, size_t *byte_offset,
                         int32_t *dtype, int64_t *num_jtuples, int64_t *num_prefixes, int64_t *block_elems)
{
    PlanKey key;
    int rc = make_key(A, C, prec, &key);
    if (rc != STTSM_OK) return rc;
    if (k < 1 || k >= A->m) return fail(STTSM_EINVAL, "k must be 1..m-1");
    Plan P;
    std::string why;
    if (!plan_build_host(key, &P, &why)) return fail(STTSM_EINVAL, why);
    if (byte_offset) *byte_offset = (size_t)P.temp_off[k];
    if (dtype) *dtype = P.temp_dtype[k] == F32 ? STTSM_F32 : STTSM_BF16;
    if (num_jtuples) *num_jtuples = P.temp_jtuples[k];
    if (num_prefixes) *num_prefixes = P.temp_prefixes[k];
    if (block_elems) *block_elems = P.temp_block[k];
    return STTSM_OK;
}

int sttsm_plan_info(const bcss_layout *A, const bcss_layout *C, int32_t prec, int32_t level, int64_t *groups,
                    int64_t *tasks, int64_t *flops, int32_t *tile)
{
    PlanKey key;
    int rc = make_key(A, C, prec, &key);
    if (rc != STTSM_OK) return rc;
    if (level < 0 || level >= A->m) return fail(STTSM_EINVAL, "level must be 0..m-1");
    Plan P;
    std::string why;
    if (!plan_build_host(key, &P, &why)) return fail(STTSM_EINVAL, why);
    const StagePlan &S = P.stages[level];
    if (groups) *groups = (int64_t)S.groups.size();
    if (tasks) *tasks = (int64_t)S.tasks.size();
    if (flops) *flops = S.flops;
    if (tile) {
        tile[0] = S.b64 ? 4 : S.fast_bf16 ? (S.tile.xres ? 3 : 2) : S.fast ? 1 : 0;
        tile[1] = S.tile.MT;
        tile[2] = S.tile.NT;
        tile[3] = S.tile.KT;
        tile[4] = S.tile.PD;
    }
    return STTSM_OK;
}

}  // extern "C"

namespace {

// Levels 0..last of the plan for (A, C, prec); level `last` writes to `out`
// (C when last = m-1, the caller's T^(1) when last = m-2).
int run_levels(const bcss_layout *A, const void *A_dev, const void *X_dev, int64_t rs_x, int64_t cs_x,
               const bcss_layout *C, int32_t prec, int last_from_end, void *out, void *ws, size_t ws_bytes,
               void *stream)
{
    PlanKey key;
    int rc = make_key(A, C, prec, &key);
    if (rc != STTSM_OK) return rc;
    if (!A_dev || !X_dev || !out) return fail(STTSM_EINVAL, "null buffer");
    if (((uintptr_t)ws & 255) != 0) return fail(STTSM_EINVAL, "workspace must be 256-byte aligned");
    std::string why;
    const Plan *P = plan_get(key, &why);
    if (!P) return fail(STTSM_ENOMEM, why);
    if (ws_bytes < P->ws_bytes || (!ws && P->ws_bytes)) return fail(STTSM_EINVAL, "workspace too small");
    return launch_levels(P, A, A_dev, X_dev, rs_x, cs_x, last_from_end, out, (char *)ws, nullptr,
                         as_stream(stream));
}

}  // namespace

namespace symt {

int launch_levels(const Plan *P, const bcss_layout *A, const void *A_dev, const void *X_dev, int64_t rs_x,
                  int64_t cs_x, int last_from_end, void *out, char *w, const char *tabs, hipStream_t s)
{
    const int last = (int)P->stages.size() - 1 - last_from_end;
    if (last < 0) return fail(STTSM_EINVAL, "order too small for this operation");
    float *x32 = P->xp_off[0] >= 0 ? (float *)(w + P->xp_off[0]) : nullptr;
    uint16_t *xhi = P->xp_off[1] >= 0 ? (uint16_t *)(w + P->xp_off[1]) : nullptr;
    uint16_t *xlo = P->xp_off[2] >= 0 ? (uint16_t *)(w + P->xp_off[2]) : nullptr;
    // A bf16 X that already has the bf16 panel's layout (rows of exactly Kx
    // = n entries, 16-byte aligned, no padding rows or columns) is read in
    // place: the panel would be a copy of it, entry for entry.
    // STTSM_X_PANEL=1 builds every panel, for measurement and tests.
    const char *xpe0 = getenv("STTSM_X_PANEL");
    const bool keep_panels = xpe0 && atoi(xpe0) == 1;
    const uint16_t *xhi_read = xhi;
    if (xhi && !keep_panels && A->dtype == STTSM_BF16 && cs_x == 1 && rs_x == P->Kx && P->n == P->Kx && P->p == P->Ppad &&
        ((uintptr_t)X_dev & 15) == 0) {
        xhi_read = (const uint16_t *)X_dev;
        xhi = nullptr;
    }
    // Likewise the fp32 panel for an fp32 X of the panel's layout.
    const float *x32_read = x32;
    if (x32 && !keep_panels && A->dtype == STTSM_F32 && cs_x == 1 && rs_x == P->Kx && P->n == P->Kx && P->p == P->Ppad &&
        ((uintptr_t)X_dev & 15) == 0) {
        x32_read = (const float *)X_dev;
        x32 = nullptr;
    }
    if ((x32 || xhi || xlo) &&
        launch_prep_x(dtype_size(A->dtype), X_dev, rs_x, cs_x, P->p, P->n, P->Ppad, P->Kx, x32, xhi, xlo, s))
        return fail(STTSM_EHIP, std::string("X panel launch failed: ") + hipGetErrorString(hipGetLastError()));
    float *xt = P->xp_off[3] >= 0 ? (float *)(w + P->xp_off[3]) : nullptr;
    // The FP32 block-copy kernel stages an fp32 X with contiguous, 16-byte
    // aligned rows and n a multiple of 4 itself (transposed into LDS), in
    // place of the transposed panel.
    const bool x_direct = xt && !keep_panels && A->dtype == STTSM_F32 && cs_x == 1 && rs_x % 4 == 0 &&
                          P->n % 4 == 0 && ((uintptr_t)X_dev & 15) == 0;
    if (xt && !x_direct &&
        launch_prep_xt(dtype_size(A->dtype), X_dev, rs_x, cs_x, P->p, P->n, P->Kt, P->Pt, xt, s))
        return fail(STTSM_EHIP, std::string("X panel launch failed: ") + hipGetErrorString(hipGetLastError()));
    const void *slot_ptr[4] = {x32_read, xhi_read, xlo, x_direct ? X_dev : (const void *)xt};
    for (int d = 0; d <= last; ++d) {
        const StagePlan &S = P->stages[d];
        StageArgs a = S.args;
        if (tabs) {
            const TabOff &t = P->tab_off[d];
            a.groups = t.groups < 0 ? nullptr : (const GroupDesc *)(tabs + t.groups);
            a.in_tab = t.in_tab < 0 ? nullptr : (const InEntry *)(tabs + t.in_tab);
            a.tasks = t.tasks < 0 ? nullptr : (const Task *)(tabs + t.tasks);
            a.fdig = t.fdig < 0 ? nullptr : (const int32_t *)(tabs + t.fdig);
            a.fopart = t.fopart < 0 ? nullptr : (const int32_t *)(tabs + t.fopart);
            a.zero_blk = t.zero < 0 ? nullptr : (const float *)(tabs + t.zero);
            a.xrec = t.xrec < 0 ? nullptr : (const XresRec *)(tabs + t.xrec);
        }
        a.in = S.in_ws < 0 ? A_dev : (const void *)(w + S.in_ws);
        a.out = d == last ? out : (void *)(w + S.out_ws);
        a.xp = slot_ptr[S.xp_slot];
        a.xp_lo = S.xp_lo_slot >= 0 ? slot_ptr[S.xp_lo_slot] : nullptr;
        a.x_direct = S.xp_slot == 3 && x_direct;
        a.x_p = (int32_t)P->p;
        a.x_n = (int32_t)P->n;
        a.x_rs = rs_x;
        const long slot = prof_slot(S.d);
        if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot], s);
        const int lrc = S.b64         ? launch_stage_b64(a, S.tile.NT, s)
                        : S.fast_bf16 ? launch_stage_bf16(a, S.tile.NT, S.tile.KT, S.tile.PD, S.tile.xres, s)
                        : S.fast  ? launch_stage_fast(a, S.tile.MT, S.tile.NT, S.tile.KT, S.tile.PD, S.d == 0, s)
                                  : launch_stage(a, S.compute, S.tile.MT, S.tile.NT, S.d == 0, s);
        if (lrc)
            return fail(STTSM_EHIP, std::string("stage launch failed: ") + hipGetErrorString(hipGetLastError()));
        if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot + 1], s);
    }
    return STTSM_OK;
}

}  // namespace symt

extern "C" {

int sttsm(const bcss_layout *A, const void *A_dev, const void *X_dev, int64_t rs_x, int64_t cs_x,
          const bcss_layout *C, void *C_dev, int32_t prec, void *ws, size_t ws_bytes, void *stream)
{
    return run_levels(A, A_dev, X_dev, rs_x, cs_x, C, prec, 0, C_dev, ws, ws_bytes, stream);
}

int64_t sttsm_all_but_one_elems(const bcss_layout *A, const bcss_layout *C, int32_t prec)
{
    PlanKey key;
    if (make_key(A, C, prec, &key) != STTSM_OK) return -1;
    if (A->m < 2) {
        fail(STTSM_EINVAL, "all modes but one needs m >= 2");
        return -1;
    }
    Plan P;
    std::string why;
    if (!plan_build_host(key, &P, &why)) {
        fail(STTSM_EINVAL, why);
        return -1;
    }
    return P.temp_jtuples[1] * P.temp_prefixes[1] * P.temp_block[1];
}

int sttsm_all_but_one(const bcss_layout *A, const void *A_dev, const void *X_dev, int64_t rs_x, int64_t cs_x,
                      const bcss_layout *C, void *T_dev, int32_t prec, void *ws, size_t ws_bytes, void *stream)
{
    if (A && A->m < 2) return fail(STTSM_EINVAL, "all modes but one needs m >= 2");
    return run_levels(A, A_dev, X_dev, rs_x, cs_x, C, prec, 1, T_dev, ws, ws_bytes, stream);
}

size_t sttsm_rank_update_workspace_bytes(const bcss_layout *A, const bcss_layout *C, int32_t prec, int32_t rows)
{
    PlanKey key;
    if (make_key(A, C, prec, &key) != STTSM_OK) return 0;
    if (A->m < 2) {
        fail(STTSM_EINVAL, "the rank-update form needs m >= 2");
        return 0;
    }
    key.generic_only = true;
    Plan P;
    RankPlan R;
    std::string why;
    if (!plan_build_host(key, &P, &why) || !rank_plan_build_host(P, rows, &R, &why)) {
        fail(STTSM_EINVAL, why);
        return 0;
    }
    return R.ws_bytes;
}

int sttsm_rank_update(const bcss_layout *A, const void *A_dev, const void *X_dev, int64_t rs_x, int64_t cs_x,
                      const bcss_layout *C, void *C_dev, int32_t prec, int32_t rows, void *ws, size_t ws_bytes,
                      void *stream)
{
    PlanKey key;
    int rc = make_key(A, C, prec, &key);
    if (rc != STTSM_OK) return rc;
    if (A->m < 2) return fail(STTSM_EINVAL, "the rank-update form needs m >= 2");
    if (rows < 1) return fail(STTSM_EINVAL, "rows per pass must be >= 1");
    if (!A_dev || !X_dev || !C_dev) return fail(STTSM_EINVAL, "null buffer");
    if (((uintptr_t)ws & 255) != 0) return fail(STTSM_EINVAL, "workspace must be 256-byte aligned");
    std::string why;
    const RankPlan *R = rank_plan_get(key, rows, &why);
    if (!R) return fail(STTSM_ENOMEM, why);
    if (ws_bytes < R->ws_bytes || !ws) return fail(STTSM_EINVAL, "workspace too small");
    const Plan *P = R->chain;
    hipStream_t s = as_stream(stream);
    char *w = (char *)ws;
    float *x32 = P->xp_off[0] >= 0 ? (float *)(w + P->xp_off[0]) : nullptr;
    uint16_t *xhi = P->xp_off[1] >= 0 ? (uint16_t *)(w + P->xp_off[1]) : nullptr;
    uint16_t *xlo = P->xp_off[2] >= 0 ? (uint16_t *)(w + P->xp_off[2]) : nullptr;
    if ((x32 || xhi || xlo) &&
        launch_prep_x(dtype_size(A->dtype), X_dev, rs_x, cs_x, P->p, P->n, P->Ppad, P->Kx, x32, xhi, xlo, s))
        return fail(STTSM_EHIP, std::string("X panel launch failed: ") + hipGetErrorString(hipGetLastError()));
    // X panel of a level, from column k0 on (fp32 panel: float, else bf16).
    auto panel = [&](int slot, int64_t k0) -> const void * {
        if (slot == 0) return x32 ? (const void *)(x32 + k0) : nullptr;
        if (slot == 1) return xhi ? (const void *)(xhi + k0) : nullptr;
        if (slot == 2) return xlo ? (const void *)(xlo + k0) : nullptr;
        return nullptr;
    };
    auto run = [&](const StagePlan &S, const void *in, void *out, int64_t k0) -> int {
        StageArgs a = S.args;
        a.in = in;
        a.out = out;
        a.xp = panel(S.xp_slot, k0);
        a.xp_lo = S.xp_lo_slot >= 0 ? panel(S.xp_lo_slot, k0) : nullptr;
        if (!a.xp || (S.xp_lo_slot >= 0 && !a.xp_lo)) return fail(STTSM_EINVAL, "X panel missing from the plan");
        const long slot = prof_slot(S.d);
        if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot], s);
        if (launch_stage(a, S.compute, S.tile.MT, S.tile.NT, S.d == 0, s))
            return fail(STTSM_EHIP, std::string("stage launch failed: ") + hipGetErrorString(hipGetLastError()));
        if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot + 1], s);
        return STTSM_OK;
    };
    // Levels above the last temporary, as in the chain.
    for (int d = 0; d + 2 < P->m; ++d) {
        const StagePlan &S = P->stages[d];
        rc = run(S, S.in_ws < 0 ? A_dev : (const void *)(w + S.in_ws), w + S.out_ws, 0);
        if (rc != STTSM_OK) return rc;
    }
    // Passes: rows of T^(1) into the buffer, then their update of C.
    void *buf = w + R->buf_off;
    for (const RankPass &ps : R->passes) {
        rc = run(ps.row, ps.row.in_ws < 0 ? A_dev : (const void *)(w + ps.row.in_ws), buf, 0);
        if (rc != STTSM_OK) return rc;
        rc = run(ps.upd, buf, C_dev, ps.k_begin);
        if (rc != STTSM_OK) return rc;
    }
    return STTSM_OK;
}

int sttsm_profile_enable(int32_t max_launches)
{
    if (max_launches < 1 || max_launches > (1 << 16)) return fail(STTSM_EINVAL, "max_launches must be 1..65536");
    std::lock_guard<std::mutex> lock(g_prof.mu);
    for (hipEvent_t e : g_prof.ev) (void)hipEventDestroy(e);
    g_prof.ev.assign(2 * (size_t)max_launches, nullptr);
    for (auto &e : g_prof.ev)
        if (hipEventCreate(&e) != hipSuccess) {
            g_prof.ev.clear();
            g_prof.level.clear();
            g_prof.on = false;
            return fail(STTSM_EHIP, "hipEventCreate failed");
        }
    g_prof.level.assign(max_launches, -1);
    g_prof.used = 0;
    g_prof.dropped = 0;
    g_prof.on = true;
    return STTSM_OK;
}

int sttsm_profile_read(double *level_ms, int64_t *level_launches, int32_t max_levels, int64_t *dropped)
{
    if (!level_ms || !level_launches || max_levels < 1) return fail(STTSM_EINVAL, "bad output arrays");
    std::lock_guard<std::mutex> lock(g_prof.mu);
    for (int i = 0; i < max_levels; ++i) { level_ms[i] = 0.0; level_launches[i] = 0; }
    for (size_t i = 0; i < g_prof.used; ++i) {
        const int lvl = g_prof.level[i];
        if (hipEventSynchronize(g_prof.ev[2 * i + 1]) != hipSuccess) return fail(STTSM_EHIP, "event wait failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]) != hipSuccess)
            return fail(STTSM_EHIP, "hipEventElapsedTime failed");
        if (lvl >= 0 && lvl < max_levels) {
            level_ms[lvl] += ms;
            level_launches[lvl] += 1;
        }
    }
    if (dropped) *dropped = g_prof.dropped;
    g_prof.used = 0;
    g_prof.dropped = 0;
    return STTSM_OK;
}

int sttsm_profile_disable(void)
{
    std::lock_guard<std::mutex> lock(g_prof.mu);
    for (hipEvent_t e : g_prof.ev) (void)hipEventDestroy(e);
    g_prof.ev.clear();
    g_prof.level.clear();
    g_prof.used = 0;
    g_prof.on = false;
    return STTSM_OK;
}

}  // extern "C"
