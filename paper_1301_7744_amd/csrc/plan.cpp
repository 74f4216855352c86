// Host plan for BCSS sttsm (see plan.hpp).
#include "plan.hpp"

#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

namespace symt {

int64_t binom(int64_t n, int64_t k)
{
    if (n < 0 || k < 0 || k > n) return (n >= 0 && k >= 0) ? 0 : -1;
    if (k > n - k) k = n - k;
    __int128 r = 1;
    for (int64_t i = 1; i <= k; ++i) {
        r = r * (n - k + i) / i;   // exact: r is binom(n-k+i, i) after this step
        if (r > (__int128)INT64_MAX) return -1;
    }
    return (int64_t)r;
}

int64_t colex_rank(const int32_t *s, int len)
{
    int64_t r = 0;
    for (int i = 0; i < len; ++i) r += binom((int64_t)s[i] + i, i + 1);
    return r;
}

std::vector<int32_t> sorted_tuples(int len, int N)
{
    std::vector<int32_t> out;
    if (len == 0) return out;
    std::vector<int32_t> s(len, 0);
    for (;;) {
        out.insert(out.end(), s.begin(), s.end());
        // colex successor: increment the first entry that can grow while the
        // tuple stays sorted; reset the entries before it to zero
        int i = 0;
        while (i < len && s[i] >= (i + 1 < len ? s[i + 1] : N - 1)) ++i;
        if (i == len) break;
        ++s[i];
        for (int l = 0; l < i; ++l) s[l] = 0;
    }
    return out;
}

bool PlanKey::operator<(const PlanKey &o) const
{
    if (m != o.m) return m < o.m;
    if (n != o.n) return n < o.n;
    if (p != o.p) return p < o.p;
    if (bA != o.bA) return bA < o.bA;
    if (bC != o.bC) return bC < o.bC;
    if (prec != o.prec) return prec < o.prec;
    if (in_dtype != o.in_dtype) return in_dtype < o.in_dtype;
    if (grouped != o.grouped) return grouped < o.grouped;
    if (generic_only != o.generic_only) return generic_only < o.generic_only;
    if (xres_records != o.xres_records) return xres_records < o.xres_records;
    return overrides < o.overrides;
}

static int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Generic-kernel tile by the rows of an input block.  Blocks of more than 128
// rows take 128-row tiles too: half the LDS of a 256-row tile, so twice the
// workgroups per CU (measured: m4_n64_b8 FP32 127 -> 119 us, m3_n256_b16 on
// the generic kernel 320 -> 262 us; STTSM_WIDE_MT=256 restores 256 rows).
static TileCfg choose_tile(int Mblk)
{
    if (Mblk > 128) {
        const char *e = getenv("STTSM_WIDE_MT");   // measurement override
        if (e && atoi(e) == 256) return {256, 64, 4, 1};
        return {128, 64, 2, 2};
    }
    if (Mblk > 64) return {128, 64, 2, 2};
    if (Mblk > 32) return {64, 64, 2, 2};
    return {32, 128, 1, 4};
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup i on XCD
// i mod 8, each XCD with its own L2), and within an XCD round-robin over its
// CUs: the l-th workgroup of an XCD shares a CU with the (l + cus)-th, where
// cus = CUs per XCD (measured: the rotation's starting CU varies from launch
// to launch, its period does not).  So the layout below
//  - deals whole row groups to XCDs (all tiles of a group read the same
//    input blocks), largest first to the XCD with the least work so far;
//  - splits, when an XCD's last round is short (r tiles past a multiple of
//    cus, 2r <= cus) and the kernel honours column ranges, r of its widest
//    tiles into two column halves, so that no CU runs a whole tile more than
//    the others;
//  - spreads each XCD's tiles over its CU slots, largest first to the
//    least-loaded slot (longest-processing-time order), within the number
//    of tiles the dispatch order gives each slot; list position 8*l + x
//    holds the l-th task of XCD x.
// cost(t) is the work of tile t.
// Tasks grouped by a locality key per row group, the keys dealt to the 8
// XCDs (largest task count first, to the least-loaded XCD), then
// interleaved so that task t runs on XCD t % 8 (workgroups are dispatched
// to the XCDs in turn).  Groups with equal keys read the same input blocks,
// so each block is fetched into one XCD's L2 (or two, at the first level).
template <class KeyFn>
static void order_tasks_by_task_key(std::vector<Task> *tasks, KeyFn key)
{
    constexpr int kXcd = 8;
    std::map<int64_t, std::vector<Task>> by_key;
    for (const Task &t : *tasks) by_key[key(t)].push_back(t);
    std::vector<std::pair<size_t, int64_t>> sizes;
    for (auto &kv : by_key) sizes.push_back({kv.second.size(), kv.first});
    std::stable_sort(sizes.begin(), sizes.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    std::vector<std::vector<Task>> bins(kXcd);
    std::vector<size_t> load(kXcd, 0);
    for (const auto &sz : sizes) {
        int best = 0;
        for (int x = 1; x < kXcd; ++x)
            if (load[x] < load[best]) best = x;
        const auto &v = by_key[sz.second];
        bins[best].insert(bins[best].end(), v.begin(), v.end());
        load[best] += v.size();
    }
    std::vector<Task> out;
    out.reserve(tasks->size());
    size_t longest = 0;
    for (auto &bn : bins) longest = std::max(longest, bn.size());
    for (size_t l = 0; l < longest; ++l)
        for (int x = 0; x < kXcd; ++x)
            if (l < bins[x].size()) out.push_back(bins[x][l]);
    tasks->swap(out);
}

static void order_tasks_by_key(std::vector<Task> *tasks, const std::vector<int64_t> &group_key)
{
    order_tasks_by_task_key(tasks, [&](const Task &t) { return group_key[t.group]; });
}

template <class Cost>
static void order_tasks_for_xcds(std::vector<Task> *tasks, Cost cost, int cus, bool split);

// Group-order layout: whole row groups dealt to the XCD with the fewest
// tiles, each XCD keeping its groups' tiles in order, so the tiles that
// share a row group's input blocks run next to each other in time.  When a
// level has more tiles than the chip holds at once this locality decides
// how often inputs come back from L2 rather than HBM (the bf16 block-copy
// kernel on m = 4 shapes ran three times slower with its tiles reordered by
// size), so every level uses it except an FP32 block-copy level whose tiles
// are all resident at once, which gets the balanced placement below.
static void order_tasks_group_major(std::vector<Task> *tasks)
{
    constexpr int kXcd = 8;
    std::vector<std::vector<Task>> bins(kXcd);
    std::vector<size_t> load(kXcd, 0);
    size_t gi = 0;
    for (size_t i = 0; i < tasks->size(); ++gi) {
        size_t j = i;
        while (j < tasks->size() && (*tasks)[j].group == (*tasks)[i].group) ++j;
        int best = (int)(gi % kXcd);   // ties: round robin
        for (int x = 0; x < kXcd; ++x)
            if (load[x] < load[best]) best = x;
        for (size_t t = i; t < j; ++t) bins[best].push_back((*tasks)[t]);
        load[best] += j - i;
        i = j;
    }
    std::vector<Task> out;
    out.reserve(tasks->size());
    size_t longest = 0;
    for (auto &b : bins) longest = std::max(longest, b.size());
    for (size_t l = 0; l < longest; ++l)
        for (int x = 0; x < kXcd; ++x)
            if (l < bins[x].size()) out.push_back(bins[x][l]);
    tasks->swap(out);
}

template <class Cost>
static void order_tasks_for_xcds(std::vector<Task> *tasks, Cost cost, int cus, bool split)
{
    constexpr int kXcd = 8;
    struct Run {
        size_t begin, end;
        int64_t work, top;
    };
    std::vector<Run> runs;
    for (size_t i = 0; i < tasks->size();) {
        size_t j = i;
        int64_t w = 0, top = 0;
        while (j < tasks->size() && (*tasks)[j].group == (*tasks)[i].group) {
            const int64_t c = cost((*tasks)[j]);
            w += c;
            top = std::max(top, c);
            ++j;
        }
        runs.push_back(Run{i, j, w, top});
        i = j;
    }
    std::stable_sort(runs.begin(), runs.end(), [](const Run &x, const Run &y) {
        return x.top != y.top ? x.top > y.top : x.work > y.work;
    });
    std::vector<std::vector<Task>> bins(kXcd);
    std::vector<int64_t> load(kXcd, 0);
    for (size_t r = 0; r < runs.size(); ++r) {
        int best = (int)(r % kXcd);   // ties: round robin
        for (int x = 0; x < kXcd; ++x)
            if (load[x] < load[best]) best = x;
        for (size_t t = runs[r].begin; t < runs[r].end; ++t) bins[best].push_back((*tasks)[t]);
        load[best] += runs[r].work;
    }
    auto by_cost = [&](const Task &x, const Task &y) { return cost(x) > cost(y); };
    const int S = std::max(cus, 1);
    for (auto &b : bins) {
        std::stable_sort(b.begin(), b.end(), by_cost);
        const int r = (int)(b.size() % (size_t)S);
        if (split && r > 0 && 2 * r <= S) {
            std::vector<Task> halves;
            int done = 0;
            for (size_t t = 0; t < b.size() && done < r; ++t) {
                Task &w = b[t];
                if (w.ncol <= 32) continue;
                const int h = (w.ncol / 32 + 1) / 2 * 32;   // first half: whole 32-column subtiles
                Task second = w;
                second.noff = (int16_t)(w.noff + h);
                second.ncol = (int16_t)(w.ncol - h);
                w.ncol = (int16_t)h;
                halves.push_back(second);
                ++done;
            }
            b.insert(b.end(), halves.begin(), halves.end());
            std::stable_sort(b.begin(), b.end(), by_cost);
        }
        // The l-th task of this XCD runs on CU slot l mod S, so slot c runs
        // cap(c) = ceil((n - c) / S) tasks.  Give each task, largest first,
        // to the least-loaded slot with room left (longest processing time
        // first under those counts), then lay the slots out in that order.
        const size_t n = b.size();
        if (n == 0) continue;
        std::vector<int64_t> sl(S, 0);
        std::vector<std::vector<int>> mine(S);
        for (size_t t = 0; t < n; ++t) {
            int best = -1;
            for (int c = 0; c < S && (size_t)c < n; ++c) {
                const size_t cap = (n - (size_t)c + S - 1) / S;
                if (mine[c].size() >= cap) continue;
                if (best < 0 || sl[c] < sl[best]) best = c;
            }
            mine[best].push_back((int)t);
            sl[best] += cost(b[t]);
        }
        std::vector<Task> laid;
        laid.reserve(n);
        for (size_t l = 0; l < n; ++l) laid.push_back(b[mine[l % S][l / S]]);
        b.swap(laid);
    }
    std::vector<Task> out;
    out.reserve(tasks->size());
    size_t longest = 0;
    for (auto &b : bins) longest = std::max(longest, b.size());
    for (size_t l = 0; l < longest; ++l)
        for (int x = 0; x < kXcd; ++x)
            if (l < bins[x].size()) out.push_back(bins[x][l]);
    tasks->swap(out);
}

// Tile override for tuning experiments: STTSM_FAST_TILE="MTxNTxKTxPD" for
// every level, or a comma-separated list per level (missing levels keep the
// default).
static bool fast_tile_override(int level, int *mt, int *nt, int *kt, int *pd)
{
    const char *e = getenv("STTSM_FAST_TILE");
    if (!e || !*e) return false;
    std::string str(e);
    std::vector<std::string> parts;
    size_t pos = 0;
    while (pos <= str.size()) {
        size_t c = str.find(',', pos);
        if (c == std::string::npos) c = str.size();
        parts.push_back(str.substr(pos, c - pos));
        pos = c + 1;
    }
    const std::string &p = parts.size() == 1 ? parts[0] : (level < (int)parts.size() ? parts[level] : std::string());
    return sscanf(p.c_str(), "%dx%dx%dx%d", mt, nt, kt, pd) == 4;
}

// Measurement override of the bf16 block-copy tiles: STTSM_BF16_TILE =
// "NTxKTxPD" for every level, or a comma-separated list per level.
static bool bf16_tile_override(int level, int *nt, int *kt, int *pd)
{
    const char *e = getenv("STTSM_BF16_TILE");
    if (!e || !*e) return false;
    std::string str(e);
    std::vector<std::string> parts;
    size_t pos = 0;
    while (pos <= str.size()) {
        size_t c = str.find(',', pos);
        if (c == std::string::npos) c = str.size();
        parts.push_back(str.substr(pos, c - pos));
        pos = c + 1;
    }
    const std::string &p = parts.size() == 1 ? parts[0] : (level < (int)parts.size() ? parts[level] : std::string());
    return sscanf(p.c_str(), "%dx%dx%d", nt, kt, pd) == 3;
}

static int kt_of(int compute) { return compute == CMP_FP32 ? 16 : 32; }

bool plan_build_host(const PlanKey &key, Plan *P, std::string *err, int cus)
{
    const int m = key.m;
    if (m < 1 || m > kMaxOrder || key.n < 1 || key.p < 1 || key.bA < 1 || key.bC < 1) {
        *err = "bad shape";
        return false;
    }
    P->m = m;
    P->n = key.n;
    P->p = key.p;
    P->bA = key.bA;
    P->bC = key.bC;
    P->prec = key.prec;
    P->in_dtype = key.in_dtype;
    const int64_t nbar64 = (key.n + key.bA - 1) / key.bA;
    const int64_t pbar64 = (key.p + key.bC - 1) / key.bC;
    if (nbar64 > (1 << 20) || pbar64 > (1 << 20)) {
        *err = "too many blocks per mode";
        return false;
    }
    const int nbar = (int)nbar64, pbar = (int)pbar64, bA = key.bA, bC = key.bC;
    P->nbar = nbar;
    P->pbar = pbar;
    P->Kpad = (int64_t)nbar * bA;
    P->Ppad = (int64_t)pbar * bC;
    P->Kx = round_up(P->Kpad, 8);
    P->Kt = round_up(P->Kpad, 32);
    P->Pt = round_up(P->Ppad, 128);
    if (P->Kpad > INT32_MAX / 2 || P->Ppad > INT32_MAX / 2) {
        *err = "dimension too large";
        return false;
    }

    // Compute form per level and storage type of each temporary.
    int cmp[kMaxOrder], tdt[kMaxOrder];
    for (int d = 0; d < m; ++d) {
        switch (key.prec) {
        case PREC_FP32: cmp[d] = CMP_FP32; break;
        case PREC_BF16: cmp[d] = CMP_BF16; break;
        case PREC_X3_FP32: cmp[d] = d == 0 ? CMP_X3 : CMP_FP32; break;
        case PREC_X3_BF16: cmp[d] = d == 0 ? CMP_X3 : CMP_BF16; break;
        default: *err = "bad precision"; return false;
        }
    }
    for (int k = 1; k < m; ++k) {
        const bool bf = key.prec == PREC_BF16 || key.prec == PREC_X3_BF16;
        tdt[k] = bf ? BF16 : F32;
    }

    // Which levels take the block-copy kernel: fp32 operands, input blocks
    // whose entries without the contracted mode number exactly 256, and bA
    // dividing the 16-wide K chunk with at least 4 (one float4 per row run).
    bool fast[kMaxOrder];
    for (int d = 0; d < m; ++d) {
        const int k = m - 1 - d;
        int64_t mblk = 1;
        for (int j = 0; j < m; ++j)
            if (j != k) mblk *= (j <= k ? bA : bC);
        const int in_dt = d == 0 ? key.in_dtype : tdt[k + 1];
        fast[d] = cmp[d] == CMP_FP32 && in_dt == F32 && mblk == 256 && (bA == 4 || bA == 8 || bA == 16) &&
                  bC % 4 == 0 && !key.generic_only && !key.grouped && fast_supported(m, nbar);
    }
    // Levels that take the block-copy bf16 kernel: bf16 operands stored bf16,
    // square blocks of 8 or 16, order 3 or 4; the output is the bf16
    // temporary, or C in fp32 at the last level.
    bool fast16[kMaxOrder];
    for (int d = 0; d < m; ++d) {
        const int k = m - 1 - d;
        const int in_dt = d == 0 ? key.in_dtype : tdt[k + 1];
        const int out_dt = k == 0 ? F32 : tdt[k];
        fast16[d] = cmp[d] == CMP_BF16 && in_dt == BF16 && out_dt == (k == 0 ? F32 : BF16) &&
                    bf16_fast_supported(m, bA, bC, nbar) && !key.generic_only;
    }

    // Workspace: X panels first.
    size_t ws = 0;
    bool need[4] = {false, false, false, false};
    for (int d = 0; d < m; ++d) {
        if (cmp[d] == CMP_FP32 && !fast[d]) need[0] = true;
        if (cmp[d] == CMP_FP32 && fast[d]) need[3] = true;
        if (cmp[d] == CMP_BF16 || cmp[d] == CMP_X3) need[1] = true;
        if (cmp[d] == CMP_X3) need[2] = true;
    }
    const size_t esz[3] = {4, 2, 2};
    for (int s = 0; s < 4; ++s) {
        if (!need[s]) continue;
        P->xp_off[s] = (int64_t)ws;
        const int64_t bytes = s < 3 ? (int64_t)P->Ppad * P->Kx * (int64_t)esz[s] : P->Kt * P->Pt * 4;
        ws += (size_t)round_up(bytes, 256);
    }
    // Temporaries T^(m-1) .. T^(1).
    for (int k = m - 1; k >= 1; --k) {
        const int d = m - 1 - k;
        const int64_t jt = binom(pbar + d, d + 1);
        const int64_t pf = binom(nbar + k - 1, k);
        int64_t blk = 1;
        for (int j = 0; j < m; ++j) blk *= (j < k ? bA : bC);
        if (jt < 0 || pf < 0 || blk <= 0) {
            *err = "temporary too large";
            return false;
        }
        const __int128 elems = (__int128)jt * pf * blk;
        const __int128 bytes = elems * (tdt[k] == F32 ? 4 : 2);
        if (bytes > ((__int128)1 << 46)) {
            *err = "temporary too large";
            return false;
        }
        P->temp_off[k] = (int64_t)ws;
        P->temp_dtype[k] = tdt[k];
        P->temp_jtuples[k] = jt;
        P->temp_prefixes[k] = pf;
        P->temp_block[k] = blk;
        ws += (size_t)round_up((int64_t)bytes, 256);
    }
    P->ws_bytes = ws;

    // Stages.
    P->stages.clear();
    P->flops = 0;
    for (int d = 0; d < m; ++d) {
        const int k = m - 1 - d;
        StagePlan S;
        S.d = d;
        S.k = k;
        S.compute = cmp[d];
        const int in_dt = d == 0 ? key.in_dtype : tdt[k + 1];
        const int out_dt = k == 0 ? F32 : tdt[k];
        if (cmp[d] == CMP_FP32 && in_dt != F32) { *err = "fp32 contraction needs fp32 input"; return false; }
        if (cmp[d] == CMP_X3 && in_dt != F32) { *err = "split contraction needs fp32 input"; return false; }

        int ext_in[kMaxOrder], ext_out[kMaxOrder];
        for (int j = 0; j < m; ++j) {
            ext_in[j] = j <= k ? bA : bC;
            ext_out[j] = j < k ? bA : bC;
        }
        int64_t gs[kMaxOrder], os[kMaxOrder];
        int64_t in_blk = 1, out_blk = 1;
        for (int j = 0; j < m; ++j) {
            gs[j] = in_blk;
            in_blk *= ext_in[j];
            os[j] = out_blk;
            out_blk *= ext_out[j];
        }
        if (in_blk > INT32_MAX / 2 || out_blk > INT32_MAX / 2) {
            *err = "block too large";
            return false;
        }
        const int Mblk = (int)(in_blk / ext_in[k]);

        StageArgs &a = S.args;
        a.m = m;
        a.k = k;
        a.nbar = nbar;
        a.bA = bA;
        a.bC = bC;
        a.Kpad = (int32_t)P->Kpad;
        a.Ppad = (int32_t)P->Ppad;
        a.Kx = (int32_t)P->Kx;
        a.Mblk = Mblk;
        a.in_f32 = in_dt == F32;
        a.out_f32 = out_dt == F32;
        const int KT = kt_of(cmp[d]);
        if (bA >= KT) {
            a.chunk_blocks = 1;
            a.chunk_k = KT;
            a.chunks_per_blk = (bA + KT - 1) / KT;
            a.nchunks = nbar * a.chunks_per_blk;
        } else {
            a.chunk_blocks = KT / bA;
            a.chunk_k = bA;
            a.chunks_per_blk = 1;
            a.nchunks = (nbar + a.chunk_blocks - 1) / a.chunk_blocks;
        }
        int nm = 0;
        for (int j = 0; j < m; ++j) {
            if (j == k) continue;
            a.mrad[nm] = ext_in[j];
            a.mmode[nm] = j;
            ++nm;
        }
        for (int i = nm; i < kMaxOrder; ++i) { a.mrad[i] = 1; a.mmode[i] = 0; }
        for (int q = 0; q <= k; ++q) {
            for (int j = 0; j < m; ++j) {
                int pos;
                if (j < k) pos = j < q ? j : j + 1;
                else if (j == k) pos = q;
                else pos = j;
                a.sq[q][j] = (int32_t)gs[pos];
            }
        }
        for (int j = 0; j < m; ++j) a.os[j] = (int32_t)os[j];
        for (int i = 0; i < kMaxOrder; ++i) a.mos[i] = i < m - 1 ? (int32_t)os[a.mmode[i]] : 0;
        a.osk = (int32_t)os[k];
        S.tile = key.grouped ? TileCfg{kGroupedMT, kGroupedNT, 2, 2} : choose_tile(Mblk);
        S.fast = fast[d];
        S.fast_bf16 = fast16[d];
        S.b64 = cmp[d] == CMP_BF16 && b64_bf16_supported(m, bA, bC, nbar, in_dt == BF16) && !key.generic_only &&
                !key.grouped;
        if (S.fast_bf16) {
            int tmt, tnt, tkt, tpd;
            bf16_fast_tile(bA, &tmt, &tnt, &tkt, &tpd);
            S.tile = TileCfg{tmt, tnt, 0, 0, tkt, tpd};
            int ont, okt, opd;
            if (!key.grouped && bf16_tile_override(d, &ont, &okt, &opd) && bf16_tile_supported(bA, ont, okt, opd))
                S.tile = TileCfg{tmt, ont, 0, 0, okt, opd};
            // The X-resident form takes the default b = 16 tile when the
            // input is bf16 and a whole X panel row fits its LDS slice, with
            // 96-column tiles (at m3_n256_b16 every level then has at most
            // 512 tasks, one per resident workgroup).  STTSM_BF16_XRES=0
            // keeps the chunk-staged kernel; "NTxPD" (NT 64, 96 or 128, PD
            // 2 or 4) picks another tile, for measurement.
            const char *xe = getenv("STTSM_BF16_XRES");
            int xnt = 96, xpd = 2;
            const bool xoff = xe && *xe && atoi(xe) == 0;
            if (xe && *xe && !xoff && sscanf(xe, "%dx%d", &xnt, &xpd) != 2) xnt = 96, xpd = 2;
            if ((xnt != 64 && xnt != 96 && xnt != 128) || (xpd != 2 && xpd != 4)) xnt = 96, xpd = 2;
            if (!key.grouped && !xoff && bf16_xres_supported(bA, (int)P->Kpad, in_dt == BF16) &&
                S.tile.NT == tnt && S.tile.KT == tkt && S.tile.PD == tpd) {
                S.tile.xres = true;
                S.tile.NT = xnt;
                S.tile.PD = xpd;
            }
        }
        for (int j = 0; j < m; ++j) {
            a.ext_in[j] = ext_in[j];
            a.gs[j] = (int32_t)gs[j];
        }
        a.xt_stride = (int32_t)P->Pt;
        // Row groups.
        const std::vector<int32_t> Jp = sorted_tuples(d, pbar);
        const int64_t nJp = d == 0 ? 1 : (int64_t)Jp.size() / d;
        const std::vector<int32_t> Ss = sorted_tuples(k, nbar);
        const int64_t nS = k == 0 ? 1 : (int64_t)Ss.size() / k;
        const int64_t npre_out = k == 0 ? 1 : binom(nbar + k - 1, k);
        const int64_t npre_in = binom(nbar + k, k + 1);
        if ((int64_t)nJp * nS > INT32_MAX || (int64_t)nJp * nS * nbar > INT32_MAX) {
            *err = "too many row groups";
            return false;
        }
        S.groups.reserve(nJp * nS);
        S.in_tab.reserve(nJp * nS * nbar);
        int32_t u[kMaxOrder];
        for (int64_t jp = 0; jp < nJp; ++jp) {
            const int32_t *J = d ? &Jp[jp * d] : nullptr;
            int64_t R = 0;   // colex rank of (jbar, J') minus jbar
            for (int i = 1; i <= d; ++i) R += binom((int64_t)J[i - 1] + i, i + 1);
            const int64_t rJ = d ? colex_rank(J, d) : 0;
            const int jcount = d == 0 ? pbar : J[0] + 1;
            for (int64_t si = 0; si < nS; ++si) {
                const int32_t *s = k ? &Ss[si * k] : nullptr;
                const int64_t rs = k ? colex_rank(s, k) : 0;
                GroupDesc g;
                g.out_base = (R * npre_out + rs) * out_blk;
                g.out_jstride = npre_out * out_blk;
                g.jcount = jcount;
                g.in_row = (int32_t)S.in_tab.size();
                S.groups.push_back(g);
                for (int ib = 0; ib < nbar; ++ib) {
                    int q = 0;
                    while (q < k && s[q] <= ib) ++q;
                    for (int i = 0; i < q; ++i) u[i] = s[i];
                    u[q] = ib;
                    for (int i = q; i < k; ++i) u[i + 1] = s[i];
                    InEntry e;
                    e.off = (rJ * npre_in + colex_rank(u, k + 1)) * in_blk;
                    e.q = q;
                    e.pad_ = 0;
                    S.in_tab.push_back(e);
                }
                S.flops += 2 * P->Kpad * (int64_t)Mblk * jcount * bC;
            }
        }
        // Generic kernel, narrow row groups (few output columns, as in the
        // levels below the first and whenever p is small): 32-column tiles
        // when they cut the padded columns by a quarter or more.
        if (!key.grouped && !S.fast && !S.fast_bf16 && Mblk > 64) {
            int64_t c32 = 0, c64 = 0;
            for (const GroupDesc &g : S.groups) {
                const int64_t N = (int64_t)g.jcount * bC;
                c32 += (N + 31) / 32 * 32;
                c64 += (N + 63) / 64 * 64;
            }
            if (4 * c32 <= 3 * c64) {
                // 128 rows: half the LDS of a 256-row tile, so twice the
                // workgroups per CU (m4_n64_b8 FP32 146 -> 125 us).
                S.tile = TileCfg{128, 32, 4, 1};
                const char *e = getenv("STTSM_NARROW_MT");   // measurement override: 256 rows
                if (e && atoi(e) == 256 && Mblk > 128) S.tile.MT = 256;
            }
        }
        if (S.fast) {
            // Tile of the block-copy kernel.  Below the first level a tile may
            // take half a block row (split along mode m-1, contiguous in
            // storage) when a half block still holds >= 256 float4.
            const bool can_half = k < m - 1 && bC % 2 == 0 && bA >= 8;
            // Measured on m=3, n=p=256, b=16: a whole block row with 64
            // columns for the first level, half rows with 128 columns for
            // middle levels, and half rows with 32 columns and loads two
            // chunks ahead for the last.  The four waves always split the
            // rows (WM = 4, WN = 1).
            S.tile = TileCfg{256, 64, 4, 1, 16, 1};
            if (can_half) S.tile = k == 0 ? TileCfg{128, 32, 4, 1, 16, 2} : TileCfg{128, 128, 4, 1, 16, 1};
            int tmt, tnt, tkt, tpd;
            if (fast_tile_override(d, &tmt, &tnt, &tkt, &tpd) && fast_tile_supported(tmt, tnt, tkt, tpd) &&
                (tmt == 256 || can_half) && tkt % bA == 0)
                S.tile = TileCfg{tmt, tnt, 4, 1, tkt, tpd};
            a.chunk_blocks = S.tile.KT / bA;
            a.chunk_k = bA;
            a.chunks_per_blk = 1;
            a.nchunks = (nbar + a.chunk_blocks - 1) / a.chunk_blocks;
            const int RS = S.tile.MT + 4;
            int64_t ms[kMaxOrder] = {};
            int64_t pv = 1;
            for (int j = 0; j < m; ++j) {
                if (j == k) continue;
                ms[j] = pv;
                pv *= ext_in[j];
            }
            for (int q = 0; q < kMaxOrder; ++q)
                for (int i = 0; i < kMaxOrder; ++i) a.lds[q][i] = 0;
            for (int q = 0; q <= k; ++q)
                for (int i = 0; i < m; ++i) {
                    int j;   // logical mode at stored position i
                    if (i < q) j = i;
                    else if (i == q) j = k;
                    else if (i <= k) j = i - 1;
                    else j = i;
                    a.lds[q][i] = j == k ? RS : (int32_t)ms[j];
                }
            // Above the last level the kernel's epilogue stores four output
            // rows at once: mode 0 must be the first row digit, with output
            // stride 1 and an extent that is a multiple of 4.
            if (k != 0 && (a.mmode[0] != 0 || a.mos[0] != 1 || a.mrad[0] % 4 != 0)) {
                *err = "block-copy epilogue: rows not in runs of four";
                return false;
            }
            // The kernel relies on stored position 0 having LDS stride RS for
            // q = 0 and 1 otherwise.
            for (int q = 0; q <= k; ++q)
                if (a.lds[q][0] != (q == 0 ? RS : 1)) {
                    *err = "block-copy staging: unexpected stride of stored position 0";
                    return false;
                }
            // Per-thread stored digits of the float4 each thread copies.
            const int MT = S.tile.MT, NF = MT * S.tile.KT / 1024, sub4 = MT * bA / 4;
            const int mt_count = Mblk / MT;
            S.fdig.assign((size_t)mt_count * NF * m * 256, 0);
            for (int mt = 0; mt < mt_count; ++mt)
                for (int f = 0; f < NF; ++f)
                    for (int t = 0; t < 256; ++t) {
                        const int F = t + 256 * f, gq = (256 * f) / sub4;
                        int r = mt * MT * bA + 4 * (F - gq * sub4);
                        for (int i = 0; i < m; ++i) {
                            S.fdig[(((size_t)mt * NF + f) * m + i) * 256 + t] = r % ext_in[i];
                            r /= ext_in[i];
                        }
                    }
            S.zero.assign((size_t)in_blk, 0.f);
            // Output offset of every block row.
            S.fopart.assign(Mblk, 0);
            for (int row = 0; row < Mblk; ++row) {
                int r = row, op = 0;
                for (int i = 0; i < m - 1; ++i) {
                    op += (r % a.mrad[i]) * a.mos[i];
                    r /= a.mrad[i];
                }
                S.fopart[row] = op;
            }
        }
        if (S.b64) {
            // Tiles of four consecutive row groups (their rows stacked) and
            // NT columns up to the largest of their column counts.  NT: the
            // fewest resident rounds times the tile width (ties: wider).
            const int ng = (int)S.groups.size();
            auto count = [&](int nt) {
                int64_t c = 0;
                for (int g = 0; g < ng; g += 4) {
                    int jmax = 0;
                    for (int i = g; i < std::min(ng, g + 4); ++i) jmax = std::max(jmax, S.groups[i].jcount);
                    c += (jmax * bC + nt - 1) / nt;
                }
                return c;
            };
            int best = 256;
            int64_t best_cost = INT64_MAX;
            for (int nt : {256, 192, 128}) {
                const int64_t cost = (count(nt) + cus - 1) / cus * nt;
                if (cost < best_cost) best = nt, best_cost = cost;
            }
            S.tile = TileCfg{256, best, 4, 2, 64, 2};
            for (int g = 0; g < ng; g += 4) {
                const int cnt = std::min(4, ng - g);
                int jmax = 0;
                for (int i = g; i < g + cnt; ++i) jmax = std::max(jmax, S.groups[i].jcount);
                const int N = jmax * bC;
                for (int nt = 0; nt * best < N; ++nt)
                    S.tasks.push_back(Task{g, (int16_t)cnt, (int16_t)nt, 0, (int16_t)std::min(best, N - nt * best)});
            }
        }
        // Tasks.
        const int mtiles = S.b64 ? 0 : (Mblk + S.tile.MT - 1) / S.tile.MT;
        for (int32_t gi = 0; gi < (int32_t)S.groups.size() && !S.b64; ++gi) {
            const int N = S.groups[gi].jcount * bC;
            const int ntiles = (N + S.tile.NT - 1) / S.tile.NT;
            for (int mt = 0; mt < mtiles; ++mt)
                for (int nt = 0; nt < ntiles; ++nt)
                    S.tasks.push_back(Task{gi, (int16_t)mt, (int16_t)nt, 0, (int16_t)std::min(S.tile.NT, N - nt * S.tile.NT)});
        }
        // Workgroups of the FP32 block-copy kernel a CU holds at once (LDS
        // and registers of the instantiated tiles: three for 256-row or
        // 128-column tiles, four or more for the narrower ones).
        const int per_cu = S.tile.MT == 256 || S.tile.NT >= 128 ? 3 : 4;
        if (S.fast && S.tasks.size() <= (size_t)per_cu * cus) {
            // Every tile of the level is resident at once, so the order only
            // decides which CU runs which tile: balance the CUs.  Work of a tile: MFMAs in whole
            // 32-column subtiles, plus staging that does not shrink with the
            // columns.  Only the FP32 block-copy kernel reads noff / ncol
            // (so only it may split).
            const int MT = S.tile.MT;
            order_tasks_for_xcds(&S.tasks, [&](const Task &t) -> int64_t {
                return (int64_t)std::min(MT, Mblk - t.mt * MT) * ((t.ncol + 31) / 32 * 32 + 16);
            }, std::max(cus / 8, 1), true);
        } else if (S.b64 && d == 0) {
            // First level: tiles in blocks of 4 tile rows x 8 tile columns,
            // each block on one XCD, which then reads 4 tile rows of A and 8
            // column slices of X (at n = p = 4096: 24 MB per XCD against
            // 36 MB with whole tile rows per XCD; fetch 302 -> 186 MB, level
            // 0 about 3% faster).  The second level's triangular tile grid
            // keeps whole tile rows per XCD (blocks fetched more there).
            order_tasks_by_task_key(&S.tasks, [](const Task &t) {
                return (int64_t)(t.group / 16) * 65536 + t.nt / 8;
            });
        } else if (S.tile.xres && key.xres_records) {
            // Locality key of a row group: below the first level the groups
            // of one C-block tuple J' read only that tuple's slab of the
            // input temporary; at the first level a stored A block is read
            // by the prefixes it contains, whose largest indices take at
            // most two values, so the key is the prefix's largest index.
            std::vector<int64_t> key_of(S.groups.size());
            for (int64_t jp = 0; jp < nJp; ++jp)
                for (int64_t si = 0; si < nS; ++si)
                    key_of[jp * nS + si] = d > 0 ? jp : (k > 0 ? Ss[si * k + k - 1] : 0);
            order_tasks_by_key(&S.tasks, key_of);
        } else {
            order_tasks_group_major(&S.tasks);
        }
        if (mtiles > 32767 || (int64_t)P->Ppad / S.tile.NT > 32767 || S.tasks.size() > (size_t)INT32_MAX) {
            *err = "too many tasks";
            return false;
        }
        if (S.tile.xres && key.xres_records) {
            // One record per task, in the final task order.
            if (nbar > 16) {
                *err = "X-resident kernel: more than 16 input blocks";
                return false;
            }
            S.xrec.resize(S.tasks.size());
            for (size_t t = 0; t < S.tasks.size(); ++t) {
                const Task &tk = S.tasks[t];
                const GroupDesc &g = S.groups[tk.group];
                XresRec r{};
                for (int i = 0; i < nbar; ++i) {
                    const InEntry &e = S.in_tab[(size_t)g.in_row + i];
                    r.off[i] = e.off;
                    r.q_bits |= (e.q & 3) << (2 * i);
                }
                r.out_base = g.out_base;
                r.out_jstride = g.out_jstride;
                r.n0 = tk.nt * S.tile.NT;
                r.mt = tk.mt;
                r.jcount = g.jcount;
                S.xrec[t] = r;
            }
        }
        a.ntasks = (int32_t)S.tasks.size();
        S.in_ws = d == 0 ? -1 : P->temp_off[k + 1];
        S.out_ws = k == 0 ? -1 : P->temp_off[k];
        S.out_elems = k == 0 ? 0 : P->temp_jtuples[k] * P->temp_prefixes[k] * P->temp_block[k];
        if (cmp[d] == CMP_FP32) { S.xp_slot = S.fast ? 3 : 0; S.xp_lo_slot = -1; }
        else if (cmp[d] == CMP_BF16) { S.xp_slot = 1; S.xp_lo_slot = -1; }
        else { S.xp_slot = 1; S.xp_lo_slot = 2; }
        P->flops += S.flops;
        P->stages.push_back(std::move(S));
    }
    return true;
}

template <class T>
static bool upload(const std::vector<T> &v, T **dst, std::string *err);
template <class T>
static bool upload_vec(const std::vector<T> &v, T **dst, std::string *err)
{
    return upload(v, dst, err);
}
template <class T>
static bool upload(const std::vector<T> &v, T **dst, std::string *err)
{
    *dst = nullptr;
    if (v.empty()) return true;
    if (hipMalloc((void **)dst, v.size() * sizeof(T)) != hipSuccess) {
        *err = "hipMalloc failed for plan tables";
        *dst = nullptr;
        return false;
    }
    if (hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        *err = "hipMemcpy failed for plan tables";
        return false;
    }
    return true;
}

struct DevKey {
    int dev;
    PlanKey k;
    bool operator<(const DevKey &o) const { return dev != o.dev ? dev < o.dev : k < o.k; }
};

static std::mutex g_plan_mu;
static std::map<DevKey, std::unique_ptr<Plan>> g_plans;

const Plan *plan_get(const PlanKey &key, std::string *err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = "hipGetDevice failed";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_plan_mu);
    DevKey dk{dev, key};
    auto it = g_plans.find(dk);
    if (it != g_plans.end()) return it->second.get();
    std::unique_ptr<Plan> P(new Plan);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (!plan_build_host(key, P.get(), err, cus)) return nullptr;
    for (auto &S : P->stages) {
        if (!upload(S.groups, &S.d_groups, err) || !upload(S.in_tab, &S.d_in_tab, err) ||
            !upload(S.tasks, &S.d_tasks, err) || !upload(S.fdig, &S.d_fdig, err) ||
            !upload(S.fopart, &S.d_fopart, err) || !upload(S.zero, &S.d_zero, err) ||
            !upload(S.xrec, &S.d_xrec, err))
            return nullptr;   // tables of a failed plan are leaked, never used
        S.args.xrec = S.d_xrec;
        S.args.zero_blk = S.d_zero;
        S.args.fdig = S.d_fdig;
        S.args.fopart = S.d_fopart;
        S.args.groups = S.d_groups;
        S.args.in_tab = S.d_in_tab;
        S.args.tasks = S.d_tasks;
    }
    const Plan *out = P.get();
    g_plans.emplace(dk, std::move(P));
    return out;
}

static std::map<DevKey, std::unique_ptr<Plan>> g_host_plans;

template <class T>
static int64_t pack_table(const std::vector<T> &v, std::vector<unsigned char> *blob)
{
    if (v.empty()) return -1;
    const size_t off = (blob->size() + 255) & ~(size_t)255;
    blob->resize(off + v.size() * sizeof(T));
    memcpy(blob->data() + off, v.data(), v.size() * sizeof(T));
    return (int64_t)off;
}

const Plan *plan_get_host(const PlanKey &key, std::string *err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = "hipGetDevice failed";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_plan_mu);
    DevKey dk{dev, key};
    auto it = g_host_plans.find(dk);
    if (it != g_host_plans.end()) return it->second.get();
    std::unique_ptr<Plan> P(new Plan);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (!plan_build_host(key, P.get(), err, cus)) return nullptr;
    for (auto &S : P->stages) {
        TabOff t;
        t.groups = pack_table(S.groups, &P->tab_blob);
        t.in_tab = pack_table(S.in_tab, &P->tab_blob);
        t.tasks = pack_table(S.tasks, &P->tab_blob);
        t.fdig = pack_table(S.fdig, &P->tab_blob);
        t.fopart = pack_table(S.fopart, &P->tab_blob);
        t.zero = pack_table(S.zero, &P->tab_blob);
        t.xrec = pack_table(S.xrec, &P->tab_blob);
        P->tab_off.push_back(t);
    }
    P->tab_blob.resize((P->tab_blob.size() + 255) & ~(size_t)255);
    const Plan *out = P.get();
    g_host_plans.emplace(dk, std::move(P));
    return out;
}

// ------------------------------------------------------------------ meta table
struct MetaKey {
    int dev, m, nbar, b;
    bool operator<(const MetaKey &o) const
    {
        if (dev != o.dev) return dev < o.dev;
        if (m != o.m) return m < o.m;
        if (nbar != o.nbar) return nbar < o.nbar;
        return b < o.b;
    }
};
static std::map<MetaKey, std::unique_ptr<MetaTable>> g_meta;

const MetaTable *meta_get(int m, int nbar, int b, std::string *err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = "hipGetDevice failed";
        return nullptr;
    }
    int64_t total = 1;
    for (int j = 0; j < m; ++j) {
        total *= nbar;
        if (total > (1 << 24)) {
            *err = "meta-data tensor too large (nbar^m > 2^24)";
            return nullptr;
        }
    }
    std::lock_guard<std::mutex> lock(g_plan_mu);
    MetaKey key{dev, m, nbar, b};
    auto it = g_meta.find(key);
    if (it != g_meta.end()) return it->second.get();
    std::unique_ptr<MetaTable> T(new MetaTable);
    T->m = m;
    T->nbar = nbar;
    T->b = b;
    T->tuples = sorted_tuples(m, nbar);
    T->rank.resize(total);
    T->perm.resize(total);
    std::map<std::vector<int>, int> perm_ids;
    int64_t bpow[kMaxOrder];
    bpow[0] = 1;
    for (int j = 1; j < m; ++j) bpow[j] = bpow[j - 1] * b;
    int32_t t[kMaxOrder], u[kMaxOrder];
    std::vector<int> sigma(m);
    for (int64_t f = 0; f < total; ++f) {
        int64_t r = f;
        for (int j = 0; j < m; ++j) { t[j] = (int32_t)(r % nbar); r /= nbar; }
        for (int j = 0; j < m; ++j) sigma[j] = j;
        std::stable_sort(sigma.begin(), sigma.end(), [&](int x, int y) { return t[x] < t[y]; });
        for (int j = 0; j < m; ++j) u[j] = t[sigma[j]];
        T->rank[f] = colex_rank(u, m);
        // logical mode sigma[i] sits at stored position i
        std::vector<int> pos(m);
        for (int i = 0; i < m; ++i) pos[sigma[i]] = i;
        auto ins = perm_ids.emplace(pos, (int)perm_ids.size());
        if (ins.second)
            for (int j = 0; j < m; ++j) T->perm_strides.push_back((int32_t)bpow[pos[j]]);
        T->perm[f] = ins.first->second;
    }
    const int64_t nblk = (int64_t)T->tuples.size() / m;
    for (int64_t r = 0; r < nblk; ++r) {
        int mask = 0;
        for (int j = 0; j + 1 < m; ++j) mask |= (T->tuples[r * m + j] == T->tuples[r * m + j + 1] ? 1 : 0) << j;
        if (mask) {
            T->rep_blocks.push_back((int32_t)r);
            T->rep_masks.push_back((uint8_t)mask);
        }
    }
    if (!upload(T->rank, &T->d_rank, err) || !upload(T->perm, &T->d_perm, err) ||
        !upload(T->perm_strides, &T->d_perm_strides, err) || !upload(T->tuples, &T->d_tuples, err) ||
        !upload(T->rep_blocks, &T->d_rep_blocks, err) || !upload(T->rep_masks, &T->d_rep_masks, err))
        return nullptr;
    const MetaTable *out = T.get();
    g_meta.emplace(key, std::move(T));
    return out;
}

namespace {
std::map<std::pair<int, int>, std::unique_ptr<StabTable>> g_stab;   // (device, m)
}

const StabTable *stab_get(int m, std::string *err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = "hipGetDevice failed";
        return nullptr;
    }
    if (m < 1 || m > kMaxOrder) {
        *err = "bad order";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_plan_mu);
    auto it = g_stab.find({dev, m});
    if (it != g_stab.end()) return it->second.get();
    std::unique_ptr<StabTable> T(new StabTable);
    T->m = m;
    const int nmask = 1 << (m - 1);
    for (int mask = 0; mask < nmask; ++mask) {
        // run id of every position
        int run[kMaxOrder];
        run[0] = 0;
        for (int j = 1; j < m; ++j) run[j] = run[j - 1] + (((mask >> (j - 1)) & 1) ? 0 : 1);
        T->start.push_back((int32_t)(T->perm.size() / m));
        std::vector<int> pi(m);
        for (int j = 0; j < m; ++j) pi[j] = j;
        do {
            bool keep = true;
            for (int j = 0; j < m && keep; ++j) keep = run[pi[j]] == run[j];
            if (keep) {
                int32_t inv[kMaxOrder] = {};
                for (int j = 0; j < m; ++j) {
                    T->perm.push_back((uint8_t)pi[j]);
                    inv[pi[j]] = j;
                }
                T->pinv.insert(T->pinv.end(), inv, inv + kMaxOrder);
            }
        } while (std::next_permutation(pi.begin(), pi.end()));
    }
    T->start.push_back((int32_t)(T->perm.size() / m));
    if (!upload(T->start, &T->d_start, err) || !upload(T->perm, &T->d_perm, err) || !upload(T->pinv, &T->d_pinv, err))
        return nullptr;
    const StabTable *out = T.get();
    g_stab.emplace(std::make_pair(dev, m), std::move(T));
    return out;
}

namespace {
std::map<std::tuple<int, int, int, int, bool>, std::unique_ptr<VecPlan>> g_vec;   // (device, m, nbar, b, upload)
}

bool rank_plan_build_host(const Plan &P, int rows, RankPlan *R, std::string *err)
{
    const int m = P.m;
    if (m < 2 || (int)P.stages.size() != m) {
        *err = "the rank-update form needs m >= 2";
        return false;
    }
    for (const StagePlan &S : P.stages)
        if (S.fast || S.fast_bf16) {
            *err = "the rank-update form runs on the generic kernels";
            return false;
        }
    if (rows < 1) {
        *err = "rows per pass must be >= 1";
        return false;
    }
    const int nbar = P.nbar;
    const int S = std::min(rows, nbar);
    const StagePlan &L = P.stages[m - 2];   // contracts mode 1, writes T^(1)
    const StagePlan &U = P.stages[m - 1];   // contracts mode 0, writes C
    const int64_t blk = P.temp_block[1];    // a T^(1) block: bA * bC^(m-1) entries
    const int esz = P.temp_dtype[1] == F32 ? 4 : 2;
    R->rows = S;
    R->passes.clear();
    // T^(1) is the last region of the chain's workspace; the pass buffer
    // takes its place.
    R->buf_off = P.temp_off[1];
    R->buf_elems = P.temp_jtuples[1] * S * blk;
    R->ws_bytes = (size_t)R->buf_off + (size_t)round_up(R->buf_elems * esz, 256);
    for (int a0 = 0; a0 < nbar; a0 += S) {
        const int Sc = std::min(S, nbar - a0);
        RankPass ps;
        ps.k_begin = (int64_t)a0 * P.bA;
        // Row level.  Its groups are (trailing tuple, prefix i0), numbered
        // jp * nbar + i0, with T^(1) block (jrank, i0) at (jrank * nbar + i0)
        // blocks; in the pass buffer it sits at (jrank * Sc + i0 - a0).
        StagePlan &row = ps.row;
        row.d = L.d;
        row.k = L.k;
        row.compute = L.compute;
        row.tile = L.tile;
        row.args = L.args;
        row.in_ws = L.in_ws;
        row.xp_slot = L.xp_slot;
        row.xp_lo_slot = L.xp_lo_slot;
        std::vector<int32_t> remap(L.groups.size(), -1);
        for (size_t gi = 0; gi < L.groups.size(); ++gi) {
            const int i0 = (int)(gi % nbar);
            if (i0 < a0 || i0 >= a0 + Sc) continue;
            GroupDesc g = L.groups[gi];
            const int64_t jr = (g.out_base / blk - i0) / nbar;
            if ((jr * nbar + i0) * blk != g.out_base || g.out_jstride != (int64_t)nbar * blk) {
                *err = "rank-update form: unexpected layout of T^(1)";
                return false;
            }
            g.out_base = (jr * Sc + (i0 - a0)) * blk;
            g.out_jstride = (int64_t)Sc * blk;
            remap[gi] = (int32_t)row.groups.size();
            row.groups.push_back(g);
            row.flops += 2 * P.Kpad * (int64_t)L.args.Mblk * g.jcount * P.bC;
        }
        for (const Task &t : L.tasks) {
            if (remap[t.group] < 0) continue;
            Task u = t;
            u.group = remap[t.group];
            row.tasks.push_back(u);
        }
        row.args.ntasks = (int32_t)row.tasks.size();
        // Update level: every C group, its input table cut to the pass's
        // contracted blocks a0 .. a0+Sc-1 and rebased onto the pass buffer;
        // X is read from column k_begin on.
        StagePlan &upd = ps.upd;
        upd.d = U.d;
        upd.k = U.k;
        upd.compute = U.compute;
        upd.tile = U.tile;
        upd.args = U.args;
        upd.xp_slot = U.xp_slot;
        upd.xp_lo_slot = U.xp_lo_slot;
        for (const GroupDesc &g0 : U.groups) {
            GroupDesc g = g0;
            g.in_row = (int32_t)upd.in_tab.size();
            upd.groups.push_back(g);
            for (int ib = a0; ib < a0 + Sc; ++ib) {
                InEntry e = U.in_tab[(size_t)g0.in_row + ib];
                const int64_t jr = (e.off / blk - ib) / nbar;
                if ((jr * nbar + ib) * blk != e.off || e.q != 0) {
                    *err = "rank-update form: unexpected layout of T^(1)";
                    return false;
                }
                e.off = (jr * Sc + (ib - a0)) * blk;
                upd.in_tab.push_back(e);
            }
            upd.flops += 2 * (int64_t)Sc * P.bA * U.args.Mblk * g.jcount * P.bC;
        }
        upd.tasks = U.tasks;
        StageArgs &ua = upd.args;
        ua.nbar = Sc;
        ua.Kpad = Sc * P.bA;
        ua.nchunks = ua.chunk_blocks > 1 ? (Sc + ua.chunk_blocks - 1) / ua.chunk_blocks : Sc * ua.chunks_per_blk;
        ua.accumulate = a0 > 0;
        ua.ntasks = (int32_t)upd.tasks.size();
        R->passes.push_back(std::move(ps));
    }
    return true;
}

struct RankKey {
    DevKey dk;
    int rows;
    bool operator<(const RankKey &o) const { return rows != o.rows ? rows < o.rows : dk < o.dk; }
};
static std::map<RankKey, std::unique_ptr<RankPlan>> g_rank;

const RankPlan *rank_plan_get(const PlanKey &key0, int rows, std::string *err)
{
    PlanKey key = key0;
    key.generic_only = true;
    key.grouped = false;
    const Plan *P = plan_get(key, err);
    if (!P) return nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *err = "hipGetDevice failed";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_plan_mu);
    const RankKey rk{DevKey{dev, key}, std::max(std::min(rows, P->nbar), 0)};   // rows >= nbar: one pass
    auto it = g_rank.find(rk);
    if (it != g_rank.end()) return it->second.get();
    std::unique_ptr<RankPlan> R(new RankPlan);
    if (!rank_plan_build_host(*P, rows, R.get(), err)) return nullptr;
    R->chain = P;
    const StagePlan &L = P->stages[P->m - 2];
    for (RankPass &ps : R->passes) {
        if (!upload(ps.row.groups, &ps.row.d_groups, err) || !upload(ps.row.tasks, &ps.row.d_tasks, err) ||
            !upload(ps.upd.groups, &ps.upd.d_groups, err) || !upload(ps.upd.in_tab, &ps.upd.d_in_tab, err) ||
            !upload(ps.upd.tasks, &ps.upd.d_tasks, err))
            return nullptr;   // tables of a failed plan are leaked, never used
        ps.row.args.groups = ps.row.d_groups;
        ps.row.args.in_tab = L.d_in_tab;   // the row level reads T^(2) (or A) as the chain does
        ps.row.args.tasks = ps.row.d_tasks;
        ps.upd.args.groups = ps.upd.d_groups;
        ps.upd.args.in_tab = ps.upd.d_in_tab;
        ps.upd.args.tasks = ps.upd.d_tasks;
    }
    const RankPlan *out = R.get();
    g_rank.emplace(rk, std::move(R));
    return out;
}

const VecPlan *vec_plan_get(int m, int nbar, int b, bool upload, std::string *err)
{
    int dev = 0;
    if (upload && hipGetDevice(&dev) != hipSuccess) {
        *err = "hipGetDevice failed";
        return nullptr;
    }
    if (m < 2 || m > kMaxOrder || nbar < 1 || b < 1) {
        *err = "bad shape";
        return nullptr;
    }
    const int64_t nblocks = binom((int64_t)nbar + m - 1, m);
    if (nblocks < 0 || nblocks > (int64_t)INT32_MAX / kMaxOrder) {
        *err = "too many blocks";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_plan_mu);
    const auto key = std::make_tuple(upload ? dev : -1, m, nbar, b, upload);
    auto it = g_vec.find(key);
    if (it != g_vec.end()) return it->second.get();
    std::unique_ptr<VecPlan> P(new VecPlan);
    P->m = m;
    P->nbar = nbar;
    P->b = b;
    int64_t bm = 1;
    for (int j = 0; j < m; ++j) bm *= b;
    const std::vector<int32_t> tuples = sorted_tuples(m, nbar);
    // factorials for the multinomial weights
    double fact[kMaxOrder + 1];
    fact[0] = 1;
    for (int i = 1; i <= kMaxOrder; ++i) fact[i] = fact[i - 1] * i;
    std::vector<std::vector<VecEntry>> per_u(nbar);
    for (int64_t r = 0; r < nblocks; ++r) {
        const int32_t *s = &tuples[r * m];
        for (int q = 0; q < m; ++q) {
            if (q > 0 && s[q] == s[q - 1]) continue;   // first position of each distinct index
            // (m-1)! / prod over values of (count after removing one s[q])!
            double w = fact[m - 1];
            int i = 0;
            while (i < m) {
                int j = i;
                while (j < m && s[j] == s[i]) ++j;
                const int cnt = (j - i) - (s[i] == s[q] ? 1 : 0);
                w /= fact[cnt];
                i = j;
            }
            VecEntry e{};
            e.r = (int32_t)r;
            e.q = q;
            e.w = (float)w;
            for (int k = 0; k < m; ++k) e.s[k] = s[k];
            per_u[s[q]].push_back(e);
            P->terms += bm;
        }
    }
    P->u_chunk.push_back(0);
    for (int u = 0; u < nbar; ++u) {
        const std::vector<VecEntry> &L = per_u[u];
        for (size_t i = 0; i < L.size(); i += kVecChunk) {
            P->chunk_begin.push_back((int32_t)P->entries.size() + (int32_t)i);
            P->chunk_u.push_back(u);
        }
        P->entries.insert(P->entries.end(), L.begin(), L.end());
        P->u_chunk.push_back((int32_t)P->chunk_u.size());
    }
    P->chunk_begin.push_back((int32_t)P->entries.size());
    P->block_major = m == 3 && (b == 4 || b == 8 || b == 16);
    if (P->block_major) {
        P->u_entry.push_back(0);
        for (int u = 0; u < nbar; ++u) P->u_entry.push_back(P->u_entry.back() + (int32_t)per_u[u].size());
        std::vector<std::vector<int32_t>> per_r(nblocks);
        for (size_t e = 0; e < P->entries.size(); ++e) per_r[P->entries[e].r].push_back((int32_t)e);
        P->blk_begin.push_back(0);
        for (int64_t r = 0; r < nblocks; ++r) {
            P->blk_terms.insert(P->blk_terms.end(), per_r[r].begin(), per_r[r].end());
            P->blk_begin.push_back((int32_t)P->blk_terms.size());
        }
    }
    if (upload && (!upload_vec(P->entries, &P->d_entries, err) || !upload_vec(P->chunk_begin, &P->d_chunk_begin, err) ||
                   !upload_vec(P->chunk_u, &P->d_chunk_u, err) || !upload_vec(P->u_chunk, &P->d_u_chunk, err) ||
                   !upload_vec(P->blk_begin, &P->d_blk_begin, err) || !upload_vec(P->blk_terms, &P->d_blk_terms, err) ||
                   !upload_vec(P->u_entry, &P->d_u_entry, err)))
        return nullptr;
    const VecPlan *out = P.get();
    g_vec.emplace(key, std::move(P));
    return out;
}

}  // namespace symt
