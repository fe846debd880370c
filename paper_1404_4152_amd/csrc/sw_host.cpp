// Host side of libswmi: the C ABI declared in include/swmi.h.
//
// Database open (section III, stage ii and the offline index): subjects are
// stable-sorted by ascending length.  Short subjects are dealt into groups of
// 128 (64 lanes x 2 packed halves) laid out interleaved for coalesced wave
// loads, padded with a residue code that scores 0 (section III.B.1).  The
// longest subjects, which would hold one lane for too long, form a long list
// served wave-per-pair (inside the lane-per-subject kernel's work queue when
// it runs in int32), as does any database too small to fill the GPU
// lane-per-subject.
//
// Search (stages i and iv): build the query profile (section III.B.2; row r
// holds the scores of the whole query against residue r), run the kernels,
// recompute flagged narrow-tier pairs exactly, then sort or select the scores.
// Batches of queries share one persistent launch (captured once per shape in
// a HIP graph); the server keeps the database resident and coalesces the
// requests in flight into shared passes over database chunks.
//
// Alignment with traceback (sw_db_align): the optimal local alignments of one
// query against chosen database sequences, computed on the GPU with one
// direction byte per cell and a walk back.
#include <fcntl.h>
#include <hip/hip_runtime.h>
#include <sys/mman.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/swmi.h"
#include "sw_internal.h"
#include "sw_sched.h"

using namespace swmi;

static_assert(kNoAllocScratchBytes == (size_t)SW_NOALLOC_SCRATCH_BYTES, "scratch size");

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPX(expr)                                                                   \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            return fail(SW_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

#define TRY(expr)                     \
    do {                              \
        int rc_ = (expr);             \
        if (rc_ != SW_OK) return rc_; \
    } while (0)

double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Grow-only device buffer.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    int reserve(size_t want) {
        if (want <= bytes) return SW_OK;
        release();
        if (want == 0) return SW_OK;
        if (getenv("SWMI_FAIL_ALLOC")) return fail(SW_ENOMEM, "device allocation refused (SWMI_FAIL_ALLOC)");
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return fail(SW_ENOMEM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
        }
        bytes = want;
        return SW_OK;
    }
    template <class T> T *as() const { return (T *)p; }
};

// Grow-only pinned host buffer.
struct HostBuf {
    void *p = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf() {
        if (p) (void)hipHostFree(p);
    }
    int reserve(size_t want) {
        if (want <= bytes) return SW_OK;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(SW_ENOMEM, "hipHostMalloc(%zu) failed", want);
        }
        bytes = want;
        return SW_OK;
    }
    template <class T> T *as() const { return (T *)p; }
};

struct Plan {
    int tier = TIER_F16X2;
    int strip = 32;
    int waves = 4;
    int thr = kThrF16;
    int profile = SW_PROFILE_PAIR;
};

constexpr int kIntraWaves = 4;
constexpr size_t kResHead = 64;   // bytes of pass counters ahead of the top-k results   // waves per workgroup of the wave-per-pair kernel (long list)
// Subjects longer than this never go into a lane-per-subject group: one lane
// would hold its SIMD too long and its boundary buffer would be large.
constexpr int64_t kGroupMaxLen = 8192;

int intra_T_for(int64_t max_qlen) {
    if (max_qlen <= 256) return 4;
    if (max_qlen <= 512) return 8;
    return 16;
}

// Query columns a wave-per-pair pass evaluates for a query: whole passes of
// 64 x ti columns, except that the packed kernel at 16 columns per lane runs
// its last pass at 4, 8 or 12 when those hold the rest.
int64_t long_columns(int64_t qlen, int ti, bool packed) {
    const int64_t pw = 64LL * ti;
    if (!packed || ti != 16) return round_up(qlen, pw);
    const int64_t full = (qlen - 1) / pw, rem = qlen - full * pw;
    return full * pw + (rem <= 256 ? 256 : rem <= 512 ? 512 : rem <= 768 ? 768 : 1024);
}

int qlen_bucket(int64_t qlen) {
    int b = 0;
    while ((64LL << b) < qlen && b < 20) ++b;
    return b;
}

// The autotuner's entry for launches of several queries at once.
constexpr int kBatchBucket = -1;

// Work item lists of one device pass, built on the host.
struct Items {
    std::vector<int32_t> inter_q, inter_g;   // lane-per-subject: (slot, first group of block)
    std::vector<int32_t> intra_q, intra_ids; // wave-per-pair: (slot, per_item subject ids)
    int per_item = kIntraWaves;              // subjects per wave-per-pair item
    bool fused = false;                      // wave-per-pair items run in the lane-per-subject kernel
};

// Subjects per wave of the wave-per-pair kernel: two packed fp16 halves when
// there are enough pairs to keep every SIMD busy with half as many waves, one
// exact int32 alignment otherwise (and in the int16 plan).  Below that count
// the longest pair sets the makespan either way and the int32 kernel measured
// as fast or faster (one query against 2M subjects: ~2,200 long pairs).
// all_long: the launch has no lane-per-subject work (a small database, or a
// server pass at the long list's scan position); ti: its columns per lane.
int intra_per_wave(const Plan &plan, int64_t pairs, int cus, bool all_long = false, int ti = 16) {
    if (plan.tier != TIER_F16X2) return 1;
    if (pairs >= 32LL * cus) return 2;
    // Alone in its launch, the packed kernel halves the waves of a small long
    // list.  On databases of 100-6,000 subjects of 20-2,000 residues it took
    // 7-18% less time per search than the int32 long list, except at 8
    // columns per lane below about 1,500 pairs (up to 7% more).
    if (all_long && pairs > 0 && (ti != 8 || pairs >= 6LL * cus)) return 2;
    return 1;
}

// Whether an int32 long list runs inside the lane-per-subject kernel's own
// work queue (one subject per wave, long items first) instead of as a second
// kernel beside it.  A second kernel's waves each take a SIMD slot that a
// lane-per-subject wave needs (that kernel fills the register file at two
// waves per SIMD); how much that costs depended on where the dispatcher
// placed them, by up to 6% of a search from one process to the next.  Fused,
// the long list only costs its own arithmetic.  Only the fp16 plan at strip
// kFuseStrip has fused variants, and only where the wave-per-pair profile
// fits the lane-per-subject kernel's LDS.
bool fuse_ok(const sw_db *db, const Plan &plan, int ti);

// Kernels and grids of one pass.
struct Launch {
    Plan plan;
    int Ti = 16;
    int grid_inter = 0, grid_long = 0, grid_ovf = 0;
    bool packed_long = false;   // wave-per-pair items hold two subjects per wave
    bool fused_long = false;    // wave-per-pair items run in the lane-per-subject kernel
};

}  // namespace

// Host side of a database's device layout (pack_db).
struct Packed {
    int64_t n_seqs = 0, total_res = 0, max_len = 0;
    int32_t alphabet = 0;
    std::vector<int64_t> len;            // caller order
    std::vector<int32_t> long_ids;       // longest first
    int64_t long_res = 0, long_threshold = 0;
    bool fixed_cut = false;
    int32_t n_groups = 0, max_rows = 0;
    std::vector<int32_t> grp_rows;       // ascending
    int64_t inter_res = 0, inter_padded_rows = 0;
    std::vector<int32_t> grp_ids;        // n_groups x 128, -1 = empty slot
    std::vector<int64_t> grp_res_prefix; // n_groups + 1
    std::vector<int64_t> gbase;          // first code of each group
    std::vector<uint16_t> codes;         // pair codes
};

struct sw_db {
    int device = 0;
    std::string arch;
    hipStream_t stream = nullptr;
    // Second stream for the long list, forked from and joined to the search's
    // stream so the wave-per-pair kernel overlaps the lane-per-subject kernel.
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    int64_t n_seqs = 0;
    int alphabet = 0, R = 0;
    int64_t total_res = 0;
    int64_t max_len = 0;
    std::vector<int64_t> len;         // caller order
    // lane-per-subject groups
    int32_t n_groups = 0;
    int32_t max_rows = 0;
    std::vector<int32_t> grp_rows;    // host copy, ascending
    int64_t inter_res = 0;            // residues in groups
    int64_t inter_padded_rows = 0;    // sum of rows * 128
    std::vector<int32_t> grp_ids;     // host copy: caller ids of each group's 128 slots
    std::vector<int64_t> grp_res_prefix;  // residues in groups [0, g)
    // long list (caller ids), longest first: subjects too long for any group
    std::vector<int32_t> long_ids;
    int64_t long_res = 0;
    int64_t long_threshold = 0;
    bool fixed_cut = false;           // the caller fixed the split at open
    // device copies
    DevBuf d_res, d_off, d_codes, d_grp_base, d_grp_rows, d_grp_ids;
    DevBuf d_long_ids;                // long_ids on the device (sw_db_search_dev_noalloc)
    // per-call workspaces (plain and batched searches)
    DevBuf w_stage, w_scores, w_ovf, w_scr_inter, w_scr_intra, w_topk;
    // the pass counters (64 bytes), then the top-k indices and scores, so that
    // one copy brings all of them back into the pinned h_res
    DevBuf w_res;
    HostBuf h_stage, h_res;
    DevBuf w_al_meta, w_al_dir, w_al_ops, w_al_scr;   // sw_db_align workspaces
    HostBuf h_al;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    std::mutex mu;
    sw_search_opts opts{};
    sw_stats last{};
    std::map<int, Plan> tuned;        // autotuner: query-length bucket -> plan
    int cus = 256;
    std::string signature;
    // captured batch graph and the key of every argument it was captured with
    hipGraphExec_t graph = nullptr;
    std::string graph_key;
    bool server_attached = false;
};

namespace {

int validate_scoring(const sw_db *db, const sw_scoring *sc) {
    if (!sc) return fail(SW_EINVAL, "scoring is NULL");
    if (!sc->matrix) return fail(SW_EINVAL, "scoring matrix is NULL");
    if (sc->alphabet != db->alphabet)
        return fail(SW_EINVAL, "scoring alphabet %d differs from the database's %d", sc->alphabet,
                    db->alphabet);
    if (sc->alpha < 0) return fail(SW_EINVAL, "alpha < 0");
    if (sc->beta < sc->alpha) return fail(SW_EINVAL, "beta < alpha (beta = open + extension)");
    if (sc->beta > (1 << 30)) return fail(SW_EINVAL, "beta > 2^30");
    return SW_OK;
}

int validate_query(const sw_db *db, const uint8_t *q, int64_t qlen) {
    if (qlen < 1 || qlen > SW_MAX_LEN)
        return fail(SW_EINVAL, "query length %lld not in 1..2^24", (long long)qlen);
    if (!q) return fail(SW_EINVAL, "query is NULL");
    for (int64_t j = 0; j < qlen; ++j)
        if (q[j] >= db->alphabet)
            return fail(SW_EINVAL, "query code %d at %lld >= alphabet %d", q[j], (long long)j,
                        db->alphabet);
    return SW_OK;
}

// alpha: the gap extension of the search (0 when it varies per query).
// nq: queries in the launch; a launch of several takes the autotuner's batch
// entry when it has one.
Plan plan_for(const sw_db *db, int64_t max_qlen, int alpha, int32_t nq = 1) {
    Plan p;
    auto it = nq > 1 ? db->tuned.find(kBatchBucket) : db->tuned.end();
    if (it == db->tuned.end()) it = db->tuned.find(qlen_bucket(max_qlen));
    if (it != db->tuned.end()) p = it->second;
    // The fp16 tier's ceiling falls by 36 per unit of alpha (frame offsets);
    // past kFrameMaxAlpha the int16 tier flags far fewer lanes.
    if (p.tier == TIER_F16X2 && alpha > kFrameMaxAlpha) p.tier = TIER_I16X2;
    if (db->opts.tier) p.tier = db->opts.tier;
    if (db->opts.strip) p.strip = db->opts.strip;
    if (db->opts.waves) p.waves = db->opts.waves;
    if (p.strip == 64) p.waves = 4;
    if (p.waves == 6 && p.strip != 32) p.waves = 4;
    // The pair profile must fit in LDS.
    while (p.strip > 16 && inter_lds_bytes(db->R, p.strip) > 150 * 1024) p.strip /= 2;
    p.thr = p.tier == TIER_I16X2 ? kThrI16 : kThrF16;
    // the score-profile kernel exists for one plan only
    p.profile = db->opts.profile == SW_PROFILE_SCORE && p.tier == TIER_F16X2 && p.strip == 32 &&
                        p.waves == 4 && db->alphabet <= kSpMaxAlphabet
                    ? SW_PROFILE_SCORE
                    : SW_PROFILE_PAIR;
    if (db->opts.sat_threshold > 0 && db->opts.sat_threshold < p.thr) p.thr = db->opts.sat_threshold;
    return p;
}

// Query profile (section III.B.2): row r holds the scores of every query
// position against residue r; the pad row and the columns past the query are 0.
void write_profile(int8_t *dst, const uint8_t *q, int64_t qlen, int32_t mpad, const sw_scoring *sc,
                   int R) {
    const int A = sc->alphabet;
    for (int r = 0; r < R; ++r) {
        int8_t *row = dst + (int64_t)r * mpad;
        if (r < A)
            for (int64_t j = 0; j < qlen; ++j) row[j] = sc->matrix[q[j] * A + r];
        else
            std::memset(row, 0, (size_t)qlen);
        std::memset(row + qlen, 0, (size_t)(mpad - qlen));
    }
}

// Which groups a search runs lane-per-subject.  A wave works through one
// group per item, so the longest group must not hold its wave for longer than
// the average wave's share of the whole search, or it alone sets the
// makespan; longer groups go to the wave-per-pair kernel instead.  With many
// queries the share is large and every group stays lane-per-subject.
// Returns the number of leading groups (a multiple of the block size) to run
// lane-per-subject, and appends the routed subjects to `long_ids`.
// The cut alone (allocates nothing): the number of leading groups.
int64_t route_cut_groups(const sw_db *db, const Plan &plan, const int32_t *mpad, int64_t nq,
                         int resident_waves) {
    const int W = plan.waves;
    if (db->n_groups == 0) return 0;
    int64_t g_cut = db->n_groups;
    if (!db->fixed_cut) {
        double strips = 0, max_strips = 1;
        for (int64_t x = 0; x < nq; ++x) {
            const double ms = (mpad[x] + plan.strip - 1) / plan.strip;
            strips += ms;
            max_strips = std::max<double>(max_strips, ms);
        }
        const double rows = (double)db->inter_padded_rows / kGroup;
        const double share = strips * rows / std::max(resident_waves, 1) / max_strips;
        const int64_t rows_cut = std::max<int64_t>(1024, (int64_t)share);
        const int32_t cut32 = (int32_t)std::min<int64_t>(rows_cut, INT32_MAX);
        g_cut = std::upper_bound(db->grp_rows.begin(), db->grp_rows.end(), cut32) -
                db->grp_rows.begin();
        if (g_cut < db->n_groups) g_cut = g_cut / W * W;
    }
    return g_cut;
}

int64_t route_cut(const sw_db *db, const Plan &plan, const std::vector<int32_t> &mpad,
                  int resident_waves, std::vector<int32_t> &long_ids) {
    long_ids = db->long_ids;
    if (db->n_groups == 0) return 0;
    const int64_t g_cut =
        route_cut_groups(db, plan, mpad.data(), (int64_t)mpad.size(), resident_waves);
    std::vector<int32_t> routed;
    for (int64_t g = db->n_groups - 1; g >= g_cut; --g)
        for (int x = kGroup - 1; x >= 0; --x) {
            const int32_t id = db->grp_ids[(size_t)g * kGroup + x];
            if (id >= 0) routed.push_back(id);
        }
    // longest first: the fixed long list precedes every routed group
    std::stable_sort(routed.begin(), routed.end(),
                     [&](int32_t a, int32_t b) { return db->len[a] > db->len[b]; });
    long_ids.insert(long_ids.end(), routed.begin(), routed.end());
    return g_cut;
}

// Lane-per-subject items for `slots` against group blocks [b0, b1) and, if
// with_long, wave-per-pair items against `long_ids`; each list longest first
// (the GPU analogue of the guided schedule of section III.A).
// stride > 1 keeps every stride-th block only (autotuner sampling).
void build_items(const sw_db *db, const Plan &plan, const std::vector<int32_t> &slots,
                 const std::vector<int32_t> &mpad, const std::vector<int64_t> &qlen, int64_t b0,
                 int64_t b1, bool with_long, const std::vector<int32_t> &long_ids, int64_t stride,
                 bool fuse, Items &it) {
    const int W = plan.waves;
    std::vector<std::pair<int64_t, std::pair<int32_t, int32_t>>> v;
    v.reserve((size_t)slots.size() * (size_t)std::max<int64_t>(b1 - b0, 0));
    for (size_t x = 0; x < slots.size(); ++x) {
        const int32_t s = slots[x];
        const int64_t strips = (mpad[x] + plan.strip - 1) / plan.strip;
        for (int64_t bk = b0; bk < b1; ++bk) {
            if (stride > 1 && (bk % stride) != 0) continue;
            const int last = (int)std::min<int64_t>(db->n_groups, (bk + 1) * W) - 1;
            v.push_back({(int64_t)db->grp_rows[last] * strips, {s, (int32_t)(bk * W)}});
        }
    }
    std::stable_sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    it.inter_q.resize(v.size());
    it.inter_g.resize(v.size());
    for (size_t i = 0; i < v.size(); ++i) {
        it.inter_q[i] = v[i].second.first;
        it.inter_g[i] = v[i].second.second;
    }
    it.intra_q.clear();
    it.intra_ids.clear();
    it.fused = false;
    if (!with_long) return;
    const int64_t nlong = (int64_t)long_ids.size();
    const int64_t max_q = qlen.empty() ? 1 : *std::max_element(qlen.begin(), qlen.end());
    const int pw = intra_per_wave(plan, nlong * (int64_t)slots.size(), db->cus, v.empty(),
                                  intra_T_for(max_q));
    it.fused = fuse && pw == 1;
    const int per = it.fused ? W : kIntraWaves * pw;
    it.per_item = per;
    const int64_t nlblk = (nlong + per - 1) / per;
    std::vector<std::pair<int64_t, std::pair<int32_t, int64_t>>> u;
    for (size_t x = 0; x < slots.size(); ++x)
        for (int64_t bk = 0; bk < nlblk; ++bk) {
            if (stride > 1 && (bk % stride) != 0) continue;
            u.push_back({db->len[long_ids[bk * per]] * qlen[x], {slots[x], bk}});
        }
    std::stable_sort(u.begin(), u.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    it.intra_q.resize(u.size());
    it.intra_ids.resize(u.size() * per);
    for (size_t i = 0; i < u.size(); ++i) {
        it.intra_q[i] = u[i].second.first;
        for (int w = 0; w < per; ++w) {
            const int64_t x = u[i].second.second * per + w;
            it.intra_ids[i * per + w] = x < nlong ? long_ids[x] : -1;
        }
    }
}

// Work of one server pass: slot `slot` against lane-per-subject blocks
// [b0, b1), or against the whole long list.
struct PassWork {
    int32_t slot = 0;
    int32_t mpad = 0;
    int64_t qlen = 0;
    int64_t b0 = 0, b1 = 0;
    bool long_list = false;
};

// Items of a server pass: every (slot, block) of the work list and every
// (slot, long-list block), each list longest first as in build_items.
void build_work_items(const sw_db *db, const Plan &plan, const std::vector<PassWork> &work,
                      const std::vector<int32_t> &long_ids, bool fuse, Items &it) {
    const int W = plan.waves;
    std::vector<std::pair<int64_t, std::pair<int32_t, int32_t>>> v;
    int64_t n_long_slots = 0;
    for (const PassWork &w : work) {
        if (w.long_list) {
            ++n_long_slots;
            continue;
        }
        const int64_t strips = (w.mpad + plan.strip - 1) / plan.strip;
        for (int64_t bk = w.b0; bk < w.b1; ++bk) {
            const int last = (int)std::min<int64_t>(db->n_groups, (bk + 1) * W) - 1;
            v.push_back({(int64_t)db->grp_rows[last] * strips, {w.slot, (int32_t)(bk * W)}});
        }
    }
    std::stable_sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    it.inter_q.resize(v.size());
    it.inter_g.resize(v.size());
    for (size_t i = 0; i < v.size(); ++i) {
        it.inter_q[i] = v[i].second.first;
        it.inter_g[i] = v[i].second.second;
    }
    it.intra_q.clear();
    it.intra_ids.clear();
    const int64_t nlong = (int64_t)long_ids.size();
    const int pw = intra_per_wave(plan, nlong * n_long_slots, db->cus);
    it.fused = fuse && pw == 1 && n_long_slots > 0 && nlong > 0;
    const int per = it.fused ? W : kIntraWaves * pw;
    it.per_item = per;
    if (n_long_slots == 0 || nlong == 0) return;
    const int64_t nlblk = (nlong + per - 1) / per;
    std::vector<std::pair<int64_t, std::pair<int32_t, int64_t>>> u;
    for (const PassWork &w : work)
        if (w.long_list)
            for (int64_t bk = 0; bk < nlblk; ++bk)
                u.push_back({db->len[long_ids[bk * per]] * w.qlen, {w.slot, bk}});
    std::stable_sort(u.begin(), u.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    it.intra_q.resize(u.size());
    it.intra_ids.resize(u.size() * per);
    for (size_t i = 0; i < u.size(); ++i) {
        it.intra_q[i] = u[i].second.first;
        for (int x = 0; x < per; ++x) {
            const int64_t j = u[i].second.second * per + x;
            it.intra_ids[i * per + x] = j < nlong ? long_ids[j] : -1;
        }
    }
}

Launch launch_config(const sw_db *db, const Plan &plan, int64_t max_qlen, int64_t n_inter,
                     int64_t n_intra, bool fused = false) {
    Launch L;
    L.plan = plan;
    L.Ti = intra_T_for(max_qlen);
    L.fused_long = fused && n_intra > 0;
    L.grid_inter = (int)std::min<int64_t>(
        L.fused_long ? n_inter + n_intra : n_inter,
        plan.profile == SW_PROFILE_SCORE
            ? inter_sp_max_grid(db->R, plan.waves)
            : inter_max_grid(db->R, plan.tier, plan.strip, plan.waves, L.fused_long ? L.Ti : 0));
    // either wave-per-pair kernel (int32 or packed: the same profile and feed
    // rings per workgroup)
    const int per_cu =
        std::max(1, std::min(160 * 1024 / (wpp_lds_bytes(db->R, L.Ti, kIntraWaves) + 64), 8));
    L.grid_long = (int)std::min<int64_t>(n_intra, (int64_t)per_cu * db->cus);
    const int per_cu16 = std::max(1, std::min(160 * 1024 / (wpp_lds_bytes(db->R, 16, 1) + 64), 8));
    L.grid_ovf = std::min(per_cu16 * db->cus * kIntraWaves, 4096);
    return L;
}

bool fuse_ok(const sw_db *db, const Plan &plan, int ti) {
    return plan.profile == SW_PROFILE_PAIR && plan.tier == TIER_F16X2 && plan.strip == kFuseStrip &&
           (plan.waves == 4 || plan.waves == 6 || plan.waves == 8) &&
           wpp_lds_bytes(db->R, ti, plan.waves) <= inter_lds_bytes(db->R, plan.strip);
}

int64_t intra_scratch_rows(const sw_db *db) {
    return round_up(std::max<int64_t>(db->max_len, 1), 64) + 128;
}

// Device buffers a pass reads and writes.
struct PassBufs {
    QuerySet qs{};
    const int32_t *it_q = nullptr, *it_g = nullptr, *il_q = nullptr, *il_ids = nullptr;
    int64_t n_inter = 0, n_intra = 0;
    int32_t *scores = nullptr;
    int32_t *ovf_q = nullptr, *ovf_id = nullptr;
    int64_t ovf_cap = 0;
    int32_t *counters = nullptr;   // inter head, overflow count, long head, recompute head
    uint32_t *scr_inter = nullptr;
    int32_t scr_rows = 0;          // rows per wave slot of scr_inter
    int32_t *scr_intra = nullptr;
};

// Enqueue one pass: counter reset (a fill kernel, safe under graph capture),
// lane-per-subject kernel, wave-per-pair kernel on the long list, exact
// recompute of flagged lanes.  Optional events bracket the first kernel;
// ev_r (optional) is recorded just before the recompute.
// The long list's makespan is its longest pair, so it should start at once
// and share the GPU with the lane-per-subject work:
//  * L.fused_long: its items run first in the lane-per-subject kernel's own
//    work queue (one launch; see fuse_ok);
//  * otherwise, with `overlap`, it runs on the database's second stream,
//    launched before the lane-per-subject kernel (the other order measured
//    slower and erratic), and joins before the recompute.
int enqueue_pass(const sw_db *db, const Launch &L, const PassBufs &b, hipStream_t st,
                 hipEvent_t ev_a = nullptr, hipEvent_t ev_b = nullptr, bool overlap = false,
                 hipEvent_t ev_r = nullptr) {
    HIPX(launch_fill_i32(b.counters, 0, 4, st));
    const bool fused = L.fused_long && b.n_intra > 0;
    const bool fork = overlap && !fused && b.n_inter > 0 && b.n_intra > 0;
    if (fork) {
        HIPX(hipEventRecord(db->fork, st));
        HIPX(hipStreamWaitEvent(db->aux, db->fork, 0));
    }
    IntraArgs ia{};
    ia.res = db->d_res.as<uint8_t>();
    ia.off = db->d_off.as<int64_t>();
    ia.qs = b.qs;
    ia.R = db->R;
    ia.pass_scratch = b.scr_intra;
    ia.max_len_pad = intra_scratch_rows(db);
    ia.scores = b.scores;
    ia.n_seqs = db->n_seqs;
    ia.thr = L.plan.thr;
    ia.ovf_q = b.ovf_q;
    ia.ovf_id = b.ovf_id;
    ia.ovf_count = b.counters + 1;
    ia.ovf_cap = b.ovf_cap;
    auto launch_long_aux = [&]() -> int {
        IntraArgs la = ia;
        la.item_q = b.il_q;
        la.item_ids = b.il_ids;
        la.n_items = (int32_t)b.n_intra;
        la.counter = b.counters + 2;
        if (L.packed_long) HIPX(launch_intra2(la, L.Ti, kIntraWaves, L.grid_long, db->aux));
        else HIPX(launch_intra(la, L.Ti, kIntraWaves, L.grid_long, db->aux));
        HIPX(hipEventRecord(db->join, db->aux));
        return SW_OK;
    };
    if (fork) TRY(launch_long_aux());
    if (ev_a) HIPX(hipEventRecord(ev_a, st));
    if (b.n_inter > 0 || fused) {
        InterArgs a{};
        a.codes = db->d_codes.as<uint16_t>();
        a.grp_base = db->d_grp_base.as<int64_t>();
        a.grp_rows = db->d_grp_rows.as<int32_t>();
        a.grp_ids = db->d_grp_ids.as<int32_t>();
        a.n_groups = db->n_groups;
        a.item_q = b.it_q;
        a.item_g = b.it_g;
        a.n_items = (int32_t)b.n_inter;
        a.counter = b.counters + 0;
        a.qs = b.qs;
        a.R = db->R;
        a.thr = L.plan.thr;
        a.scratch = b.scr_inter;
        a.max_rows = b.scr_rows;
        a.scores = b.scores;
        a.n_seqs = db->n_seqs;
        a.ovf_q = b.ovf_q;
        a.ovf_id = b.ovf_id;
        a.ovf_count = b.counters + 1;
        a.ovf_cap = b.ovf_cap;
        IntraArgs fl = ia;
        fl.item_q = b.il_q;
        fl.item_ids = b.il_ids;
        fl.n_items = (int32_t)b.n_intra;
        if (L.plan.profile == SW_PROFILE_SCORE) {
            if (!b.qs.qc) return fail(SW_EINVAL, "internal: score profile without query codes");
            HIPX(launch_inter_sp(a, L.plan.strip, L.plan.waves, L.grid_inter, st));
        } else {
            HIPX(launch_inter(a, fused ? &fl : nullptr, L.Ti, L.plan.tier, L.plan.strip, L.plan.waves,
                              L.grid_inter, st));
        }
    }
    if (ev_b) HIPX(hipEventRecord(ev_b, st));
    const bool packed_long = L.packed_long;
    if (b.n_intra > 0 && !fork && !fused) {
        IntraArgs la = ia;
        la.item_q = b.il_q;
        la.item_ids = b.il_ids;
        la.n_items = (int32_t)b.n_intra;
        la.counter = b.counters + 2;
        if (packed_long) HIPX(launch_intra2(la, L.Ti, kIntraWaves, L.grid_long, st));
        else HIPX(launch_intra(la, L.Ti, kIntraWaves, L.grid_long, st));
    }
    if (fork) HIPX(hipStreamWaitEvent(st, db->join, 0));
    if (ev_r) HIPX(hipEventRecord(ev_r, st));
    // Only the lane-per-subject kernel leaves flagged pairs for this launch:
    // the packed wave-per-pair kernel recomputes its own, and the int32 one
    // flags nothing.
    if (b.n_inter > 0) {
        IntraArgs oa = ia;
        oa.item_q = b.ovf_q;
        oa.item_ids = b.ovf_id;
        oa.n_items_dev = b.counters + 1;
        oa.counter = b.counters + 3;
        // the launch's own columns per lane: a short query's pass is narrower
        HIPX(launch_intra(oa, L.Ti, 1, L.grid_ovf, st));
    }
    return SW_OK;
}

size_t topk_work_bytes(int32_t nq, int32_t k) {
    return (size_t)nq * (256 * 4 + 4 * 4 + kTopkBlocks * 4 + (size_t)k * 8);
}

TopkWork topk_work(void *base, int32_t nq, int32_t k) {
    TopkWork tw;
    tw.hist = (uint32_t *)base;
    tw.state = (int32_t *)(tw.hist + (size_t)nq * 256);
    tw.eqcnt = tw.state + (size_t)nq * 4;
    tw.cand_s = tw.eqcnt + (size_t)nq * kTopkBlocks;
    tw.cand_i = tw.cand_s + (size_t)nq * k;
    return tw;
}

// Layout of the per-call staging area (host pinned -> device, one copy).
struct StageLayout {
    size_t prof = 0, ptrs = 0, mpad = 0, qlen = 0, gap = 0, items = 0, total = 0;
    size_t qc = 0, qcd = 0;   // score profile: pointer per query, then matrix + codes blocks
};

// code_bytes > 0: the score-profile kernel's per-query blocks (after the profiles).
StageLayout stage_layout(int32_t nq, int64_t prof_bytes, const Items &it, int64_t code_bytes = 0) {
    // Fixed-size parts first: their offsets depend only on nq and the item
    // counts, which a captured graph's key pins; the profiles go last.
    StageLayout s;
    size_t o = 0;
    s.ptrs = o;
    o += (size_t)round_up((int64_t)nq * 8, 256);
    s.mpad = o;
    o += (size_t)round_up((int64_t)nq * 4, 256);
    s.qlen = o;
    o += (size_t)round_up((int64_t)nq * 4, 256);
    s.gap = o;
    o += (size_t)round_up((int64_t)nq * 8, 256);
    s.items = o;
    o += (size_t)round_up((int64_t)(it.inter_q.size() * 2 + it.intra_q.size() * (1 + it.per_item)) * 4, 256);
    s.qc = o;
    if (code_bytes > 0) o += (size_t)round_up((int64_t)nq * 8, 256);
    s.prof = o;
    o += (size_t)round_up(prof_bytes, 256);
    s.qcd = o;
    o += (size_t)round_up(code_bytes, 256);
    s.total = o;
    return s;
}

// The search path for nq queries in one fused pass.  Outputs (any may be null):
//   scores_host: nq * n_seqs; scores_dev: device pointer (nq * n_seqs);
//   top_s/top_i: nq * k when k > 0.
//   item_stride > 1 evaluates only every stride-th block (autotuner timing).
//   use_graph: capture the device work in a HIP graph and replay it on later
//   calls of the same shape.
int run_search(sw_db *db, int32_t nq, const uint8_t *q_res, const int64_t *q_off,
               const sw_scoring *sc, int32_t k, int32_t *top_s, int64_t *top_i,
               int32_t *scores_host, int32_t *scores_dev, hipStream_t user_stream,
               int64_t item_stride = 1, bool use_graph = false) {
    const double t_start = now_ms();
    TRY(validate_scoring(db, sc));
    if (nq < 1) return fail(SW_EINVAL, "nq < 1");
    if (!q_res || !q_off) return fail(SW_EINVAL, "queries are NULL");
    if (k < 0 || k > SW_MAX_K) return fail(SW_EINVAL, "k not in 1..%d", SW_MAX_K);
    std::vector<int64_t> qlen(nq);
    std::vector<int32_t> mpad(nq);
    std::vector<int64_t> poff(nq);
    int64_t prof_bytes = 0, sum_qlen = 0, max_qlen = 0;
    for (int32_t q = 0; q < nq; ++q) {
        qlen[q] = q_off[q + 1] - q_off[q];
        TRY(validate_query(db, q_res + q_off[q], qlen[q]));
        mpad[q] = (int32_t)round_up(qlen[q], kQPad);
        poff[q] = prof_bytes;
        prof_bytes += (int64_t)db->R * mpad[q];
        sum_qlen += qlen[q];
        max_qlen = std::max(max_qlen, qlen[q]);
    }
    if ((int64_t)nq * db->n_seqs > ((int64_t)1 << 40)) return fail(SW_EINVAL, "batch too large");
    HIPX(hipSetDevice(db->device));
    hipStream_t st = user_stream ? user_stream : db->stream;
    const Plan plan = plan_for(db, max_qlen, sc->alpha, nq);
    const int64_t n = db->n_seqs;

    std::vector<int32_t> slots(nq);
    std::iota(slots.begin(), slots.end(), 0);
    std::vector<int32_t> long_ids;
    const int resident = (plan.profile == SW_PROFILE_SCORE
                              ? inter_sp_max_grid(db->R, plan.waves)
                              : inter_max_grid(db->R, plan.tier, plan.strip, plan.waves)) * plan.waves;
    const int64_t g_cut = route_cut(db, plan, mpad, resident, long_ids);
    Items it;
    const int64_t nblk = (g_cut + plan.waves - 1) / plan.waves;
    build_items(db, plan, slots, mpad, qlen, 0, nblk, true, long_ids, item_stride,
                fuse_ok(db, plan, intra_T_for(max_qlen)), it);
    const int64_t n_inter = (int64_t)it.inter_q.size(), n_intra = (int64_t)it.intra_q.size();
    if (n_inter > INT32_MAX || n_intra > INT32_MAX) return fail(SW_EINVAL, "batch too large");
    Launch L = launch_config(db, plan, max_qlen, n_inter, n_intra, it.fused);
    L.packed_long = !it.fused && it.per_item == 2 * kIntraWaves;
    const int32_t rows_alloc = g_cut > 0 ? db->grp_rows[g_cut - 1] : 0;
    int64_t long_res = 0;
    for (int32_t id : long_ids) long_res += db->len[id];

    // ---- device workspaces ----
    // score profile: per query the A x A matrix, then its codes padded to mpad with the pad letter
    const int64_t A = db->alphabet;
    std::vector<int64_t> qcoff(nq, 0);
    int64_t code_bytes = 0;
    if (plan.profile == SW_PROFILE_SCORE)
        for (int32_t q = 0; q < nq; ++q) {
            qcoff[q] = code_bytes;
            code_bytes += round_up(A * A + mpad[q], 16);
        }
    const StageLayout sl = stage_layout(nq, prof_bytes, it, code_bytes);
    TRY(db->w_stage.reserve(sl.total));
    TRY(db->w_scores.reserve((size_t)nq * n * 4 + 4));
    TRY(db->w_ovf.reserve((size_t)nq * n * 8 + 8));
    if (n_inter > 0)
        TRY(db->w_scr_inter.reserve((size_t)L.grid_inter * plan.waves * rows_alloc * 512));
    // wave-per-pair scratch: one slot per wave of whichever kernel runs the long list
    const int64_t long_slots = L.fused_long ? (int64_t)L.grid_inter * plan.waves
                                            : (int64_t)L.grid_long * kIntraWaves;
    const int64_t intra_slots = std::max<int64_t>(long_slots, L.grid_ovf);
    TRY(db->w_scr_intra.reserve((size_t)intra_slots * intra_scratch_rows(db) * 8));
    if (k > 0) TRY(db->w_topk.reserve(topk_work_bytes(nq, k)));
    const size_t res_bytes = kResHead + (size_t)nq * k * 12;
    TRY(db->w_res.reserve(res_bytes));
    TRY(db->h_res.reserve(res_bytes));

    // ---- host staging (the previous call may still be reading it) ----
    TRY(db->h_stage.reserve(sl.total));
    HIPX(hipStreamSynchronize(st));
    uint8_t *hs = db->h_stage.as<uint8_t>();
    uint8_t *ds = db->w_stage.as<uint8_t>();
    for (int32_t q = 0; q < nq; ++q)
        write_profile((int8_t *)(hs + sl.prof + poff[q]), q_res + q_off[q], qlen[q], mpad[q], sc,
                      db->R);
    {
        const int8_t **ptrs = (const int8_t **)(hs + sl.ptrs);
        int32_t *mp = (int32_t *)(hs + sl.mpad), *ql = (int32_t *)(hs + sl.qlen);
        int32_t *gp = (int32_t *)(hs + sl.gap);
        for (int32_t q = 0; q < nq; ++q) {
            ptrs[q] = (const int8_t *)(ds + sl.prof + poff[q]);
            mp[q] = mpad[q];
            ql[q] = (int32_t)qlen[q];
            gp[2 * q] = sc->alpha;
            gp[2 * q + 1] = sc->beta;
        }
        if (code_bytes > 0) {
            const uint8_t **qc = (const uint8_t **)(hs + sl.qc);
            for (int32_t q = 0; q < nq; ++q) {
                uint8_t *blk = hs + sl.qcd + qcoff[q];
                qc[q] = ds + sl.qcd + qcoff[q];
                std::memcpy(blk, sc->matrix, (size_t)(A * A));
                std::memcpy(blk + A * A, q_res + q_off[q], (size_t)qlen[q]);
                std::memset(blk + A * A + qlen[q], (int)A, (size_t)(mpad[q] - qlen[q]));
            }
        }
        int32_t *p = (int32_t *)(hs + sl.items);
        std::memcpy(p, it.inter_q.data(), n_inter * 4);
        std::memcpy(p + n_inter, it.inter_g.data(), n_inter * 4);
        std::memcpy(p + 2 * n_inter, it.intra_q.data(), n_intra * 4);
        std::memcpy(p + 2 * n_inter + n_intra, it.intra_ids.data(), n_intra * it.per_item * 4);
    }
    HIPX(hipMemcpyAsync(ds, hs, sl.total, hipMemcpyHostToDevice, st));

    PassBufs pb;
    pb.qs.qp = (const int8_t *const *)(ds + sl.ptrs);
    pb.qs.mpad = (const int32_t *)(ds + sl.mpad);
    pb.qs.qlen = (const int32_t *)(ds + sl.qlen);
    pb.qs.gap = (const int32_t *)(ds + sl.gap);
    pb.qs.qc = code_bytes > 0 ? (const uint8_t *const *)(ds + sl.qc) : nullptr;
    pb.it_q = (const int32_t *)(ds + sl.items);
    pb.it_g = pb.it_q + n_inter;
    pb.il_q = pb.it_g + n_inter;
    pb.il_ids = pb.il_q + n_intra;
    pb.n_inter = n_inter;
    pb.n_intra = n_intra;
    pb.scores = scores_dev ? scores_dev : db->w_scores.as<int32_t>();
    pb.ovf_q = db->w_ovf.as<int32_t>();
    pb.ovf_id = pb.ovf_q + (size_t)nq * n;
    pb.ovf_cap = (int64_t)nq * n;
    pb.counters = db->w_res.as<int32_t>();
    pb.scr_inter = db->w_scr_inter.as<uint32_t>();
    pb.scr_rows = rows_alloc;
    pb.scr_intra = db->w_scr_intra.as<int32_t>();
    int64_t *d_ti = k > 0 ? (int64_t *)(db->w_res.as<uint8_t>() + kResHead) : nullptr;
    int32_t *d_ts = d_ti ? (int32_t *)(d_ti + (size_t)nq * k) : nullptr;

    auto enqueue_all = [&](hipStream_t s, bool events) -> int {
        TRY(enqueue_pass(db, L, pb, s, events ? db->ev[0] : nullptr, events ? db->ev[1] : nullptr,
                         true, events ? db->ev[4] : nullptr));
        if (events) HIPX(hipEventRecord(db->ev[2], s));
        if (k > 0)
            HIPX(launch_topk(pb.scores, n, nq, nullptr, k, topk_work(db->w_topk.p, nq, k), d_ts,
                             d_ti, s));
        return SW_OK;
    };

    bool graphed = false;
    if (use_graph && db->opts.graph >= 0) {
        // Every kernel argument of the pass is fixed by this key; what changes
        // between calls of one shape (profiles, items) arrives by the staging copy.
        char key[512];
        snprintf(key, sizeof key, "%d|%d|%d|%d|%d|%d|%d|%d|%lld|%lld|%d|%d|%d|%d|%p|%p|%p|%p|%p|%p|%p|%p",
                 rows_alloc, nq, k, plan.tier, plan.strip, plan.waves, plan.thr, plan.profile, (long long)n_inter,
                 (long long)n_intra, L.Ti, L.grid_inter, L.grid_long, L.grid_ovf, (void *)ds,
                 (void *)pb.scores, (void *)pb.ovf_q, (void *)pb.counters, (void *)pb.scr_inter,
                 (void *)pb.scr_intra, db->w_topk.p, (void *)d_ti);
        if (!db->graph || db->graph_key != key) {
            if (db->graph) {
                (void)hipGraphExecDestroy(db->graph);
                db->graph = nullptr;
            }
            // Capture on the library's own stream, ordered after the staging copy.
            hipStream_t cs = db->stream;
            if (st != cs) {
                HIPX(hipEventRecord(db->ev[3], st));
                HIPX(hipStreamWaitEvent(cs, db->ev[3], 0));
            }
            HIPX(hipStreamSynchronize(cs));
            hipGraph_t g = nullptr;
            HIPX(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_all(cs, false);
            hipError_t e = hipStreamEndCapture(cs, &g);
            if (rc != SW_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return fail(SW_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&db->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                db->graph = nullptr;
                return fail(SW_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(e));
            }
            db->graph_key = key;
        }
        HIPX(hipEventRecord(db->ev[0], st));
        HIPX(hipGraphLaunch(db->graph, st));
        HIPX(hipEventRecord(db->ev[2], st));
        graphed = true;
    } else {
        TRY(enqueue_all(st, true));
    }
    if (scores_host && n > 0)
        HIPX(hipMemcpyAsync(scores_host, pb.scores, (size_t)nq * n * 4, hipMemcpyDeviceToHost, st));
    // counters and top-k in one copy to pinned memory
    HIPX(hipMemcpyAsync(db->h_res.p, db->w_res.p, res_bytes, hipMemcpyDeviceToHost, st));
    HIPX(hipStreamSynchronize(st));
    int32_t ctr_h[4];
    std::memcpy(ctr_h, db->h_res.p, sizeof ctr_h);
    if (k > 0) {
        const uint8_t *hr = db->h_res.as<uint8_t>() + kResHead;
        std::memcpy(top_i, hr, (size_t)nq * k * 8);
        std::memcpy(top_s, hr + (size_t)nq * k * 8, (size_t)nq * k * 4);
    }

    float ms_k = 0, ms_i = -1, ms_r = -1, ms_l = -1;
    HIPX(hipEventElapsedTime(&ms_k, db->ev[0], db->ev[2]));
    if (!graphed) {
        HIPX(hipEventElapsedTime(&ms_i, db->ev[0], db->ev[1]));
        HIPX(hipEventElapsedTime(&ms_r, db->ev[4], db->ev[2]));
        // the wave-per-pair kernel alone on the stream, between the two (a
        // long list fused into the lane-per-subject launch is timed in ms_i)
        if (n_inter == 0 && n_intra > 0 && !L.fused_long)
            HIPX(hipEventElapsedTime(&ms_l, db->ev[1], db->ev[4]));
    }
    sw_stats &s = db->last;
    s = sw_stats{};
    s.cells = sum_qlen * db->total_res;
    int64_t padded = 0;
    int64_t inter_rows = 0;
    for (int64_t g = 0; g < g_cut; ++g) inter_rows += (int64_t)db->grp_rows[g] * kGroup;
    for (int32_t q = 0; q < nq; ++q)
        padded += round_up((int64_t)mpad[q], (int64_t)plan.strip) * inter_rows +
                  long_columns(qlen[q], L.Ti, L.packed_long) * long_res;
    s.padded_cells = padded;
    s.inter_cells = sum_qlen * db->grp_res_prefix[g_cut];
    s.recomputed_pairs = ctr_h[1];
    s.intra_pairs = (int64_t)long_ids.size() * nq;
    s.kernel_ms = ms_k;
    s.inter_ms = ms_i;
    s.recompute_ms = ms_r;
    s.long_ms = ms_l;
    s.total_ms = now_ms() - t_start;
    s.tier = plan.tier;
    s.strip = plan.strip;
    s.waves = plan.waves;
    s.graphed = graphed ? 1 : 0;
    s.fused_long = L.fused_long ? 1 : 0;
    s.profile = plan.profile;
    return SW_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: time candidate plans on a strided sample of the work, per
// query-length bucket, and keep the fastest.
// ---------------------------------------------------------------------------
const Plan kCandidates[] = {
    {TIER_F16X2, 32, 4, 0}, {TIER_F16X2, 64, 4, 0}, {TIER_F16X2, 32, 8, 0},
    {TIER_I16X2, 32, 4, 0}, {TIER_I16X2, 64, 4, 0}, {TIER_F16X2, 16, 8, 0},
};

bool read_cache(sw_db *db, const char *path) {
    FILE *f = fopen(path, "r");
    if (!f) return false;
    std::string text;
    char buf[4096];
    size_t r;
    while ((r = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, r);
    fclose(f);
    const std::string sig = "\"signature\": \"" + db->signature + "\"";
    if (text.find(sig) == std::string::npos) return false;
    std::map<int, Plan> t;
    size_t pos = 0;
    while ((pos = text.find("{\"bucket\":", pos)) != std::string::npos) {
        int b, tier, strip, waves;
        if (sscanf(text.c_str() + pos, "{\"bucket\": %d, \"tier\": %d, \"strip\": %d, \"waves\": %d",
                   &b, &tier, &strip, &waves) == 4 &&
            (tier == TIER_F16X2 || tier == TIER_I16X2) && (strip == 16 || strip == 32 || strip == 64) &&
            (waves == 4 || waves == 6 || waves == 8)) {
            Plan p;
            p.tier = tier;
            p.strip = strip;
            p.waves = waves;
            t[b] = p;
        }
        ++pos;
    }
    if (t.empty()) return false;
    db->tuned = t;
    return true;
}

int write_cache(const sw_db *db, const char *path, const std::map<int, double> &gcups) {
    FILE *f = fopen(path, "w");
    if (!f) return fail(SW_EINVAL, "cannot write autotune cache %s", path);
    fprintf(f, "{\"signature\": \"%s\", \"entries\": [\n", db->signature.c_str());
    size_t i = 0;
    for (const auto &kv : db->tuned) {
        auto g = gcups.find(kv.first);
        fprintf(f, "  {\"bucket\": %d, \"tier\": %d, \"strip\": %d, \"waves\": %d, \"gcups\": %.1f}%s\n",
                kv.first, kv.second.tier, kv.second.strip, kv.second.waves,
                g == gcups.end() ? 0.0 : g->second, ++i < db->tuned.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    fclose(f);
    return SW_OK;
}

int autotune(sw_db *db, const sw_scoring *sc, const int32_t *qlens, int32_t n_qlens,
             const char *cache_path) {
    TRY(validate_scoring(db, sc));
    if (n_qlens < 0 || (n_qlens > 0 && !qlens)) return fail(SW_EINVAL, "bad query-length list");
    if (cache_path && read_cache(db, cache_path)) return SW_OK;
    if (db->n_groups == 0) return SW_OK;   // nothing runs lane-per-subject
    const sw_search_opts saved = db->opts;
    std::map<int, double> best_gcups;
    // Time every stride-th block only, but keep at least 16 items per resident
    // workgroup: with fewer, the tail of the work queue, not the plan, decides.
    const int64_t resident = inter_max_grid(db->R, TIER_F16X2, 32, 4);
    const int64_t stride =
        std::max<int64_t>(1, std::min<int64_t>(8, (db->n_groups / 4) / (16 * resident)));
    uint32_t lcg = 12345u;
    // GCUPS of one plan: best of `reps` timed runs after one warm-up run (the
    // first run warms caches and buffers; single runs of one plan vary by
    // 10-20% with how the long list's kernel shares the chip).
    auto time_plan = [&](const Plan &cand, const std::vector<uint8_t> &q, int64_t str,
                         int reps, double *gcups) -> int {
        sw_search_opts o{};
        o.tier = cand.tier;
        o.strip = cand.strip;
        o.waves = cand.waves;
        db->opts = o;
        const int64_t off[2] = {0, (int64_t)q.size()};
        double ms = 1e30;
        for (int rep = 0; rep <= reps; ++rep) {
            const int rc = run_search(db, 1, q.data(), off, sc, 0, nullptr, nullptr, nullptr,
                                      nullptr, nullptr, str);
            if (rc != SW_OK) return rc;
            if (rep > 0) ms = std::min(ms, (double)db->last.inter_ms);
        }
        *gcups = (double)db->last.inter_cells / str / (ms * 1e6);
        return SW_OK;
    };
    for (int32_t x = 0; x < n_qlens; ++x) {
        const int64_t L = std::max(1, std::min(qlens[x], SW_MAX_LEN));
        const int b = qlen_bucket(L);
        if (best_gcups.count(b)) continue;
        std::vector<uint8_t> q((size_t)L);
        for (auto &c : q) {
            lcg = lcg * 1664525u + 1013904223u;
            c = (uint8_t)((lcg >> 16) % (uint32_t)db->alphabet);
        }
        // Screen every candidate on the sampled blocks, then time the two best
        // on the whole database and keep the faster.
        std::vector<std::pair<double, Plan>> screened;
        for (const Plan &cand : kCandidates) {
            if (inter_lds_bytes(db->R, cand.strip) > 150 * 1024) continue;
            double gc = 0;
            const int rc = time_plan(cand, q, stride, 1, &gc);
            if (rc != SW_OK) {
                db->opts = saved;
                return rc;
            }
            screened.push_back({gc, cand});
        }
        std::stable_sort(screened.begin(), screened.end(),
                         [](const auto &x, const auto &y) { return x.first > y.first; });
        double best = -1;
        Plan best_plan = screened.empty() ? Plan{} : screened[0].second;
        for (size_t i = 0; i < screened.size() && i < 2; ++i) {
            double gc = screened[i].first;
            if (stride > 1) {
                const int rc = time_plan(screened[i].second, q, 1, 2, &gc);
                if (rc != SW_OK) {
                    db->opts = saved;
                    return rc;
                }
            }
            if (gc > best) {
                best = gc;
                best_plan = screened[i].second;
            }
        }
        db->tuned[b] = best_plan;
        best_gcups[b] = best;
    }
    // A launch of several queries runs one plan for all of them, and the
    // winner for its longest query's bucket can be a poor choice for the mix.
    // Time the distinct bucket winners and the default plan on a batch of up
    // to 32 of the given lengths (every stride-th block, at most about 4e12
    // cells a run) and keep the fastest as the batch entry; with a single
    // candidate, nothing is timed.
    if (n_qlens > 1 && !best_gcups.empty()) {
        std::vector<Plan> cands{Plan{}};
        for (const auto &kv : db->tuned) {
            if (kv.first == kBatchBucket) continue;
            bool seen = false;
            for (const Plan &c : cands)
                seen = seen || (c.tier == kv.second.tier && c.strip == kv.second.strip &&
                                c.waves == kv.second.waves);
            if (!seen && inter_lds_bytes(db->R, kv.second.strip) <= 150 * 1024)
                cands.push_back(kv.second);
        }
        const int32_t m_max = std::min<int32_t>(n_qlens, 32);
        const double cell_cap = 4e12 * (double)stride / (double)std::max<int64_t>(1, db->total_res);
        int32_t m = 0;
        std::vector<int64_t> off(1, 0);
        std::vector<uint8_t> qs;
        for (int32_t x = 0; x < m_max && (m < 2 || (double)qs.size() < cell_cap); ++x, ++m) {
            const int64_t L = std::max(1, std::min(qlens[(int64_t)x * n_qlens / m_max], SW_MAX_LEN));
            for (int64_t j = 0; j < L; ++j) {
                lcg = lcg * 1664525u + 1013904223u;
                qs.push_back((uint8_t)((lcg >> 16) % (uint32_t)db->alphabet));
            }
            off.push_back((int64_t)qs.size());
        }
        const int32_t longest = *std::max_element(qlens, qlens + n_qlens);
        const int lb = qlen_bucket(std::max(1, std::min(longest, SW_MAX_LEN)));
        double best = best_gcups.count(lb) ? best_gcups[lb] : 0.0;
        Plan best_plan = cands.size() == 1 ? cands[0] : db->tuned.at(lb);
        if (cands.size() > 1) best = -1;
        for (size_t ci = 0; cands.size() > 1 && ci < cands.size(); ++ci) {
            const Plan &cand = cands[ci];
            sw_search_opts o{};
            o.tier = cand.tier;
            o.strip = cand.strip;
            o.waves = cand.waves;
            db->opts = o;
            double ms = 1e30;
            for (int rep = 0; rep <= 2; ++rep) {
                const int rc = run_search(db, m, qs.data(), off.data(), sc, 0, nullptr, nullptr,
                                          nullptr, nullptr, nullptr, stride);
                if (rc != SW_OK) {
                    db->opts = saved;
                    return rc;
                }
                if (rep > 0) ms = std::min(ms, (double)db->last.inter_ms);
            }
            const double gc = (double)db->last.inter_cells / stride / (ms * 1e6);
            if (gc > best) {
                best = gc;
                best_plan = cand;
            }
        }
        db->tuned[kBatchBucket] = best_plan;
        best_gcups[kBatchBucket] = best;
    }
    db->opts = saved;
    if (cache_path) TRY(write_cache(db, cache_path, best_gcups));
    return SW_OK;
}

}  // namespace

// ===========================================================================
// Serving: continuous batching over database chunks.
//
// The database stays resident.  Its lane-per-subject blocks are cut into
// chunks; the long list is one more position of a circular scan.  Each pass
// runs every admitted request against the scan's current position in one
// launch; a request admitted between passes starts at the next position and
// completes once it has visited every position.  A request's scores do not
// depend on which others share its passes, so results are the same alone and
// in the mix.
// ===========================================================================
namespace {

struct Request {
    uint64_t ticket = 0;
    std::vector<uint8_t> query;
    std::vector<int8_t> matrix;
    int32_t alpha = 0, beta = 0, k = 0;
    int64_t bytes = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int32_t slot = -1;
    int32_t next = 0;        // next database position to visit
    int32_t remaining = 0;   // database positions still to visit
    int32_t passes = 0;      // passes (launches) this request took part in
    int32_t shared = 0;      // of those, passes that also served another request
    int rc = SW_OK;
    bool done = false;
    std::vector<int32_t> top_s;
    std::vector<int64_t> top_i;
};

}  // namespace

struct sw_server {
    sw_db *db = nullptr;
    sw_server_opts opts{};
    Plan plan;                   // requests with alpha <= kFrameMaxAlpha (fp16 unless overridden)
    Plan plan16;                 // requests with larger alpha: the int16 tier, same waves
    bool split_tiers = false;    // high-alpha requests run in their own int16 sub-pass
    int64_t blocks = 0, chunk_blocks = 0, n_chunks = 0, n_pos = 0;
    std::vector<SchedPos> pos;   // per database position: residues, items, subjects
    int64_t pass_cells = 0;      // work a pass aims for (cells)
    int64_t pass_items = 0;      // lane-per-subject items a pass aims for (load balance)
    int64_t g_cut = 0;
    int64_t ovf_cap = 0;
    int32_t scr_rows = 0;
    std::vector<int32_t> long_ids;   // wave-per-pair subjects, longest first
    bool has_long = false;
    int32_t slots = 0;
    // device state
    std::vector<std::unique_ptr<DevBuf>> prof;   // query profile per slot
    DevBuf d_meta, d_scores, d_ovf, d_counters, d_scr_inter, d_scr_intra, d_items, d_topk, d_top,
        d_rows;
    HostBuf h_items, h_meta, h_top, h_rows;
    Launch L, L16;
    size_t items_half = 0;       // bytes of item staging per sub-pass (h_items holds two)
    bool fuse = false;           // int32 long-list items may run in the lane-per-subject kernel
    int grid_fused = 0;          // resident workgroups of that fused kernel
    // host state
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> waiting;
    std::vector<std::shared_ptr<Request>> active;   // by slot (nullptr = free)
    std::unordered_map<uint64_t, std::shared_ptr<Request>> table;
    uint64_t next_ticket = 1;
    int64_t used_bytes = 0;
    int32_t waiters = 0;     // threads inside sw_server_wait
    bool stop = false;
    std::thread worker;
    std::string fatal;
};

namespace {

int server_setup(sw_server *s) {
    sw_db *db = s->db;
    HIPX(hipSetDevice(db->device));
    s->plan = plan_for(db, 512, 0);
    s->plan.profile = SW_PROFILE_PAIR;   // passes carry no query codes
    const int W = s->plan.waves;
    // A request whose alpha would lower the fp16 ceiling past kFrameMaxAlpha
    // runs in an int16 sub-pass of its own (the planner's choice for a plain
    // search), over the same positions: the same waves per workgroup, so the
    // same blocks.
    s->plan16 = s->plan;
    s->split_tiers = db->opts.tier == 0 && s->plan.tier == TIER_F16X2;
    if (s->split_tiers) {
        s->plan16.tier = TIER_I16X2;
        s->plan16.strip = 32;
        s->plan16.thr = kThrI16;
        if (db->opts.sat_threshold > 0 && db->opts.sat_threshold < s->plan16.thr)
            s->plan16.thr = db->opts.sat_threshold;
    }
    {
        // route as if half the slots held 400-residue queries
        const int slots = s->opts.max_active > 0 ? s->opts.max_active : 64;
        std::vector<int32_t> mp(std::max(1, slots / 2), 448);
        const int resident = inter_max_grid(db->R, s->plan.tier, s->plan.strip, W) * W;
        s->g_cut = route_cut(db, s->plan, mp, resident, s->long_ids);
    }
    s->blocks = (s->g_cut + W - 1) / W;
    const int64_t cb = s->opts.chunk_groups > 0 ? (s->opts.chunk_groups + W - 1) / W
                                                : std::max<int64_t>(1, (s->blocks + 15) / 16);
    s->chunk_blocks = std::max<int64_t>(1, cb);
    s->n_chunks = s->blocks > 0 ? (s->blocks + s->chunk_blocks - 1) / s->chunk_blocks : 0;
    s->has_long = !s->long_ids.empty();
    s->n_pos = s->n_chunks + (s->has_long ? 1 : 0);
    s->slots = s->opts.max_active > 0 ? s->opts.max_active : 64;
    for (int64_t p = 0; p < s->n_chunks; ++p) {
        const int64_t g0 = p * s->chunk_blocks * W;
        const int64_t g1 = std::min(s->g_cut, (p + 1) * s->chunk_blocks * W);
        SchedPos sp;
        sp.res = db->grp_res_prefix[g1] - db->grp_res_prefix[g0];
        sp.items = std::min(s->blocks, (p + 1) * s->chunk_blocks) - p * s->chunk_blocks;
        sp.subj = (g1 - g0) * kGroup;
        s->pos.push_back(sp);
    }
    if (s->has_long) {
        SchedPos sp;
        for (int32_t id : s->long_ids) sp.res += db->len[id];
        sp.subj = (int64_t)s->long_ids.size();
        s->pos.push_back(sp);
    }
    {
        // A pass aims for the work of twelve 400-residue queries against an
        // average position (~50 ms on 5M subjects) and for eight lane-per-
        // subject items per resident workgroup: with fewer, the queue's tail
        // (workgroups idle while the last items finish) takes a large share of
        // every pass.
        int64_t tot = 0;
        for (const SchedPos &sp : s->pos) tot += sp.res;
        s->pass_cells = std::max<int64_t>(1, 12 * 400 * (tot / std::max<int64_t>(1, s->n_pos)));
        s->pass_items = 8LL * inter_max_grid(db->R, s->plan.tier, s->plan.strip, W);
    }
    if (s->opts.memory_budget <= 0) s->opts.memory_budget = (int64_t)1 << 30;
    if (s->opts.queue_capacity <= 0) s->opts.queue_capacity = 65536;
    s->prof.resize(s->slots);
    for (auto &p : s->prof) p.reset(new DevBuf());
    s->active.assign(s->slots, nullptr);
    const int64_t n = db->n_seqs;
    // the largest pass: every slot against every chunk and the long list
    const int64_t inter_items = (int64_t)s->slots * std::max<int64_t>(s->blocks, 1);
    const int per = kIntraWaves;   // the int32 layout has the most items
    const int64_t nlblk = ((int64_t)s->long_ids.size() + per - 1) / per;
    const int64_t intra_items = (int64_t)s->slots * nlblk;
    s->L = launch_config(db, s->plan, 1 << 14, std::max<int64_t>(inter_items, 1),
                         std::max<int64_t>(intra_items, 1));
    s->L16 = launch_config(db, s->plan16, 1 << 14, std::max<int64_t>(inter_items, 1),
                           std::max<int64_t>(intra_items, 1));
    s->fuse = fuse_ok(db, s->plan, s->L.Ti);
    s->grid_fused = s->fuse ? inter_max_grid(db->R, s->plan.tier, s->plan.strip, W, s->L.Ti) : 0;
    const int grid_inter_max = std::max(s->L.grid_inter, s->L16.grid_inter);
    TRY(s->d_meta.reserve((size_t)s->slots * 24 + 256));
    TRY(s->h_meta.reserve((size_t)s->slots * 24 + 256));
    std::memset(s->h_meta.p, 0, (size_t)s->slots * 24 + 256);
    TRY(s->d_scores.reserve((size_t)s->slots * n * 4 + 4));
    const int64_t chunk_subj = std::max<int64_t>(s->chunk_blocks * W * kGroup, (int64_t)s->long_ids.size());
    s->ovf_cap = (int64_t)s->slots * chunk_subj;
    TRY(s->d_ovf.reserve((size_t)s->ovf_cap * 8 + 8));
    TRY(s->d_counters.reserve(256));
    s->scr_rows = s->g_cut > 0 ? db->grp_rows[s->g_cut - 1] : 0;
    if (s->g_cut > 0)
        TRY(s->d_scr_inter.reserve((size_t)std::max(grid_inter_max, s->grid_fused) * W *
                                   s->scr_rows * 512));
    const int64_t islots = std::max<int64_t>(
        std::max<int64_t>((int64_t)s->L.grid_long * kIntraWaves, (int64_t)s->grid_fused * W),
        s->L.grid_ovf);
    TRY(s->d_scr_intra.reserve((size_t)islots * intra_scratch_rows(db) * 8));
    // a pass may hold lane-per-subject and wave-per-pair items together
    // (two sub-passes: fp16 requests, then int16 ones, each with its own half)
    s->items_half = (size_t)round_up((inter_items * 2 + intra_items * (1 + per) + 64) * 4, 256);
    TRY(s->d_items.reserve(2 * s->items_half));
    TRY(s->h_items.reserve(2 * s->items_half));
    TRY(s->d_topk.reserve(topk_work_bytes(s->slots, SW_MAX_K)));
    TRY(s->d_top.reserve((size_t)s->slots * SW_MAX_K * 12));
    TRY(s->h_top.reserve((size_t)s->slots * SW_MAX_K * 12));
    TRY(s->d_rows.reserve((size_t)s->slots * 4));
    TRY(s->h_rows.reserve((size_t)s->slots * 4));
    return SW_OK;
}

// Admit waiting requests in arrival order while a slot and the memory budget
// allow.  A request that does not fit the budget yet lets later, smaller ones
// pass it, until it has waited kAdmitAgeMs; from then on nothing passes it, so
// it is admitted as soon as enough admitted work completes.  Called with
// s->mu held; returns the newly admitted requests.
constexpr double kAdmitAgeMs = 2000.0;

std::vector<std::shared_ptr<Request>> admit(sw_server *s) {
    std::vector<std::shared_ptr<Request>> out;
    const double now = now_ms();
    for (auto it = s->waiting.begin(); it != s->waiting.end();) {
        auto &r = *it;
        int slot = -1;
        for (int i = 0; i < s->slots; ++i)
            if (!s->active[i]) {
                slot = i;
                break;
            }
        if (slot < 0) break;
        if (s->used_bytes + r->bytes > s->opts.memory_budget) {
            if (now - r->t_submit >= kAdmitAgeMs) break;
            ++it;
            continue;
        }
        r->slot = slot;
        r->next = 0;
        r->remaining = (int32_t)s->n_pos;
        r->t_admit = now;
        s->used_bytes += r->bytes;
        s->active[slot] = r;
        out.push_back(r);
        it = s->waiting.erase(it);
    }
    return out;
}

int server_pass(sw_server *s, const std::vector<std::shared_ptr<Request>> &fresh,
                std::vector<std::shared_ptr<Request>> &finished) {
    sw_db *db = s->db;
    hipStream_t st = db->stream;
    const int R = db->R;
    HIPX(hipStreamSynchronize(st));
    // profiles and per-slot metadata of newly admitted requests
    if (!fresh.empty()) {
        const int8_t **ptrs = (const int8_t **)s->h_meta.p;
        int32_t *mp = (int32_t *)(s->h_meta.as<uint8_t>() + (size_t)s->slots * 8);
        int32_t *ql = mp + s->slots;
        int32_t *gp = ql + s->slots;
        std::vector<uint8_t> staging;
        for (auto &r : fresh) {
            const int64_t L = (int64_t)r->query.size();
            const int32_t m = (int32_t)round_up(L, kQPad);
            DevBuf &pb = *s->prof[r->slot];
            // grow-only, by doubling from 2,048 columns: a slot meets longer
            // queries over time, and each reallocation frees device memory
            // (which waits for the device) between passes
            const size_t want = (size_t)R * m;
            if (want > pb.bytes) TRY(pb.reserve(std::max({want, 2 * pb.bytes, (size_t)R * 2048})));
            staging.resize((size_t)R * m);
            sw_scoring sc{db->alphabet, r->matrix.data(), r->alpha, r->beta};
            write_profile((int8_t *)staging.data(), r->query.data(), L, m, &sc, R);
            HIPX(hipMemcpy(pb.p, staging.data(), staging.size(), hipMemcpyHostToDevice));
            ptrs[r->slot] = pb.as<int8_t>();
            mp[r->slot] = m;
            ql[r->slot] = (int32_t)L;
            gp[2 * r->slot] = r->alpha;
            gp[2 * r->slot + 1] = r->beta;
        }
        HIPX(hipMemcpy(s->d_meta.p, s->h_meta.p, (size_t)s->slots * 24, hipMemcpyHostToDevice));
    }
    // This pass's work (sw_sched.h): the oldest request advances one position,
    // then shortest remaining work first, up to the pass budget.
    std::vector<Request *> act;
    for (int i = 0; i < s->slots; ++i)
        if (s->active[i] && s->active[i]->remaining > 0) act.push_back(s->active[i].get());
    if (act.empty()) return SW_OK;
    std::vector<SchedReq> sreq(act.size());
    for (size_t i = 0; i < act.size(); ++i)
        sreq[i] = SchedReq{act[i]->ticket, (int64_t)act[i]->query.size(), act[i]->next,
                           act[i]->remaining};
    std::vector<SchedTake> takes;
    sched_plan_pass(sreq, s->pos, SchedBudget{s->pass_cells, s->pass_items, s->ovf_cap}, takes);
    std::vector<PassWork> work;
    std::vector<Request *> riders;
    for (const SchedTake &t : takes) {
        Request *r = act[t.req];
        PassWork w;
        w.slot = r->slot;
        w.qlen = (int64_t)r->query.size();
        w.mpad = (int32_t)round_up(w.qlen, kQPad);
        if (t.pos < s->n_chunks) {
            w.b0 = (int64_t)t.pos * s->chunk_blocks;
            w.b1 = std::min(s->blocks, w.b0 + s->chunk_blocks);
        } else {
            w.long_list = true;
        }
        work.push_back(w);
        riders.push_back(r);
    }
    for (size_t i = 0; i < act.size(); ++i) {
        act[i]->next = sreq[i].next;
        act[i]->remaining = sreq[i].remaining;
    }
    std::sort(riders.begin(), riders.end());
    riders.erase(std::unique(riders.begin(), riders.end()), riders.end());
    // Requests whose alpha is past the fp16 tier's range run in an int16
    // sub-pass after the fp16 one (same stream, so they use the counters and
    // the overflow list one after the other).
    std::vector<PassWork> sub[2];
    for (const PassWork &w : work)
        sub[s->split_tiers && s->active[w.slot]->alpha > kFrameMaxAlpha ? 1 : 0].push_back(w);
    PassBufs pb;
    uint8_t *dm = s->d_meta.as<uint8_t>();
    pb.qs.qp = (const int8_t *const *)dm;
    pb.qs.mpad = (const int32_t *)(dm + (size_t)s->slots * 8);
    pb.qs.qlen = pb.qs.mpad + s->slots;
    pb.qs.gap = pb.qs.qlen + s->slots;
    pb.scores = s->d_scores.as<int32_t>();
    const int64_t cap = s->ovf_cap;
    pb.ovf_q = s->d_ovf.as<int32_t>();
    pb.ovf_id = pb.ovf_q + cap;
    pb.ovf_cap = cap;
    pb.counters = s->d_counters.as<int32_t>();
    pb.scr_inter = s->d_scr_inter.as<uint32_t>();
    pb.scr_rows = s->scr_rows;
    pb.scr_intra = s->d_scr_intra.as<int32_t>();
    for (int x = 0; x < 2; ++x) {
        if (sub[x].empty()) continue;
        const Plan &plan = x ? s->plan16 : s->plan;
        const Launch &base = x ? s->L16 : s->L;
        Items it;
        build_work_items(db, plan, sub[x], s->long_ids, x ? false : s->fuse, it);
        const int64_t n_inter = (int64_t)it.inter_q.size(), n_intra = (int64_t)it.intra_q.size();
        int32_t *hi = (int32_t *)(s->h_items.as<uint8_t>() + x * s->items_half);
        int32_t *di = (int32_t *)(s->d_items.as<uint8_t>() + x * s->items_half);
        std::memcpy(hi, it.inter_q.data(), n_inter * 4);
        std::memcpy(hi + n_inter, it.inter_g.data(), n_inter * 4);
        std::memcpy(hi + 2 * n_inter, it.intra_q.data(), n_intra * 4);
        std::memcpy(hi + 2 * n_inter + n_intra, it.intra_ids.data(), n_intra * it.per_item * 4);
        const size_t ib = (size_t)(2 * n_inter + n_intra * (1 + it.per_item)) * 4;
        if (ib) HIPX(hipMemcpyAsync(di, hi, ib, hipMemcpyHostToDevice, st));
        pb.it_q = di;
        pb.it_g = pb.it_q + n_inter;
        pb.il_q = pb.it_g + n_inter;
        pb.il_ids = pb.il_q + n_intra;
        pb.n_inter = n_inter;
        pb.n_intra = n_intra;
        Launch L = base;
        // columns per lane of the wave-per-pair work (long list, recompute)
        // from this sub-pass's longest query; setup sized everything for the
        // widest
        int64_t max_q = 1;
        for (const PassWork &w : sub[x]) max_q = std::max(max_q, w.qlen);
        L.Ti = intra_T_for(max_q);
        L.fused_long = it.fused && n_intra > 0;
        L.packed_long = !it.fused && it.per_item == 2 * kIntraWaves;
        L.grid_inter = L.fused_long
                           ? (int)std::min<int64_t>(n_inter + n_intra, s->grid_fused)
                           : (int)std::min<int64_t>(std::max<int64_t>(n_inter, 1), base.grid_inter);
        L.grid_long = (int)std::min<int64_t>(std::max<int64_t>(n_intra, 1), base.grid_long);
        TRY(enqueue_pass(db, L, pb, st, nullptr, nullptr, true));
    }
    // requests that visited their last position get top-k
    std::vector<int32_t> done_rows;
    for (Request *rp : riders) {
        auto &r = s->active[rp->slot];
        r->passes++;
        if (riders.size() > 1) r->shared++;
        if (r->remaining == 0) {
            finished.push_back(r);
            done_rows.push_back(r->slot);
        }
    }
    if (!done_rows.empty()) {
        const int32_t nd = (int32_t)done_rows.size();
        int32_t kmax = 0;
        for (auto &r : finished) kmax = std::max(kmax, r->k);
        int32_t *rows_h = s->h_rows.as<int32_t>();
        std::memcpy(rows_h, done_rows.data(), (size_t)nd * 4);
        HIPX(hipMemcpyAsync(s->d_rows.p, rows_h, (size_t)nd * 4, hipMemcpyHostToDevice, st));
        int64_t *d_ti = s->d_top.as<int64_t>();
        int32_t *d_ts = (int32_t *)(d_ti + (size_t)nd * kmax);
        HIPX(launch_topk(pb.scores, db->n_seqs, nd, s->d_rows.as<int32_t>(), kmax,
                         topk_work(s->d_topk.p, nd, kmax), d_ts, d_ti, st));
        int64_t *h_ti = s->h_top.as<int64_t>();
        int32_t *h_ts = (int32_t *)(h_ti + (size_t)nd * kmax);
        HIPX(hipMemcpyAsync(h_ti, d_ti, (size_t)nd * kmax * 12, hipMemcpyDeviceToHost, st));
        HIPX(hipStreamSynchronize(st));
        for (int32_t x = 0; x < nd; ++x) {
            auto &r = finished[x];
            r->top_s.assign(h_ts + (size_t)x * kmax, h_ts + (size_t)x * kmax + r->k);
            r->top_i.assign(h_ti + (size_t)x * kmax, h_ti + (size_t)x * kmax + r->k);
        }
    } else {
        HIPX(hipStreamSynchronize(st));
    }
    return SW_OK;
}

void server_loop(sw_server *s) {
    (void)hipSetDevice(s->db->device);
    for (;;) {
        std::vector<std::shared_ptr<Request>> fresh;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            auto any_active = [&] {
                for (auto &a : s->active)
                    if (a) return true;
                return false;
            };
            s->cv_work.wait(lk, [&] { return s->stop || any_active() || !s->waiting.empty(); });
            if (s->stop) break;
            fresh = admit(s);
        }
        std::vector<std::shared_ptr<Request>> finished;
        const int rc = s->n_pos > 0 ? server_pass(s, fresh, finished) : SW_OK;
        std::lock_guard<std::mutex> lk(s->mu);
        if (rc != SW_OK) {
            // a device failure ends every request in flight
            s->fatal = g_err;
            for (auto &a : s->active)
                if (a) {
                    a->rc = rc;
                    a->done = true;
                    a->t_done = now_ms();
                    s->used_bytes -= a->bytes;
                    a = nullptr;
                }
            s->cv_done.notify_all();
            continue;
        }
        if (s->n_pos == 0) {   // empty database: every admitted request is done at once
            for (auto &a : s->active)
                if (a) {
                    a->top_s.assign(a->k, -1);
                    a->top_i.assign(a->k, -1);
                    finished.push_back(a);
                }
        }
        for (auto &r : finished) {
            r->done = true;
            r->t_done = now_ms();
            s->used_bytes -= r->bytes;
            s->active[r->slot] = nullptr;
        }
        if (!finished.empty()) s->cv_done.notify_all();
    }
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &a : s->active)
        if (a && !a->done) {
            a->rc = SW_ESTOPPED;
            a->done = true;
        }
    for (auto &w : s->waiting) {
        w->rc = SW_ESTOPPED;
        w->done = true;
    }
    s->waiting.clear();
    s->cv_done.notify_all();
}

}  // namespace

// ===========================================================================
// Database layout (section III, stage ii and the offline index): validation,
// the host-side packing into length-sorted groups, and the upload.
// ===========================================================================
namespace {

int validate_db(const uint8_t *residues, const int64_t *offsets, int64_t n_seqs, int32_t alphabet) {
    if (n_seqs < 0) return fail(SW_EINVAL, "n_seqs < 0");
    if (n_seqs > INT32_MAX - 1) return fail(SW_EINVAL, "too many sequences");
    if (alphabet < 1 || alphabet > SW_MAX_ALPHABET)
        return fail(SW_EINVAL, "alphabet %d not in 1..%d", alphabet, SW_MAX_ALPHABET);
    if (!offsets) return fail(SW_EINVAL, "offsets is NULL");
    if (offsets[0] != 0) return fail(SW_EINVAL, "offsets[0] != 0");
    for (int64_t i = 0; i < n_seqs; ++i) {
        const int64_t L = offsets[i + 1] - offsets[i];
        if (L < 0) return fail(SW_EINVAL, "offsets decrease at %lld", (long long)i);
        if (L > SW_MAX_LEN) return fail(SW_EINVAL, "sequence %lld longer than 2^24", (long long)i);
    }
    const int64_t total = offsets[n_seqs];
    if (total > 0 && !residues) return fail(SW_EINVAL, "residues is NULL");
    // Code check, split over threads for big databases.
    const int nth = (int)std::max<int64_t>(1, std::min<int64_t>(16, total >> 24));
    std::vector<int64_t> bad(nth, -1);
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
        th.emplace_back([&, t] {
            const int64_t lo = total * t / nth, hi = total * (t + 1) / nth;
            for (int64_t i = lo; i < hi; ++i)
                if (residues[i] >= alphabet) {
                    bad[t] = i;
                    return;
                }
        });
    for (auto &x : th) x.join();
    for (int t = 0; t < nth; ++t)
        if (bad[t] >= 0)
            return fail(SW_EINVAL, "residue code %d at %lld >= alphabet %d", residues[bad[t]],
                        (long long)bad[t], alphabet);
    return SW_OK;
}

// A handle with its streams and events on `device`, and no database yet.
int db_create(int device, int32_t alphabet, std::unique_ptr<sw_db> &out) {
    std::unique_ptr<sw_db> db(new sw_db());
    db->device = device;
    db->alphabet = alphabet;
    db->R = alphabet + 1;
    // Check the multiply-shift division used for pair codes.
    {
        const int R = db->R, magic = (65536 + R - 1) / R;
        for (int a = 0; a < R * R; ++a)
            if (((a * magic) >> 16) != a / R) return fail(SW_EINVAL, "internal: division check failed");
    }
    HIPX(hipSetDevice(db->device));
    {
        hipDeviceProp_t p;
        HIPX(hipGetDeviceProperties(&p, db->device));
        db->cus = p.multiProcessorCount;
        db->arch = p.gcnArchName;
    }
    HIPX(prepare_kernels());
    HIPX(noalloc_scratch_init(db->device));
    HIPX(hipStreamCreateWithFlags(&db->stream, hipStreamNonBlocking));
    HIPX(hipStreamCreateWithFlags(&db->aux, hipStreamNonBlocking));
    for (auto &e : db->ev) HIPX(hipEventCreate(&e));
    HIPX(hipEventCreateWithFlags(&db->fork, hipEventDisableTiming));
    HIPX(hipEventCreateWithFlags(&db->join, hipEventDisableTiming));
    out = std::move(db);
    return SW_OK;
}

// Host side of the device layout: subjects stable-sorted by length; the
// longest (or, for a database too small to give every SIMD a wavefront,
// all) form the long list; the rest are dealt into groups of 128 whose pair
// codes are interleaved [chunk of 4 rows][lane][row] and padded with the
// zero-score residue (the dummy residue of section III.B.1).
// long_threshold as in sw_db_opts; cus: compute units of the target device.
int pack_db(const uint8_t *residues, const int64_t *offsets, int64_t n_seqs, int32_t alphabet,
            int32_t long_threshold, int cus, Packed &pk) {
    pk = Packed{};
    pk.n_seqs = n_seqs;
    pk.alphabet = alphabet;
    pk.total_res = offsets[n_seqs];
    const int R = alphabet + 1;
    pk.len.resize(n_seqs);
    for (int64_t i = 0; i < n_seqs; ++i) {
        pk.len[i] = offsets[i + 1] - offsets[i];
        pk.max_len = std::max(pk.max_len, pk.len[i]);
    }
    std::vector<int32_t> order(n_seqs);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return pk.len[x] < pk.len[y]; });

    // ---- split: lane-per-subject groups vs the long list ----
    const int64_t simds = 4LL * cus;
    int64_t cut;   // subjects longer than cut go to the long list
    pk.fixed_cut = long_threshold != 0;
    if (long_threshold == -1) cut = INT64_MAX;
    else if (long_threshold == 1) cut = -1;
    else if (long_threshold > 1) cut = long_threshold;
    else if (n_seqs < simds * kGroup) cut = -1;   // cannot give every SIMD a wavefront
    else cut = kGroupMaxLen;   // each search routes its own cut below this (route_cut)
    int64_t n_short = 0;
    while (n_short < n_seqs && pk.len[order[n_short]] <= cut) ++n_short;
    pk.long_threshold = cut;
    for (int64_t i = n_seqs - 1; i >= n_short; --i) {
        pk.long_ids.push_back(order[i]);
        pk.long_res += pk.len[order[i]];
    }

    // ---- groups of 128 (lane l: lo = 128g + l, hi = 128g + 64 + l) ----
    const int32_t ng = (int32_t)((n_short + kGroup - 1) / kGroup);
    pk.n_groups = ng;
    pk.gbase.resize(ng);
    pk.grp_ids.assign((size_t)ng * kGroup, -1);
    pk.grp_rows.resize(ng);
    int64_t codes_total = 0;
    for (int32_t g = 0; g < ng; ++g) {
        const int64_t last = std::min<int64_t>(n_short, (int64_t)(g + 1) * kGroup) - 1;
        const int64_t rows = std::max<int64_t>(kChunk, round_up(pk.len[order[last]], kChunk));
        pk.grp_rows[g] = (int32_t)rows;
        pk.gbase[g] = codes_total;
        codes_total += rows * kWave;
        pk.max_rows = std::max<int32_t>(pk.max_rows, (int32_t)rows);
        pk.inter_padded_rows += rows * kGroup;
        pk.grp_res_prefix.push_back(pk.inter_res);
        for (int x = 0; x < kGroup; ++x) {
            const int64_t si = (int64_t)g * kGroup + x;
            if (si < n_short) {
                pk.grp_ids[(size_t)g * kGroup + x] = order[si];
                pk.inter_res += pk.len[order[si]];
            }
        }
    }
    pk.grp_res_prefix.push_back(pk.inter_res);
    pk.codes.resize((size_t)codes_total);
    const int nth = (int)std::max(1, std::min(16, ng / 64));
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
        th.emplace_back([&, t] {
            const uint16_t padc = (uint16_t)(R - 1);
            for (int32_t g = t; g < ng; g += nth) {
                const int64_t rows = pk.grp_rows[g];
                uint16_t *dst = pk.codes.data() + pk.gbase[g];
                for (int l = 0; l < kWave; ++l) {
                    const int32_t lo = pk.grp_ids[(size_t)g * kGroup + l];
                    const int32_t hi = pk.grp_ids[(size_t)g * kGroup + kWave + l];
                    const uint8_t *slo = lo >= 0 ? residues + offsets[lo] : nullptr;
                    const uint8_t *shi = hi >= 0 ? residues + offsets[hi] : nullptr;
                    const int64_t nlo = lo >= 0 ? pk.len[lo] : 0, nhi = hi >= 0 ? pk.len[hi] : 0;
                    for (int64_t i = 0; i < rows; ++i) {
                        const uint16_t a = i < nlo ? slo[i] : padc;
                        const uint16_t b = i < nhi ? shi[i] : padc;
                        // chunk i/4, lane l, row i%4
                        dst[(i / kChunk) * (kWave * kChunk) + l * kChunk + (i % kChunk)] =
                            (uint16_t)(a * R + b);
                    }
                }
            }
        });
    for (auto &x : th) x.join();
    return SW_OK;
}

// A packed database in memory: the arrays of a Packed, or of one chunk of an
// on-disk index (mapped).
struct PackedView {
    int64_t n_seqs = 0, total_res = 0, max_len = 0;
    int64_t long_res = 0, long_threshold = 0, inter_res = 0, inter_padded_rows = 0;
    int32_t n_groups = 0, max_rows = 0, n_long = 0;
    bool fixed_cut = false;
    int64_t n_codes = 0;
    const uint8_t *residues = nullptr;
    const int64_t *offsets = nullptr;        // n_seqs + 1
    const int32_t *long_ids = nullptr;       // n_long
    const int32_t *grp_rows = nullptr;       // n_groups
    const int32_t *grp_ids = nullptr;        // n_groups * 128
    const int64_t *grp_res_prefix = nullptr; // n_groups + 1
    const int64_t *gbase = nullptr;          // n_groups
    const uint16_t *codes = nullptr;         // n_codes
};

PackedView view_of(const Packed &pk, const uint8_t *residues, const int64_t *offsets) {
    PackedView v;
    v.n_seqs = pk.n_seqs;
    v.total_res = pk.total_res;
    v.max_len = pk.max_len;
    v.long_res = pk.long_res;
    v.long_threshold = pk.long_threshold;
    v.inter_res = pk.inter_res;
    v.inter_padded_rows = pk.inter_padded_rows;
    v.n_groups = pk.n_groups;
    v.max_rows = pk.max_rows;
    v.n_long = (int32_t)pk.long_ids.size();
    v.fixed_cut = pk.fixed_cut;
    v.n_codes = (int64_t)pk.codes.size();
    v.residues = residues;
    v.offsets = offsets;
    v.long_ids = pk.long_ids.data();
    v.grp_rows = pk.grp_rows.data();
    v.grp_ids = pk.grp_ids.data();
    v.grp_res_prefix = pk.grp_res_prefix.data();
    v.gbase = pk.gbase.data();
    v.codes = pk.codes.data();
    return v;
}

// Device bytes of a packed database (residues, offsets, codes, group tables,
// long list).
int64_t view_device_bytes(const PackedView &v) {
    return v.total_res + (v.n_seqs + 1) * 8 + v.n_codes * 2 +
           (int64_t)v.n_groups * (8 + 4 + kGroup * 4) + (int64_t)v.n_long * 4;
}

// Make `db` the packed database `v`: host fields copied from it, device
// copies on `st`, waited for before returning (v's memory may go away then).
// Device buffers only grow, so a handle reloaded with chunk after chunk keeps
// the largest chunk's allocation.
int db_install(sw_db *db, const PackedView &v, hipStream_t st) {
    HIPX(hipSetDevice(db->device));
    if (db->graph) {
        (void)hipGraphExecDestroy(db->graph);
        db->graph = nullptr;
        db->graph_key.clear();
    }
    const int64_t n = v.n_seqs, total = v.total_res;
    const int32_t ng = v.n_groups;
    db->n_seqs = n;
    db->total_res = total;
    db->max_len = v.max_len;
    db->len.resize(n);
    for (int64_t i = 0; i < n; ++i) db->len[i] = v.offsets[i + 1] - v.offsets[i];
    db->n_groups = ng;
    db->max_rows = v.max_rows;
    db->grp_rows.assign(v.grp_rows, v.grp_rows + ng);
    db->inter_res = v.inter_res;
    db->inter_padded_rows = v.inter_padded_rows;
    db->grp_res_prefix.assign(v.grp_res_prefix, v.grp_res_prefix + ng + 1);
    db->long_ids.assign(v.long_ids, v.long_ids + v.n_long);
    db->long_res = v.long_res;
    db->long_threshold = v.long_threshold;
    db->fixed_cut = v.fixed_cut;
    db->grp_ids.assign(v.grp_ids, v.grp_ids + (size_t)ng * kGroup);
    db->tuned.clear();
    {
        char sig[512];
        snprintf(sig, sizeof sig, "%s|cu%d|n%lld|res%lld|A%d|max%lld", db->arch.c_str(), db->cus,
                 (long long)n, (long long)total, db->alphabet, (long long)db->max_len);
        db->signature = sig;
    }
    TRY(db->d_res.reserve((size_t)std::max<int64_t>(total, 1)));
    TRY(db->d_off.reserve((size_t)(n + 1) * 8));
    if (total > 0) HIPX(hipMemcpyAsync(db->d_res.p, v.residues, (size_t)total, hipMemcpyHostToDevice, st));
    HIPX(hipMemcpyAsync(db->d_off.p, v.offsets, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, st));
    if (ng > 0) {
        TRY(db->d_codes.reserve((size_t)v.n_codes * 2));
        TRY(db->d_grp_base.reserve((size_t)ng * 8));
        TRY(db->d_grp_rows.reserve((size_t)ng * 4));
        TRY(db->d_grp_ids.reserve((size_t)ng * kGroup * 4));
        HIPX(hipMemcpyAsync(db->d_codes.p, v.codes, (size_t)v.n_codes * 2, hipMemcpyHostToDevice, st));
        HIPX(hipMemcpyAsync(db->d_grp_base.p, v.gbase, (size_t)ng * 8, hipMemcpyHostToDevice, st));
        HIPX(hipMemcpyAsync(db->d_grp_rows.p, v.grp_rows, (size_t)ng * 4, hipMemcpyHostToDevice, st));
        HIPX(hipMemcpyAsync(db->d_grp_ids.p, v.grp_ids, (size_t)ng * kGroup * 4,
                            hipMemcpyHostToDevice, st));
    }
    if (v.n_long > 0) {
        TRY(db->d_long_ids.reserve((size_t)v.n_long * 4));
        HIPX(hipMemcpyAsync(db->d_long_ids.p, v.long_ids, (size_t)v.n_long * 4,
                            hipMemcpyHostToDevice, st));
    }
    HIPX(hipStreamSynchronize(st));
    return SW_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *sw_last_error(void) { return g_err.c_str(); }

const char *sw_version(void) { return "swmi 0.2 (gfx950)"; }

int sw_db_open(const uint8_t *residues, const int64_t *offsets, int64_t n_seqs, int32_t alphabet,
               const sw_db_opts *opts, sw_db **out) {
    g_err.clear();
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = nullptr;
    TRY(validate_db(residues, offsets, n_seqs, alphabet));
    const int device = opts && opts->device > 0 ? opts->device : 0;
    std::unique_ptr<sw_db> db;
    TRY(db_create(device, alphabet, db));
    Packed pk;
    TRY(pack_db(residues, offsets, n_seqs, alphabet, opts ? opts->long_threshold : 0, db->cus, pk));
    TRY(db_install(db.get(), view_of(pk, residues, offsets), db->stream));
    *out = db.release();
    return SW_OK;
}

void sw_db_close(sw_db *db) {
    if (!db) return;
    (void)hipSetDevice(db->device);
    if (db->stream) (void)hipStreamSynchronize(db->stream);
    if (db->graph) (void)hipGraphExecDestroy(db->graph);
    if (db->aux) (void)hipStreamSynchronize(db->aux);
    for (auto &e : db->ev)
        if (e) (void)hipEventDestroy(e);
    if (db->fork) (void)hipEventDestroy(db->fork);
    if (db->join) (void)hipEventDestroy(db->join);
    if (db->stream) (void)hipStreamDestroy(db->stream);
    if (db->aux) (void)hipStreamDestroy(db->aux);
    delete db;
}

int64_t sw_db_size(const sw_db *db) { return db ? db->n_seqs : -1; }

int sw_db_set_opts(sw_db *db, const sw_search_opts *opts) {
    g_err.clear();
    if (!db) return fail(SW_EINVAL, "db is NULL");
    std::lock_guard<std::mutex> lk(db->mu);
    if (!opts) {
        db->opts = sw_search_opts{};
        return SW_OK;
    }
    if (opts->tier < 0 || opts->tier > 2) return fail(SW_EINVAL, "tier not in 0..2");
    if (opts->strip && opts->strip != 16 && opts->strip != 32 && opts->strip != 64)
        return fail(SW_EINVAL, "strip must be 16, 32 or 64");
    if (opts->waves && opts->waves != 4 && opts->waves != 6 && opts->waves != 8)
        return fail(SW_EINVAL, "waves must be 4, 6 or 8");
    if (opts->strip == 64 && opts->waves && opts->waves != 4)
        return fail(SW_EINVAL, "strip 64 runs with 4 waves per workgroup");
    if (opts->waves == 6 && opts->strip && opts->strip != 32)
        return fail(SW_EINVAL, "6 waves per workgroup runs with strip 32");
    if (opts->sat_threshold < 0) return fail(SW_EINVAL, "sat_threshold < 0");
    if (opts->graph < -1 || opts->graph > 0) return fail(SW_EINVAL, "graph must be 0 or -1");
    if (opts->profile != SW_PROFILE_PAIR && opts->profile != SW_PROFILE_SCORE)
        return fail(SW_EINVAL, "profile must be SW_PROFILE_PAIR or SW_PROFILE_SCORE");
    db->opts = *opts;
    return SW_OK;
}

int sw_db_last_stats(sw_db *db, sw_stats *out) {
    g_err.clear();
    if (!db || !out) return fail(SW_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(db->mu);
    *out = db->last;
    return SW_OK;
}

static int busy(sw_db *db) {
    return db->server_attached ? fail(SW_EBUSY, "a server is running on this database") : SW_OK;
}

int sw_db_search(sw_db *db, const uint8_t *query, int32_t qlen, const sw_scoring *sc,
                 int32_t *scores, void *hip_stream) {
    g_err.clear();
    if (!db) return fail(SW_EINVAL, "db is NULL");
    if (!scores && db->n_seqs > 0) return fail(SW_EINVAL, "scores is NULL");
    std::lock_guard<std::mutex> lk(db->mu);
    TRY(busy(db));
    const int64_t off[2] = {0, qlen};
    return run_search(db, 1, query, off, sc, 0, nullptr, nullptr, scores, nullptr,
                      (hipStream_t)hip_stream);
}

int sw_db_search_dev(sw_db *db, const uint8_t *query, int32_t qlen, const sw_scoring *sc,
                     int32_t *scores_dev, void *hip_stream) {
    g_err.clear();
    if (!db) return fail(SW_EINVAL, "db is NULL");
    if (!scores_dev && db->n_seqs > 0) return fail(SW_EINVAL, "scores_dev is NULL");
    std::lock_guard<std::mutex> lk(db->mu);
    TRY(busy(db));
    const int64_t off[2] = {0, qlen};
    return run_search(db, 1, query, off, sc, 0, nullptr, nullptr, nullptr, scores_dev,
                      (hipStream_t)hip_stream);
}

// The search of sw_db_search_dev with every buffer in the device's fixed
// scratch array: no hipMalloc, hipFree, pinned staging or host container.
// The plan, the cut and the grids are worked out on the host from numbers
// alone; the profile, query set and work lists are written by one setup
// kernel; then the same pass as every other search runs.  Grids shrink until
// their boundary and pass buffers fit what the fixed parts leave.
int sw_db_search_dev_noalloc(sw_db *db, const uint8_t *query_dev, int32_t qlen,
                             const sw_scoring *sc, int32_t *scores_dev, void *hip_stream) {
    g_err.clear();
    if (!db) return fail(SW_EINVAL, "db is NULL");
    if (!query_dev) return fail(SW_EINVAL, "query_dev is NULL");
    if (qlen < 1 || qlen > SW_MAX_LEN) return fail(SW_EINVAL, "query length %d not in 1..2^24", qlen);
    if (!scores_dev && db->n_seqs > 0) return fail(SW_EINVAL, "scores_dev is NULL");
    std::lock_guard<std::mutex> lk(db->mu);
    TRY(busy(db));
    TRY(validate_scoring(db, sc));
    HIPX(hipSetDevice(db->device));
    uint8_t *base = noalloc_scratch(db->device);
    if (!base) return fail(SW_EDEVICE, "no-allocation scratch not initialised on device %d", db->device);
    hipStream_t st = hip_stream ? (hipStream_t)hip_stream : db->stream;
    const int64_t n = db->n_seqs;
    if (n == 0) return SW_OK;

    Plan plan = plan_for(db, qlen, sc->alpha);
    plan.profile = SW_PROFILE_PAIR;   // the fixed scratch holds no query codes
    const int W = plan.waves;
    const int32_t mpad = (int32_t)round_up(qlen, kQPad);
    const int resident = inter_max_grid(db->R, plan.tier, plan.strip, W) * W;
    const int64_t g_cut = route_cut_groups(db, plan, &mpad, 1, resident);
    const int64_t n_inter = (g_cut + W - 1) / W;
    const int64_t n_long = (int64_t)db->long_ids.size() + (db->n_groups - g_cut) * kGroup;
    const int Ti = intra_T_for(qlen);
    const int pw = intra_per_wave(plan, n_long, db->cus, n_inter == 0, Ti);
    const bool fused = fuse_ok(db, plan, Ti) && pw == 1;
    const int per = fused ? W : kIntraWaves * pw;
    const int64_t n_intra = (n_long + per - 1) / per;
    Launch L = launch_config(db, plan, qlen, n_inter, n_intra, fused);
    L.packed_long = !fused && per == 2 * kIntraWaves;
    const int32_t rows_alloc = g_cut > 0 ? db->grp_rows[g_cut - 1] : 0;

    // ---- fixed parts of the scratch ----
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += (size_t)round_up((int64_t)bytes, 256);
        return at;
    };
    const size_t o_ctr = take(16);
    const size_t o_qs = take(8 + 4 + 4 + 8);
    const size_t o_prof = take((size_t)db->R * mpad);
    const size_t o_it = take((size_t)n_inter * 8);
    const size_t o_il = take((size_t)n_intra * (1 + per) * 4);
    const size_t o_ovf = take((size_t)n * 8);
    if (o + 512 > kNoAllocScratchBytes)
        return fail(SW_EINVAL, "query of %d residues against %lld subjects needs %zu bytes of fixed "
                    "state, more than the %zu-byte no-allocation scratch", qlen, (long long)n, o,
                    kNoAllocScratchBytes);
    // ---- grids within what is left ----
    // what is left, less the alignment of the two regions below
    const size_t rem = kNoAllocScratchBytes - o - 512;
    const size_t per_slot = (size_t)intra_scratch_rows(db) * 8;        // one wave-per-pair wave
    const size_t per_wg = (size_t)W * rows_alloc * 512;               // one lane-per-subject workgroup
    int64_t grid_inter = 0, slots = 0;
    const bool inter_launch = n_inter > 0 || L.fused_long;
    if (inter_launch) {
        if (fused) {
            grid_inter = std::min<int64_t>(L.grid_inter, (int64_t)(rem / (per_wg + (size_t)W * per_slot)));
            slots = grid_inter * W;
        } else {
            const size_t want_i = (size_t)std::max<int64_t>((int64_t)L.grid_long * kIntraWaves,
                                                            L.grid_ovf) * per_slot;
            const size_t keep_i = std::max(per_slot * kIntraWaves, std::min(want_i, rem / 4));
            grid_inter = keep_i < rem ? std::min<int64_t>(L.grid_inter, (int64_t)((rem - keep_i) / per_wg)) : 0;
            slots = (int64_t)((rem - (size_t)grid_inter * per_wg) / per_slot);
        }
    } else {
        slots = (int64_t)(rem / per_slot);
    }
    const int64_t grid_long = std::min<int64_t>(L.grid_long, slots / kIntraWaves);
    const int64_t grid_ovf = std::min<int64_t>(L.grid_ovf, slots);
    if ((inter_launch && grid_inter < 1) || (n_intra > 0 && !fused && grid_long < 1) || grid_ovf < 1)
        return fail(SW_EINVAL, "query of %d residues against this database does not fit the "
                    "%zu-byte no-allocation scratch (groups of up to %d rows, subjects of up to "
                    "%lld residues)", qlen, kNoAllocScratchBytes, rows_alloc, (long long)db->max_len);
    L.grid_inter = (int)grid_inter;
    L.grid_long = (int)grid_long;
    L.grid_ovf = (int)grid_ovf;
    const size_t o_b = take((size_t)grid_inter * per_wg);
    const size_t o_i = take((size_t)std::max<int64_t>(slots, 1) * per_slot);
    (void)o_i;

    NoAllocSetup su{};
    su.q = query_dev;
    su.qlen = qlen;
    su.mpad = mpad;
    su.R = db->R;
    su.A = db->alphabet;
    std::memcpy(su.matrix, sc->matrix, (size_t)db->alphabet * db->alphabet);
    su.alpha = sc->alpha;
    su.beta = sc->beta;
    su.prof = (int8_t *)(base + o_prof);
    su.qp = (const int8_t **)(base + o_qs);
    su.mpad_out = (int32_t *)(base + o_qs + 8);
    su.qlen_out = (int32_t *)(base + o_qs + 12);
    su.gap_out = (int32_t *)(base + o_qs + 16);
    su.it_q = (int32_t *)(base + o_it);
    su.it_g = su.it_q + n_inter;
    su.n_inter = (int32_t)n_inter;
    su.waves = W;
    su.il_q = (int32_t *)(base + o_il);
    su.il_ids = su.il_q + n_intra;
    su.n_intra = (int32_t)n_intra;
    su.per = per;
    su.long_static = db->d_long_ids.as<int32_t>();
    su.n_static = (int32_t)db->long_ids.size();
    su.grp_ids = db->d_grp_ids.as<int32_t>();
    su.g_cut = (int32_t)g_cut;
    su.n_groups = db->n_groups;
    HIPX(launch_noalloc_setup(su, st));

    PassBufs pb;
    pb.qs.qp = su.qp;
    pb.qs.mpad = su.mpad_out;
    pb.qs.qlen = su.qlen_out;
    pb.qs.gap = su.gap_out;
    pb.it_q = su.it_q;
    pb.it_g = su.it_g;
    pb.il_q = su.il_q;
    pb.il_ids = su.il_ids;
    pb.n_inter = n_inter;
    pb.n_intra = n_intra;
    pb.scores = scores_dev;
    pb.ovf_q = (int32_t *)(base + o_ovf);
    pb.ovf_id = pb.ovf_q + n;
    pb.ovf_cap = n;
    pb.counters = (int32_t *)(base + o_ctr);
    pb.scr_inter = (uint32_t *)(base + o_b);
    pb.scr_rows = rows_alloc;
    pb.scr_intra = (int32_t *)(base + o_i);
    TRY(enqueue_pass(db, L, pb, st));
    if (!hip_stream) HIPX(hipStreamSynchronize(st));
    sw_stats &stt = db->last;
    stt = sw_stats{};
    stt.cells = (int64_t)qlen * db->total_res;
    stt.inter_cells = (int64_t)qlen * db->grp_res_prefix[g_cut];
    stt.intra_pairs = (int64_t)db->long_ids.size() +
                      std::max<int64_t>(0, n - (int64_t)db->long_ids.size() - g_cut * kGroup);
    stt.kernel_ms = stt.total_ms = stt.inter_ms = stt.recompute_ms = stt.long_ms = -1;
    stt.recomputed_pairs = -1;   // not read back (nothing is copied to the host)
    stt.tier = plan.tier;
    stt.strip = plan.strip;
    stt.waves = W;
    stt.fused_long = L.fused_long ? 1 : 0;
    return SW_OK;
}

int sw_db_topk(sw_db *db, const uint8_t *query, int32_t qlen, const sw_scoring *sc, int32_t k,
               int32_t *top_scores, int64_t *top_idx, void *hip_stream) {
    g_err.clear();
    if (!db) return fail(SW_EINVAL, "db is NULL");
    if (k < 1 || k > SW_MAX_K) return fail(SW_EINVAL, "k not in 1..%d", SW_MAX_K);
    if (!top_scores || !top_idx) return fail(SW_EINVAL, "top-k outputs are NULL");
    std::lock_guard<std::mutex> lk(db->mu);
    TRY(busy(db));
    const int64_t off[2] = {0, qlen};
    return run_search(db, 1, query, off, sc, k, top_scores, top_idx, nullptr, nullptr,
                      (hipStream_t)hip_stream);
}

int sw_db_search_batch(sw_db *db, int32_t nq, const uint8_t *q_res, const int64_t *q_off,
                       const sw_scoring *sc, int32_t k, int32_t *top_scores, int64_t *top_idx,
                       int32_t *all_scores, void *hip_stream) {
    g_err.clear();
    if (!db) return fail(SW_EINVAL, "db is NULL");
    if (k < 1 || k > SW_MAX_K) return fail(SW_EINVAL, "k not in 1..%d", SW_MAX_K);
    if (!top_scores || !top_idx) return fail(SW_EINVAL, "top-k outputs are NULL");
    std::lock_guard<std::mutex> lk(db->mu);
    TRY(busy(db));
    return run_search(db, nq, q_res, q_off, sc, k, top_scores, top_idx, all_scores, nullptr,
                      (hipStream_t)hip_stream, 1, true);
}

// Alignment with traceback: direction bytes are kept for every cell of a
// batch's pairs, so pairs go in batches of at most kAlignBatchBytes of them
// (a single larger pair runs alone, up to kAlignMaxPairBytes).
namespace {
constexpr size_t kAlignBatchBytes = (size_t)1 << 30;
constexpr size_t kAlignMaxPairBytes = (size_t)16 << 30;

int align_pairs(sw_db *db, const uint8_t *query, int64_t qlen, const sw_scoring *sc,
                const int64_t *ids, int32_t n_ids, sw_alignment *out, uint32_t *ops) {
    const int R = db->R;
    const int32_t mpad = (int32_t)round_up(qlen, kQPad);
    const int32_t ldq = (int32_t)round_up(qlen, 16);
    hipStream_t st = db->stream;
    const int64_t max_len_pad = intra_scratch_rows(db);
    int64_t ops_pos = 0;
    for (int32_t b0 = 0; b0 < n_ids;) {
        // this batch: [b0, b1)
        int32_t b1 = b0;
        size_t dir_bytes = 0, ops_n = 0;
        while (b1 < n_ids) {
            const size_t pb = (size_t)db->len[ids[b1]] * (size_t)ldq;
            if (pb > kAlignMaxPairBytes)
                return fail(SW_ENOMEM, "alignment of subject %lld needs %zu bytes of traceback",
                            (long long)ids[b1], pb);
            if (b1 > b0 && dir_bytes + pb > kAlignBatchBytes) break;
            dir_bytes += pb;
            ops_n += (size_t)db->len[ids[b1]] + (size_t)qlen;
            ++b1;
        }
        const int32_t nb = b1 - b0;
        const size_t meta_bytes = (size_t)nb * (3 * 8 + 3 * 4 + 6 * 4) + (size_t)R * mpad + 256;
        // Buffers grow by half again at least (the direction bytes up to a
        // batch's bound): calls whose sizes creep up, as for queries of
        // growing length, would otherwise free and allocate on every call.
        auto grown = [](size_t want, const DevBuf &b, size_t cap) {
            return want <= b.bytes ? want : std::max(want, std::min(cap, b.bytes + b.bytes / 2));
        };
        TRY(db->w_al_meta.reserve(grown(meta_bytes, db->w_al_meta, SIZE_MAX)));
        TRY(db->h_al.reserve(std::max(meta_bytes, db->w_al_meta.bytes)));
        TRY(db->w_al_dir.reserve(grown(std::max<size_t>(dir_bytes, 16), db->w_al_dir, kAlignBatchBytes)));
        TRY(db->w_al_ops.reserve(grown(std::max<size_t>(ops_n * 4, 4), db->w_al_ops, SIZE_MAX)));
        const int grid = (nb + kAlignWaves - 1) / kAlignWaves;
        TRY(db->w_al_scr.reserve(grown((size_t)grid * kAlignWaves * (size_t)max_len_pad * 8, db->w_al_scr,
                                       SIZE_MAX)));
        // host staging: ids, dir offsets, ops offsets (int64), then the profile
        HIPX(hipStreamSynchronize(st));
        uint8_t *h = db->h_al.as<uint8_t>();
        int64_t *h_ids = (int64_t *)h, *h_doff = h_ids + nb, *h_ooff = h_doff + nb;
        int8_t *h_prof = (int8_t *)(h_ooff + nb);
        size_t d_acc = 0, o_acc = 0;
        for (int32_t k = 0; k < nb; ++k) {
            const int64_t id = ids[b0 + k];
            h_ids[k] = id;
            h_doff[k] = (int64_t)d_acc;
            h_ooff[k] = (int64_t)o_acc;
            d_acc += (size_t)db->len[id] * (size_t)ldq;
            o_acc += (size_t)db->len[id] + (size_t)qlen;
        }
        write_profile(h_prof, query, qlen, mpad, sc, R);
        const size_t stage = (size_t)nb * 24 + (size_t)R * mpad;
        uint8_t *d = db->w_al_meta.as<uint8_t>();
        HIPX(hipMemcpyAsync(d, h, stage, hipMemcpyHostToDevice, st));
        int32_t *d_end = (int32_t *)(d + round_up((int64_t)stage, 16));
        int32_t *d_out = d_end + 3 * (size_t)nb;
        AlignArgs a{};
        a.res = db->d_res.as<uint8_t>();
        a.off = db->d_off.as<int64_t>();
        a.ids = (const int64_t *)d;
        a.n_pairs = nb;
        a.qp = (const int8_t *)(d + (size_t)nb * 24);
        a.mpad = mpad;
        a.qlen = (int32_t)qlen;
        a.ldq = ldq;
        a.alpha = sc->alpha;
        a.beta = sc->beta;
        a.R = R;
        a.dir = db->w_al_dir.as<uint8_t>();
        a.dir_off = a.ids + nb;
        a.pass_scratch = db->w_al_scr.as<int32_t>();
        a.max_len_pad = max_len_pad;
        a.end = d_end;
        a.ops = db->w_al_ops.as<uint32_t>();
        a.ops_off = a.ids + 2 * (size_t)nb;
        a.out = d_out;
        HIPX(launch_align(a, st));
        // results: per pair 6 int32, then the runs of each pair
        std::vector<int32_t> res((size_t)nb * 6);
        HIPX(hipMemcpyAsync(res.data(), d_out, res.size() * 4, hipMemcpyDeviceToHost, st));
        std::vector<uint32_t> runs(o_acc);
        if (o_acc) HIPX(hipMemcpyAsync(runs.data(), a.ops, o_acc * 4, hipMemcpyDeviceToHost, st));
        HIPX(hipStreamSynchronize(st));
        for (int32_t k = 0; k < nb; ++k) {
            const int32_t *r = &res[(size_t)k * 6];
            if (r[5] < 0)
                return fail(SW_EDEVICE, "traceback of subject %lld left its bounds",
                            (long long)ids[b0 + k]);
            sw_alignment &o = out[b0 + k];
            o.score = r[0];
            o.q_begin = r[1];
            o.q_end = r[2];
            o.s_begin = r[3];
            o.s_end = r[4];
            o.n_ops = r[5];
            o.ops_offset = ops_pos;
            std::memcpy(ops + ops_pos, runs.data() + h_ooff[k], (size_t)r[5] * 4);
            ops_pos += r[5];
        }
        b0 = b1;
    }
    return SW_OK;
}
}  // namespace

int sw_db_align(sw_db *db, const uint8_t *query, int32_t qlen, const sw_scoring *sc,
                const int64_t *ids, int32_t n_ids, sw_alignment *out, uint32_t *ops,
                int64_t ops_cap, int64_t *ops_needed) {
    g_err.clear();
    if (!db) return fail(SW_EINVAL, "db is NULL");
    TRY(validate_scoring(db, sc));
    TRY(validate_query(db, query, qlen));
    if (n_ids < 0 || (n_ids > 0 && (!ids || !out))) return fail(SW_EINVAL, "bad id list or output");
    int64_t need = 0;
    for (int32_t k = 0; k < n_ids; ++k) {
        if (ids[k] < 0 || ids[k] >= db->n_seqs)
            return fail(SW_EINVAL, "id %lld not in 0..%lld", (long long)ids[k],
                        (long long)db->n_seqs - 1);
        need += db->len[ids[k]] + qlen;
    }
    if (ops_needed) *ops_needed = need;
    if (ops_cap < need || (need > 0 && !ops))
        return fail(SW_EINVAL, "ops holds %lld runs, the alignments may need %lld", (long long)ops_cap,
                    (long long)need);
    std::lock_guard<std::mutex> lk(db->mu);
    TRY(busy(db));
    HIPX(hipSetDevice(db->device));
    return align_pairs(db, query, qlen, sc, ids, n_ids, out, ops);
}

int sw_db_autotune(sw_db *db, const sw_scoring *sc, const int32_t *qlens, int32_t n_qlens,
                   const char *cache_path) {
    g_err.clear();
    if (!db) return fail(SW_EINVAL, "db is NULL");
    std::lock_guard<std::mutex> lk(db->mu);
    TRY(busy(db));
    return autotune(db, sc, qlens, n_qlens, cache_path);
}

int sw_server_start(sw_db *db, const sw_server_opts *opts, sw_server **out) {
    g_err.clear();
    if (!db || !out) return fail(SW_EINVAL, "NULL argument");
    *out = nullptr;
    std::lock_guard<std::mutex> lk(db->mu);
    TRY(busy(db));
    if (opts && (opts->max_active < 0 || opts->queue_capacity < 0 || opts->chunk_groups < 0 ||
                 opts->memory_budget < 0))
        return fail(SW_EINVAL, "negative server option");
    std::unique_ptr<sw_server> s(new sw_server());
    s->db = db;
    if (opts) s->opts = *opts;
    TRY(server_setup(s.get()));
    db->server_attached = true;
    s->worker = std::thread(server_loop, s.get());
    *out = s.release();
    return SW_OK;
}

int sw_server_submit(sw_server *srv, const uint8_t *query, int32_t qlen, const sw_scoring *sc,
                     int32_t k, uint64_t *ticket) {
    g_err.clear();
    if (!srv || !ticket) return fail(SW_EINVAL, "NULL argument");
    TRY(validate_scoring(srv->db, sc));
    TRY(validate_query(srv->db, query, qlen));
    if (k < 1 || k > SW_MAX_K) return fail(SW_EINVAL, "k not in 1..%d", SW_MAX_K);
    auto r = std::make_shared<Request>();
    r->query.assign(query, query + qlen);
    r->matrix.assign(sc->matrix, sc->matrix + (size_t)sc->alphabet * sc->alphabet);
    r->alpha = sc->alpha;
    r->beta = sc->beta;
    r->k = k;
    // per-request device state: its query profile and its top-k (the score
    // rows are per slot, allocated when the server starts)
    r->bytes = (int64_t)srv->db->R * round_up(qlen, kQPad) + (int64_t)k * 12;
    r->t_submit = now_ms();
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(SW_ESTOPPED, "server stopped");
    if (r->bytes > srv->opts.memory_budget)
        return fail(SW_EINVAL, "request needs %lld bytes, more than the memory budget",
                    (long long)r->bytes);
    if ((int64_t)srv->waiting.size() >= srv->opts.queue_capacity)
        return fail(SW_EBUSY, "request queue full");
    r->ticket = srv->next_ticket++;
    srv->table[r->ticket] = r;
    srv->waiting.push_back(r);
    *ticket = r->ticket;
    srv->cv_work.notify_one();
    return SW_OK;
}

int sw_server_wait(sw_server *srv, uint64_t ticket, int32_t *top_scores, int64_t *top_idx,
                   sw_req_stats *stats) {
    g_err.clear();
    if (!srv || !top_scores || !top_idx) return fail(SW_EINVAL, "NULL argument");
    std::shared_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        auto it = srv->table.find(ticket);
        if (it == srv->table.end())
            return fail(SW_ENOTFOUND, "unknown ticket %llu", (unsigned long long)ticket);
        r = it->second;
        srv->waiters++;
        srv->cv_done.wait(lk, [&] { return r->done; });
        srv->table.erase(ticket);
        srv->waiters--;
        srv->cv_done.notify_all();
    }
    if (r->rc != SW_OK)
        return fail(r->rc, r->rc == SW_ESTOPPED ? "server stopped" : "device failure: %s",
                    srv->fatal.c_str());
    std::memcpy(top_scores, r->top_s.data(), (size_t)r->k * 4);
    std::memcpy(top_idx, r->top_i.data(), (size_t)r->k * 8);
    if (stats) {
        *stats = sw_req_stats{};
        stats->queue_ms = r->t_admit - r->t_submit;
        stats->total_ms = r->t_done - r->t_submit;
        stats->cells = (int64_t)r->query.size() * srv->db->total_res;
        stats->passes = r->passes;
        stats->shared_passes = r->shared;
    }
    return SW_OK;
}

void sw_server_stop(sw_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    {
        // threads blocked in sw_server_wait have been woken with SW_ESTOPPED;
        // let them leave before the server goes away
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv_done.wait(lk, [&] { return srv->waiters == 0; });
    }
    {
        std::lock_guard<std::mutex> lk(srv->db->mu);
        srv->db->server_attached = false;
    }
    delete srv;
}

}  // extern "C"

// ===========================================================================
// Databases larger than device memory (section III's workflow: the database is
// sorted and indexed offline, and loaded chunk by chunk).
//
// sw_index_write sorts the subjects by length, cuts that order into chunks of
// about chunk_residues residues, and writes each chunk already packed (the
// device layout of sw_db_open) with its subjects in ascending database order,
// so a chunk's local index order is the global order.  sw_index_open maps the
// file; a search keeps the whole index on the device when it fits the memory
// budget, and otherwise streams it through two chunk slots, loading chunk c+1
// on a host thread while chunk c is searched.  Per-chunk top-k lists merge by
// (score desc, global index asc), which gives exactly the top-k of the whole
// database because ties inside a chunk already break by ascending index.
// ===========================================================================
namespace {

constexpr char kIndexMagic[8] = {'S', 'W', 'M', 'I', 'I', 'D', 'X', '1'};
constexpr int kIndexVersion = 1;
// Compute units assumed when the writer packs a chunk (MI355X): it decides
// whether a chunk is large enough to use the lane-per-subject kernel.
constexpr int kIndexCUs = 256;

struct IndexHeader {
    char magic[8];
    int32_t version, alphabet;
    int64_t n_seqs, total_res, n_chunks, chunk_residues;
    int64_t reserved[4];
};

struct ChunkEntry {
    int64_t file_off;      // first byte of the chunk's section
    int64_t bytes;         // bytes of the section
    int64_t n_seqs, total_res, device_bytes;
};

// Fixed part of a chunk section; the arrays follow, each starting at a
// multiple of 64 bytes: ids (int32 n), offsets (int64 n+1), residues (uint8),
// long_ids (int32), grp_rows (int32 ng), grp_ids (int32 ng*128),
// grp_res_prefix (int64 ng+1), gbase (int64 ng), codes (uint16).
struct ChunkHead {
    int64_t n_seqs, total_res, max_len, long_res, long_threshold, inter_res, inter_padded_rows;
    int64_t n_codes;
    int32_t n_groups, max_rows, n_long, fixed_cut;
};

int64_t al64(int64_t x) { return (x + 63) / 64 * 64; }

struct ChunkLayout {
    int64_t ids, offsets, residues, long_ids, grp_rows, grp_ids, grp_res_prefix, gbase, codes, end;
};

ChunkLayout chunk_layout(const ChunkHead &h) {
    ChunkLayout L;
    int64_t o = al64(sizeof(ChunkHead));
    L.ids = o;             o = al64(o + h.n_seqs * 4);
    L.offsets = o;         o = al64(o + (h.n_seqs + 1) * 8);
    L.residues = o;        o = al64(o + h.total_res);
    L.long_ids = o;        o = al64(o + (int64_t)h.n_long * 4);
    L.grp_rows = o;        o = al64(o + (int64_t)h.n_groups * 4);
    L.grp_ids = o;         o = al64(o + (int64_t)h.n_groups * kGroup * 4);
    L.grp_res_prefix = o;  o = al64(o + ((int64_t)h.n_groups + 1) * 8);
    L.gbase = o;           o = al64(o + (int64_t)h.n_groups * 8);
    L.codes = o;           o = al64(o + h.n_codes * 2);
    L.end = o;
    return L;
}

int write_all(FILE *f, const void *p, size_t n, int64_t at) {
    if (fseeko(f, (off_t)at, SEEK_SET) != 0) return fail(SW_EINVAL, "index: seek failed");
    if (n && fwrite(p, 1, n, f) != n) return fail(SW_ENOMEM, "index: write failed (disk full?)");
    return SW_OK;
}

}  // namespace

struct sw_index {
    int device = 0;
    int fd = -1;
    const uint8_t *map = nullptr;
    size_t map_bytes = 0;
    IndexHeader hdr{};
    std::vector<ChunkEntry> chunks;
    bool resident = false;
    int64_t budget = 0;
    // resident: one handle per chunk; streaming: two slots
    std::vector<std::unique_ptr<sw_db>> dbs;
    std::vector<int> slot_chunk;   // chunk held by each handle (-1 = none)
    std::mutex mu;
    sw_index_stats last{};
};

namespace {

PackedView chunk_view(const sw_index *ix, int64_t c, const int32_t **ids) {
    const uint8_t *base = ix->map + ix->chunks[c].file_off;
    ChunkHead h;
    std::memcpy(&h, base, sizeof h);
    const ChunkLayout L = chunk_layout(h);
    PackedView v;
    v.n_seqs = h.n_seqs;
    v.total_res = h.total_res;
    v.max_len = h.max_len;
    v.long_res = h.long_res;
    v.long_threshold = h.long_threshold;
    v.inter_res = h.inter_res;
    v.inter_padded_rows = h.inter_padded_rows;
    v.n_groups = h.n_groups;
    v.max_rows = h.max_rows;
    v.n_long = h.n_long;
    v.fixed_cut = h.fixed_cut != 0;
    v.n_codes = h.n_codes;
    v.residues = base + L.residues;
    v.offsets = (const int64_t *)(base + L.offsets);
    v.long_ids = (const int32_t *)(base + L.long_ids);
    v.grp_rows = (const int32_t *)(base + L.grp_rows);
    v.grp_ids = (const int32_t *)(base + L.grp_ids);
    v.grp_res_prefix = (const int64_t *)(base + L.grp_res_prefix);
    v.gbase = (const int64_t *)(base + L.gbase);
    v.codes = (const uint16_t *)(base + L.codes);
    if (ids) *ids = (const int32_t *)(base + L.ids);
    return v;
}

// Load chunk c into handle slot `h` (no-op if it is there already).
int load_chunk(sw_index *ix, int h, int64_t c, double *ms, int64_t *bytes) {
    if (ix->slot_chunk[h] == c) return SW_OK;
    const double t0 = now_ms();
    ix->slot_chunk[h] = -1;
    sw_db *db = ix->dbs[h].get();
    const PackedView v = chunk_view(ix, c, nullptr);
    TRY(db_install(db, v, db->aux));
    ix->slot_chunk[h] = (int)c;
    if (ms) *ms += now_ms() - t0;
    if (bytes) *bytes += view_device_bytes(v);
    return SW_OK;
}

}  // namespace

extern "C" {

int sw_index_write(const char *path, const uint8_t *residues, const int64_t *offsets,
                   int64_t n_seqs, int32_t alphabet, int64_t chunk_residues) {
    g_err.clear();
    if (!path) return fail(SW_EINVAL, "path is NULL");
    if (chunk_residues < 1) return fail(SW_EINVAL, "chunk_residues < 1");
    TRY(validate_db(residues, offsets, n_seqs, alphabet));
    std::vector<int64_t> len(n_seqs);
    for (int64_t i = 0; i < n_seqs; ++i) len[i] = offsets[i + 1] - offsets[i];
    std::vector<int32_t> order(n_seqs);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return len[x] < len[y]; });
    // Chunk assignment.  Consecutive runs of the length order would leave the
    // last chunks with only long subjects, too few to fill the chip lane-per-
    // subject, so those chunks would run entirely on the wave-per-pair kernel.
    // Instead, when subjects are short next to a chunk, the length order is
    // dealt round-robin over nc chunks: every chunk then holds the whole length
    // distribution.  Dealt this way a chunk exceeds the mean by at most two of
    // the longest subjects, so nc = ceil(total / (chunk_residues - 2 max_len))
    // keeps each within chunk_residues.  Otherwise (a single chunk, or
    // subjects longer than a quarter of a chunk) the length order is cut into
    // consecutive runs (at least one subject per chunk).
    int64_t max_len = 0;
    for (int64_t i = 0; i < n_seqs; ++i) max_len = std::max(max_len, len[i]);
    const int64_t total = offsets[n_seqs];
    const int64_t room = chunk_residues - 2 * max_len;
    std::vector<std::vector<int32_t>> members;
    int64_t layout = 0;
    if (total > chunk_residues && 4 * max_len <= chunk_residues && room > 0) {
        const int64_t nc = (total + room - 1) / room;
        members.assign((size_t)nc, {});
        for (int64_t r = 0; r < n_seqs; ++r) members[(size_t)(r % nc)].push_back(order[r]);
        layout = 1;
    } else {
        int64_t acc = 0;
        for (int64_t i = 0; i < n_seqs; ++i) {
            if (members.empty() || (acc > 0 && acc + len[order[i]] > chunk_residues)) {
                members.push_back({});
                acc = 0;
            }
            members.back().push_back(order[i]);
            acc += len[order[i]];
        }
    }
    const int64_t n_chunks = (int64_t)members.size();

    FILE *f = fopen(path, "wb");
    if (!f) return fail(SW_EINVAL, "index: cannot create %s", path);
    std::unique_ptr<FILE, int (*)(FILE *)> guard(f, fclose);
    IndexHeader hdr{};
    std::memcpy(hdr.magic, kIndexMagic, 8);
    hdr.version = kIndexVersion;
    hdr.alphabet = alphabet;
    hdr.n_seqs = n_seqs;
    hdr.total_res = offsets[n_seqs];
    hdr.n_chunks = n_chunks;
    hdr.chunk_residues = chunk_residues;
    hdr.reserved[0] = layout;   // 0: consecutive runs of the length order, 1: dealt round-robin
    std::vector<ChunkEntry> table((size_t)n_chunks);
    int64_t pos = al64((int64_t)sizeof hdr + n_chunks * (int64_t)sizeof(ChunkEntry));
    for (int64_t c = 0; c < n_chunks; ++c) {
        // the chunk's subjects in ascending database order
        std::vector<int32_t> ids = std::move(members[(size_t)c]);
        std::sort(ids.begin(), ids.end());
        const int64_t n = (int64_t)ids.size();
        std::vector<int64_t> loff(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) loff[i + 1] = loff[i] + len[ids[i]];
        std::vector<uint8_t> lres((size_t)loff[n]);
        for (int64_t i = 0; i < n; ++i)
            std::memcpy(lres.data() + loff[i], residues + offsets[ids[i]], (size_t)len[ids[i]]);
        Packed pk;
        TRY(pack_db(lres.data(), loff.data(), n, alphabet, 0, kIndexCUs, pk));
        ChunkHead h{};
        h.n_seqs = n;
        h.total_res = loff[n];
        h.max_len = pk.max_len;
        h.long_res = pk.long_res;
        h.long_threshold = pk.long_threshold;
        h.inter_res = pk.inter_res;
        h.inter_padded_rows = pk.inter_padded_rows;
        h.n_codes = (int64_t)pk.codes.size();
        h.n_groups = pk.n_groups;
        h.max_rows = pk.max_rows;
        h.n_long = (int32_t)pk.long_ids.size();
        h.fixed_cut = pk.fixed_cut ? 1 : 0;
        const ChunkLayout L = chunk_layout(h);
        TRY(write_all(f, &h, sizeof h, pos));
        TRY(write_all(f, ids.data(), (size_t)n * 4, pos + L.ids));
        TRY(write_all(f, loff.data(), (size_t)(n + 1) * 8, pos + L.offsets));
        TRY(write_all(f, lres.data(), lres.size(), pos + L.residues));
        TRY(write_all(f, pk.long_ids.data(), pk.long_ids.size() * 4, pos + L.long_ids));
        TRY(write_all(f, pk.grp_rows.data(), pk.grp_rows.size() * 4, pos + L.grp_rows));
        TRY(write_all(f, pk.grp_ids.data(), pk.grp_ids.size() * 4, pos + L.grp_ids));
        TRY(write_all(f, pk.grp_res_prefix.data(), pk.grp_res_prefix.size() * 8, pos + L.grp_res_prefix));
        TRY(write_all(f, pk.gbase.data(), pk.gbase.size() * 8, pos + L.gbase));
        TRY(write_all(f, pk.codes.data(), pk.codes.size() * 2, pos + L.codes));
        table[c].file_off = pos;
        table[c].bytes = L.end;
        table[c].n_seqs = n;
        table[c].total_res = loff[n];
        table[c].device_bytes = view_device_bytes(view_of(pk, lres.data(), loff.data()));
        pos += L.end;
    }
    TRY(write_all(f, &hdr, sizeof hdr, 0));
    TRY(write_all(f, table.data(), table.size() * sizeof(ChunkEntry), sizeof hdr));
    // the file ends at the last section's end (zero bytes of padding included)
    if (ftruncate(fileno(f), (off_t)pos) != 0) return fail(SW_ENOMEM, "index: cannot size %s", path);
    if (fflush(f) != 0) return fail(SW_ENOMEM, "index: write failed (disk full?)");
    return SW_OK;
}

int sw_index_open(const char *path, const sw_index_opts *opts, sw_index **out) {
    g_err.clear();
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = nullptr;
    if (!path) return fail(SW_EINVAL, "path is NULL");
    std::unique_ptr<sw_index> ix(new sw_index());
    ix->device = opts && opts->device > 0 ? opts->device : 0;
    ix->fd = open(path, O_RDONLY);
    if (ix->fd < 0) return fail(SW_EINVAL, "index: cannot open %s", path);
    struct stat sb;
    if (fstat(ix->fd, &sb) != 0 || sb.st_size < (off_t)sizeof(IndexHeader)) {
        close(ix->fd);
        return fail(SW_EINVAL, "index: %s is too short", path);
    }
    ix->map_bytes = (size_t)sb.st_size;
    void *m = mmap(nullptr, ix->map_bytes, PROT_READ, MAP_SHARED, ix->fd, 0);
    if (m == MAP_FAILED) {
        close(ix->fd);
        return fail(SW_ENOMEM, "index: cannot map %s", path);
    }
    ix->map = (const uint8_t *)m;
    auto bad = [&](const char *what) {
        munmap((void *)ix->map, ix->map_bytes);
        close(ix->fd);
        return fail(SW_EINVAL, "index: %s: %s", path, what);
    };
    std::memcpy(&ix->hdr, ix->map, sizeof ix->hdr);
    const IndexHeader &h = ix->hdr;
    if (std::memcmp(h.magic, kIndexMagic, 8) != 0) return bad("not an index file");
    if (h.version != kIndexVersion) return bad("unknown version");
    if (h.alphabet < 1 || h.alphabet > SW_MAX_ALPHABET || h.n_seqs < 0 || h.n_chunks < 0 ||
        (int64_t)sizeof h + h.n_chunks * (int64_t)sizeof(ChunkEntry) > (int64_t)ix->map_bytes)
        return bad("corrupt header");
    ix->chunks.resize((size_t)h.n_chunks);
    std::memcpy(ix->chunks.data(), ix->map + sizeof h, ix->chunks.size() * sizeof(ChunkEntry));
    int64_t total_dev = 0, max_dev = 0, n_sum = 0;
    for (const ChunkEntry &c : ix->chunks) {
        if (c.file_off < 0 || c.bytes < (int64_t)sizeof(ChunkHead) ||
            c.file_off + c.bytes > (int64_t)ix->map_bytes)
            return bad("chunk outside the file");
        ChunkHead ch;
        std::memcpy(&ch, ix->map + c.file_off, sizeof ch);
        if (ch.n_seqs != c.n_seqs || chunk_layout(ch).end != c.bytes) return bad("corrupt chunk");
        total_dev += c.device_bytes;
        max_dev = std::max(max_dev, c.device_bytes);
        n_sum += c.n_seqs;
    }
    if (n_sum != h.n_seqs) return bad("chunks do not cover the database");
    madvise((void *)ix->map, ix->map_bytes, MADV_SEQUENTIAL);
    int64_t budget = opts ? opts->memory_budget : 0;
    if (budget <= 0) {
        size_t fr = 0, tot = 0;
        HIPX(hipSetDevice(ix->device));
        HIPX(hipMemGetInfo(&fr, &tot));
        budget = (int64_t)(fr / 2);
    }
    ix->budget = budget;
    ix->resident = total_dev <= budget || h.n_chunks <= 1;
    if (!ix->resident && 2 * max_dev > budget) {
        munmap((void *)ix->map, ix->map_bytes);
        close(ix->fd);
        return fail(SW_ENOMEM, "index: a memory budget of %lld bytes cannot hold two chunks of up to "
                    "%lld bytes; write the index with smaller chunks", (long long)budget,
                    (long long)max_dev);
    }
    const int64_t handles = ix->resident ? h.n_chunks : 2;
    for (int64_t x = 0; x < handles; ++x) {
        std::unique_ptr<sw_db> db;
        TRY(db_create(ix->device, h.alphabet, db));
        ix->dbs.push_back(std::move(db));
        ix->slot_chunk.push_back(-1);
    }
    if (ix->resident)
        for (int64_t c = 0; c < h.n_chunks; ++c) TRY(load_chunk(ix.get(), (int)c, c, nullptr, nullptr));
    *out = ix.release();
    return SW_OK;
}

void sw_index_close(sw_index *ix) {
    if (!ix) return;
    for (auto &db : ix->dbs) sw_db_close(db.release());
    if (ix->map) munmap((void *)ix->map, ix->map_bytes);
    if (ix->fd >= 0) close(ix->fd);
    delete ix;
}

int64_t sw_index_size(const sw_index *ix) { return ix ? ix->hdr.n_seqs : -1; }

int sw_index_last_stats(sw_index *ix, sw_index_stats *out) {
    g_err.clear();
    if (!ix || !out) return fail(SW_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(ix->mu);
    *out = ix->last;
    return SW_OK;
}

int sw_index_search_batch(sw_index *ix, int32_t nq, const uint8_t *q_res, const int64_t *q_off,
                          const sw_scoring *sc, int32_t k, int32_t *top_scores, int64_t *top_idx,
                          int32_t *all_scores) {
    g_err.clear();
    if (!ix) return fail(SW_EINVAL, "index is NULL");
    if (k < 1 || k > SW_MAX_K) return fail(SW_EINVAL, "k not in 1..%d", SW_MAX_K);
    if (!top_scores || !top_idx) return fail(SW_EINVAL, "top-k outputs are NULL");
    if (nq < 1) return fail(SW_EINVAL, "nq < 1");
    if (!q_res || !q_off) return fail(SW_EINVAL, "queries are NULL");
    std::lock_guard<std::mutex> lk(ix->mu);
    const double t_start = now_ms();
    const int64_t N = ix->hdr.n_seqs;
    if ((int64_t)nq * N > ((int64_t)1 << 40)) return fail(SW_EINVAL, "batch too large");
    // running top-k per query: (score, global index), -1 fill
    std::vector<int32_t> best_s((size_t)nq * k, -1);
    std::vector<int64_t> best_i((size_t)nq * k, -1);
    sw_index_stats st{};
    st.chunks = (int64_t)ix->chunks.size();
    st.resident = ix->resident ? 1 : 0;
    if (ix->chunks.empty()) {
        if (nq > 0) {
            std::copy(best_s.begin(), best_s.end(), top_scores);
            std::copy(best_i.begin(), best_i.end(), top_idx);
        }
        ix->last = st;
        return SW_OK;
    }
    std::vector<int32_t> cs((size_t)nq * k), chunk_scores;
    std::vector<int64_t> ci((size_t)nq * k);
    std::vector<std::pair<int32_t, int64_t>> cand;
    const int64_t nc = (int64_t)ix->chunks.size();
    // streaming: chunk c in slot c % 2, chunk 0 loaded before the loop
    if (!ix->resident) TRY(load_chunk(ix, 0, 0, &st.load_ms, &st.bytes_loaded));
    for (int64_t c = 0; c < nc; ++c) {
        const int h = ix->resident ? (int)c : (int)(c % 2);
        std::thread loader;
        int load_rc = SW_OK;
        std::string load_err;
        double load_ms = 0;
        int64_t load_bytes = 0;
        if (!ix->resident && c + 1 < nc) {
            loader = std::thread([&, c] {
                load_rc = load_chunk(ix, (int)((c + 1) % 2), c + 1, &load_ms, &load_bytes);
                if (load_rc != SW_OK) load_err = g_err;
            });
        }
        const int32_t *ids = nullptr;
        const PackedView v = chunk_view(ix, c, &ids);
        sw_db *db = ix->dbs[h].get();
        int rc;
        {
            std::lock_guard<std::mutex> dlk(db->mu);
            if (all_scores) chunk_scores.resize((size_t)nq * std::max<int64_t>(v.n_seqs, 1));
            const double t0 = now_ms();
            rc = run_search(db, nq, q_res, q_off, sc, k, cs.data(), ci.data(),
                            all_scores ? chunk_scores.data() : nullptr, nullptr, nullptr);
            st.search_ms += now_ms() - t0;
            st.kernel_ms += db->last.kernel_ms;
            st.cells += db->last.cells;
        }
        if (loader.joinable()) loader.join();
        if (rc != SW_OK) return rc;
        if (load_rc != SW_OK) return fail(load_rc, "%s", load_err.c_str());
        st.load_ms += load_ms;
        st.bytes_loaded += load_bytes;
        // merge: local index -> global, then (score desc, global index asc)
        for (int32_t q = 0; q < nq; ++q) {
            cand.clear();
            for (int32_t x = 0; x < k; ++x) {
                const size_t a = (size_t)q * k + x;
                if (best_i[a] >= 0) cand.push_back({best_s[a], best_i[a]});
                if (ci[a] >= 0) cand.push_back({cs[a], (int64_t)ids[ci[a]]});
            }
            std::sort(cand.begin(), cand.end(), [](const auto &a, const auto &b) {
                return a.first != b.first ? a.first > b.first : a.second < b.second;
            });
            for (int32_t x = 0; x < k; ++x) {
                const size_t a = (size_t)q * k + x;
                best_s[a] = x < (int32_t)cand.size() ? cand[x].first : -1;
                best_i[a] = x < (int32_t)cand.size() ? cand[x].second : -1;
            }
            if (all_scores)
                for (int64_t i = 0; i < v.n_seqs; ++i)
                    all_scores[(size_t)q * N + ids[i]] = chunk_scores[(size_t)q * v.n_seqs + i];
        }
    }
    std::copy(best_s.begin(), best_s.end(), top_scores);
    std::copy(best_i.begin(), best_i.end(), top_idx);
    st.total_ms = now_ms() - t_start;
    ix->last = st;
    return SW_OK;
}

}  // extern "C"
