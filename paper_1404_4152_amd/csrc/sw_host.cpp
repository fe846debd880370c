// Host side of libswmi: the C ABI declared in include/swmi.h.
//
// Database open (section III, stage ii and the offline index): subjects are
// stable-sorted by ascending length.  Short subjects are dealt into groups of
// 128 (64 lanes x 2 packed halves) laid out interleaved for coalesced wave
// loads, padded with a residue code that scores 0 (section III.B.1).  The
// longest subjects, which would hold one lane for too long, form a long list
// served by the wave-per-pair kernel, as does any database too small to fill
// the GPU lane-per-subject.
//
// Search (stages i and iv): build the query profile (section III.B.2; row r
// holds the scores of the whole query against residue r), run the kernels,
// recompute flagged narrow-tier pairs exactly, then sort or select the scores.
#include <hip/hip_runtime.h>

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

using namespace swmi;

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

double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Grow-only device buffer.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
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

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct Plan {
    int tier = TIER_F16X2;
    int strip = 32;
    int waves = 4;
    int thr = kThrF16;
};

}  // namespace

struct sw_db {
    int device = 0;
    hipStream_t stream = nullptr;
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
    // long list (caller ids), longest first
    std::vector<int32_t> long_ids;
    int64_t long_res = 0;
    int64_t long_threshold = 0;
    // device copies
    DevBuf d_res, d_off, d_codes, d_grp_base, d_grp_rows, d_grp_ids, d_long_ids;
    // per-call workspaces
    DevBuf w_qp, w_qmeta, w_scores, w_items, w_counters, w_ovf, w_scr_inter, w_scr_intra,
        w_topk, w_top;
    HostBuf h_stage;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::mutex mu;
    sw_search_opts opts{};
    sw_stats last{};
    // autotuner table: query-length bucket -> plan
    std::map<int, Plan> tuned;
    int cus = 256;
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
    if (qlen < 1 || qlen > SW_MAX_LEN) return fail(SW_EINVAL, "query length %lld not in 1..2^24", (long long)qlen);
    if (!q) return fail(SW_EINVAL, "query is NULL");
    for (int64_t j = 0; j < qlen; ++j)
        if (q[j] >= db->alphabet)
            return fail(SW_EINVAL, "query code %d at %lld >= alphabet %d", q[j], (long long)j, db->alphabet);
    return SW_OK;
}

Plan plan_for(const sw_db *db, int64_t max_qlen) {
    Plan p;
    // Autotuned entry for this query-length bucket, if any.
    if (!db->tuned.empty()) {
        int bucket = 0;
        while ((64LL << bucket) < max_qlen && bucket < 20) ++bucket;
        auto it = db->tuned.find(bucket);
        if (it != db->tuned.end()) p = it->second;
    }
    if (db->opts.tier) p.tier = db->opts.tier;
    if (db->opts.strip) p.strip = db->opts.strip;
    if (db->opts.waves) p.waves = db->opts.waves;
    if (p.strip == 64) p.waves = 4;
    if (p.waves == 6 && p.strip != 32) p.waves = 4;
    // The pair profile must fit in LDS.
    while (p.strip > 16 && inter_lds_bytes(db->R, p.strip) > 150 * 1024) p.strip /= 2;
    p.thr = p.tier == TIER_I16X2 ? kThrI16 : kThrF16;
    if (db->opts.sat_threshold > 0 && db->opts.sat_threshold < p.thr) p.thr = db->opts.sat_threshold;
    return p;
}

int intra_T_for(int64_t max_qlen) {
    if (max_qlen <= 256) return 4;
    if (max_qlen <= 512) return 8;
    return 16;
}

struct Batch {
    int32_t nq = 0;
    std::vector<int64_t> qlen;
    std::vector<int32_t> mpad;
    std::vector<int64_t> qp_off;
    int64_t qp_bytes = 0;
    int64_t max_qlen = 0;
    int64_t sum_qlen = 0;
};

// The whole search path for nq queries.  Outputs (any may be null):
//   scores_host: nq * n_seqs; scores_dev: device pointer (nq * n_seqs);
//   top_s/top_i: nq * k when k > 0.
int run_search(sw_db *db, int32_t nq, const uint8_t *q_res, const int64_t *q_off,
               const sw_scoring *sc, int32_t k, int32_t *top_s, int64_t *top_i,
               int32_t *scores_host, int32_t *scores_dev, hipStream_t user_stream) {
    const double t_start = now_ms();
    if (int rc = validate_scoring(db, sc)) return rc;
    if (nq < 1) return fail(SW_EINVAL, "nq < 1");
    if (!q_res || !q_off) return fail(SW_EINVAL, "queries are NULL");
    if (k < 0 || k > SW_MAX_K) return fail(SW_EINVAL, "k not in 1..%d", SW_MAX_K);
    Batch b;
    b.nq = nq;
    for (int32_t q = 0; q < nq; ++q) {
        const int64_t L = q_off[q + 1] - q_off[q];
        if (int rc = validate_query(db, q_res + q_off[q], L)) return rc;
        b.qlen.push_back(L);
        b.mpad.push_back((int32_t)round_up(L, kQPad));
        b.qp_off.push_back(b.qp_bytes);
        b.qp_bytes += (int64_t)db->R * b.mpad.back();
        b.max_qlen = std::max(b.max_qlen, L);
        b.sum_qlen += L;
    }
    HIPX(hipSetDevice(db->device));
    hipStream_t st = user_stream ? user_stream : db->stream;
    const Plan plan = plan_for(db, b.max_qlen);
    const int R = db->R, A = db->alphabet;
    const int64_t n = db->n_seqs;

    // ---- work lists (host) ----
    const int W = plan.waves;
    const int nblk = (db->n_groups + W - 1) / W;
    std::vector<std::pair<int64_t, int64_t>> inter_items;   // (cost, q * nblk + blk)
    inter_items.reserve((size_t)nq * nblk);
    for (int32_t q = 0; q < nq; ++q) {
        const int64_t strips = b.mpad[q] / plan.strip;
        for (int bk = 0; bk < nblk; ++bk) {
            const int last = std::min(db->n_groups, (bk + 1) * W) - 1;
            inter_items.push_back({(int64_t)db->grp_rows[last] * strips, (int64_t)q * nblk + bk});
        }
    }
    std::stable_sort(inter_items.begin(), inter_items.end(),
                     [](const auto &x, const auto &y) { return x.first > y.first; });
    const int WI = 4;   // waves per workgroup of the wave-per-pair kernel
    const int64_t nlong = (int64_t)db->long_ids.size();
    const int64_t nlblk = (nlong + WI - 1) / WI;
    std::vector<std::pair<int64_t, int64_t>> intra_items;
    for (int32_t q = 0; q < nq; ++q)
        for (int64_t bk = 0; bk < nlblk; ++bk)
            intra_items.push_back({db->len[db->long_ids[bk * WI]] * b.qlen[q], (int64_t)q * nlblk + bk});
    std::stable_sort(intra_items.begin(), intra_items.end(),
                     [](const auto &x, const auto &y) { return x.first > y.first; });
    const int64_t n_inter = (int64_t)inter_items.size(), n_intra = (int64_t)intra_items.size();
    if (n_inter > INT32_MAX || n_intra > INT32_MAX || (int64_t)nq * n > ((int64_t)1 << 40))
        return fail(SW_EINVAL, "batch too large");

    // ---- host staging: profiles, query meta, items ----
    const size_t sz_qp = (size_t)round_up(b.qp_bytes, 256);
    const size_t sz_meta = (size_t)round_up((size_t)nq * (8 + 4 + 4), 256);
    const size_t sz_items = (size_t)round_up((n_inter * 2 + n_intra * (1 + WI)) * 4, 256);
    if (int rc = db->h_stage.reserve(sz_qp + sz_meta + sz_items)) return rc;
    // The staging buffer may still feed copies of a previous call on another stream.
    HIPX(hipStreamSynchronize(st));
    uint8_t *hs = db->h_stage.as<uint8_t>();
    int8_t *qp = (int8_t *)hs;
    for (int32_t q = 0; q < nq; ++q) {
        const uint8_t *qq = q_res + q_off[q];
        const int mp = b.mpad[q];
        int8_t *base = qp + b.qp_off[q];
        for (int r = 0; r < R; ++r) {
            int8_t *row = base + (int64_t)r * mp;
            if (r < A)
                for (int64_t j = 0; j < b.qlen[q]; ++j) row[j] = sc->matrix[qq[j] * A + r];
            else
                std::memset(row, 0, (size_t)b.qlen[q]);
            std::memset(row + b.qlen[q], 0, (size_t)(mp - b.qlen[q]));
        }
    }
    int64_t *m_off = (int64_t *)(hs + sz_qp);
    int32_t *m_mpad = (int32_t *)(m_off + nq);
    int32_t *m_qlen = m_mpad + nq;
    for (int32_t q = 0; q < nq; ++q) {
        m_off[q] = b.qp_off[q];
        m_mpad[q] = b.mpad[q];
        m_qlen[q] = (int32_t)b.qlen[q];
    }
    int32_t *it_q = (int32_t *)(hs + sz_qp + sz_meta);
    int32_t *it_g = it_q + n_inter;
    int32_t *il_q = it_g + n_inter;
    int32_t *il_ids = il_q + n_intra;
    for (int64_t i = 0; i < n_inter; ++i) {
        const int64_t key = inter_items[i].second;
        it_q[i] = (int32_t)(key / nblk);
        it_g[i] = (int32_t)((key % nblk) * W);
    }
    for (int64_t i = 0; i < n_intra; ++i) {
        const int64_t key = intra_items[i].second;
        il_q[i] = (int32_t)(key / nlblk);
        const int64_t bk = key % nlblk;
        for (int w = 0; w < WI; ++w) {
            const int64_t x = bk * WI + w;
            il_ids[i * WI + w] = x < nlong ? db->long_ids[x] : -1;
        }
    }

    // ---- device workspaces ----
    if (int rc = db->w_qp.reserve(sz_qp + sz_meta + sz_items)) return rc;
    if (int rc = db->w_scores.reserve((size_t)nq * n * 4 + 4)) return rc;
    if (int rc = db->w_counters.reserve(256)) return rc;
    if (int rc = db->w_ovf.reserve((size_t)nq * n * 8 + 8)) return rc;
    const int grid_inter = (int)std::min<int64_t>(n_inter, inter_max_grid(R, plan.strip, W));
    if (n_inter > 0)
        if (int rc = db->w_scr_inter.reserve((size_t)grid_inter * W * db->max_rows * 512)) return rc;
    const int Ti = intra_T_for(b.max_qlen);
    const int intra_lds = intra_lds_bytes(R, Ti);
    const int intra_per_cu = std::max(1, std::min(160 * 1024 / (intra_lds + 64), 8));
    const int grid_intra_cap = intra_per_cu * db->cus;
    const int64_t max_len_pad = round_up(std::max<int64_t>(db->max_len, 1), 64) + 128;
    const int grid_long = (int)std::min<int64_t>(n_intra, grid_intra_cap);
    const int grid_ovf = std::min(grid_intra_cap * WI, 4096);
    const int64_t intra_slots = std::max<int64_t>((int64_t)grid_long * WI, grid_ovf);
    if (int rc = db->w_scr_intra.reserve((size_t)intra_slots * max_len_pad * 8)) return rc;
    uint8_t *dq = db->w_qp.as<uint8_t>();
    HIPX(hipMemcpyAsync(dq, hs, sz_qp + sz_meta + sz_items, hipMemcpyHostToDevice, st));
    int32_t *ctr = db->w_counters.as<int32_t>();
    int32_t *scores = scores_dev ? scores_dev : db->w_scores.as<int32_t>();
    int32_t *ovf_q = db->w_ovf.as<int32_t>();
    int32_t *ovf_id = ovf_q + (size_t)nq * n;

    QuerySet qs;
    qs.qp = (const int8_t *)dq;
    qs.qp_off = (const int64_t *)(dq + sz_qp);
    qs.mpad = (const int32_t *)(qs.qp_off + nq);
    qs.qlen = qs.mpad + nq;
    const int32_t *d_it = (const int32_t *)(dq + sz_qp + sz_meta);

    HIPX(launch_fill_i32(ctr, 0, 64, st));
    HIPX(hipEventRecord(db->ev[0], st));
    if (n_inter > 0) {
        InterArgs a{};
        a.codes = db->d_codes.as<uint16_t>();
        a.grp_base = db->d_grp_base.as<int64_t>();
        a.grp_rows = db->d_grp_rows.as<int32_t>();
        a.grp_ids = db->d_grp_ids.as<int32_t>();
        a.n_groups = db->n_groups;
        a.item_q = d_it;
        a.item_g = d_it + n_inter;
        a.n_items = (int32_t)n_inter;
        a.counter = ctr + 0;
        a.qs = qs;
        a.R = R;
        const int cap = plan.tier == TIER_I16X2 ? 32767 : 2048;
        a.alpha = std::min(sc->alpha, cap);
        a.beta = std::min(sc->beta, cap);
        a.thr = plan.thr;
        a.scratch = db->w_scr_inter.as<uint32_t>();
        a.max_rows = db->max_rows;
        a.scores = scores;
        a.n_seqs = n;
        a.ovf_q = ovf_q;
        a.ovf_id = ovf_id;
        a.ovf_count = ctr + 1;
        a.ovf_cap = (int64_t)nq * n;
        HIPX(launch_inter(a, plan.tier, plan.strip, W, grid_inter, st));
    }
    HIPX(hipEventRecord(db->ev[1], st));
    IntraArgs ia{};
    ia.res = db->d_res.as<uint8_t>();
    ia.off = db->d_off.as<int64_t>();
    ia.qs = qs;
    ia.R = R;
    ia.alpha = sc->alpha;
    ia.beta = sc->beta;
    ia.pass_scratch = db->w_scr_intra.as<int32_t>();
    ia.max_len_pad = max_len_pad;
    ia.scores = scores;
    ia.n_seqs = n;
    if (n_intra > 0) {
        IntraArgs la = ia;
        la.item_q = d_it + 2 * n_inter;
        la.item_ids = la.item_q + n_intra;
        la.n_items = (int32_t)n_intra;
        la.counter = ctr + 2;
        HIPX(launch_intra(la, Ti, WI, grid_long, st));
    }
    if (n_inter > 0) {
        IntraArgs oa = ia;
        oa.item_q = ovf_q;
        oa.item_ids = ovf_id;
        oa.n_items_dev = ctr + 1;
        oa.counter = ctr + 3;
        HIPX(launch_intra(oa, 16, 1, grid_ovf, st));
    }
    HIPX(hipEventRecord(db->ev[2], st));

    if (k > 0) {
        const size_t tk = (size_t)nq * (256 * 4 + 4 * 4 + kTopkBlocks * 4 + (size_t)k * 8);
        if (int rc = db->w_topk.reserve(tk)) return rc;
        if (int rc = db->w_top.reserve((size_t)nq * k * 12)) return rc;
        TopkWork tw;
        tw.hist = db->w_topk.as<uint32_t>();
        tw.state = (int32_t *)(tw.hist + (size_t)nq * 256);
        tw.eqcnt = tw.state + (size_t)nq * 4;
        tw.cand_s = tw.eqcnt + (size_t)nq * kTopkBlocks;
        tw.cand_i = tw.cand_s + (size_t)nq * k;
        int64_t *d_ti = db->w_top.as<int64_t>();
        int32_t *d_ts = (int32_t *)(d_ti + (size_t)nq * k);
        HIPX(launch_topk(scores, n, nq, k, tw, d_ts, d_ti, st));
        HIPX(hipMemcpyAsync(top_s, d_ts, (size_t)nq * k * 4, hipMemcpyDeviceToHost, st));
        HIPX(hipMemcpyAsync(top_i, d_ti, (size_t)nq * k * 8, hipMemcpyDeviceToHost, st));
    }
    HIPX(hipEventRecord(db->ev[3], st));
    if (scores_host && n > 0)
        HIPX(hipMemcpyAsync(scores_host, scores, (size_t)nq * n * 4, hipMemcpyDeviceToHost, st));
    int32_t ctr_h[4] = {0, 0, 0, 0};
    HIPX(hipMemcpyAsync(ctr_h, ctr, 16, hipMemcpyDeviceToHost, st));
    if (!(scores_dev && user_stream)) HIPX(hipStreamSynchronize(st));
    else HIPX(hipStreamSynchronize(st));

    float ms_k = 0, ms_i = 0;
    HIPX(hipEventElapsedTime(&ms_k, db->ev[0], db->ev[2]));
    HIPX(hipEventElapsedTime(&ms_i, db->ev[0], db->ev[1]));
    sw_stats &s = db->last;
    s = sw_stats{};
    s.cells = b.sum_qlen * db->total_res;
    int64_t padded = 0;
    for (int32_t q = 0; q < nq; ++q)
        padded += (int64_t)b.mpad[q] * db->inter_padded_rows +
                  round_up(b.qlen[q], 64LL * Ti) * db->long_res;
    s.padded_cells = padded;
    s.inter_cells = b.sum_qlen * db->inter_res;
    s.recomputed_pairs = ctr_h[1];
    s.intra_pairs = (int64_t)nlong * nq;
    s.kernel_ms = ms_k;
    s.inter_ms = ms_i;
    s.total_ms = now_ms() - t_start;
    s.tier = plan.tier;
    s.strip = plan.strip;
    s.waves = plan.waves;
    return SW_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *sw_last_error(void) { return g_err.c_str(); }

const char *sw_version(void) { return "swmi 0.1 (gfx950)"; }

int sw_db_open(const uint8_t *residues, const int64_t *offsets, int64_t n_seqs, int32_t alphabet,
               const sw_db_opts *opts, sw_db **out) {
    g_err.clear();
    if (!out) return fail(SW_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_seqs < 0) return fail(SW_EINVAL, "n_seqs < 0");
    if (alphabet < 1 || alphabet > SW_MAX_ALPHABET)
        return fail(SW_EINVAL, "alphabet %d not in 1..%d", alphabet, SW_MAX_ALPHABET);
    if (!offsets) return fail(SW_EINVAL, "offsets is NULL");
    if (offsets[0] != 0) return fail(SW_EINVAL, "offsets[0] != 0");
    int64_t max_len = 0;
    for (int64_t i = 0; i < n_seqs; ++i) {
        const int64_t L = offsets[i + 1] - offsets[i];
        if (L < 0) return fail(SW_EINVAL, "offsets decrease at %lld", (long long)i);
        if (L > SW_MAX_LEN) return fail(SW_EINVAL, "sequence %lld longer than 2^24", (long long)i);
        max_len = std::max(max_len, L);
    }
    const int64_t total = offsets[n_seqs];
    if (total > 0 && !residues) return fail(SW_EINVAL, "residues is NULL");
    {
        // Code check, split over threads for big databases.
        const int nth = (int)std::max<int64_t>(1, std::min<int64_t>(16, total >> 24));
        std::vector<int64_t> bad(nth, -1);
        std::vector<std::thread> th;
        for (int t = 0; t < nth; ++t)
            th.emplace_back([&, t] {
                const int64_t lo = total * t / nth, hi = total * (t + 1) / nth;
                for (int64_t i = lo; i < hi; ++i)
                    if (residues[i] >= alphabet) { bad[t] = i; return; }
            });
        for (auto &x : th) x.join();
        for (int t = 0; t < nth; ++t)
            if (bad[t] >= 0)
                return fail(SW_EINVAL, "residue code %d at %lld >= alphabet %d", residues[bad[t]],
                            (long long)bad[t], alphabet);
    }
    if (n_seqs > INT32_MAX - 1) return fail(SW_EINVAL, "too many sequences");

    std::unique_ptr<sw_db> db(new sw_db());
    db->device = opts && opts->device > 0 ? opts->device : 0;
    db->n_seqs = n_seqs;
    db->alphabet = alphabet;
    db->R = alphabet + 1;
    db->total_res = total;
    db->max_len = max_len;
    const int R = db->R;
    // Check the multiply-shift division used for pair codes.
    {
        const int magic = (65536 + R - 1) / R;
        for (int a = 0; a < R * R; ++a)
            if (((a * magic) >> 16) != a / R) return fail(SW_EINVAL, "internal: division check failed");
    }
    HIPX(hipSetDevice(db->device));
    {
        hipDeviceProp_t p;
        HIPX(hipGetDeviceProperties(&p, db->device));
        db->cus = p.multiProcessorCount;
    }
    HIPX(hipStreamCreateWithFlags(&db->stream, hipStreamNonBlocking));
    for (auto &e : db->ev) HIPX(hipEventCreate(&e));

    db->len.resize(n_seqs);
    for (int64_t i = 0; i < n_seqs; ++i) db->len[i] = offsets[i + 1] - offsets[i];
    std::vector<int32_t> order(n_seqs);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return db->len[x] < db->len[y]; });

    // ---- split: lane-per-subject groups vs the long list ----
    const int64_t simds = 4LL * db->cus;
    int64_t cut;   // subjects longer than cut go to the long list
    const int32_t lt = opts ? opts->long_threshold : 0;
    if (lt == -1) cut = INT64_MAX;
    else if (lt == 1) cut = -1;
    else if (lt > 1) cut = lt;
    else {
        // Too few subjects to give every SIMD a wavefront: all wave-per-pair.
        if (n_seqs < simds * kGroup) cut = -1;
        else {
            // Longest lane-per-subject group may hold its SIMD for at most half the
            // average per-SIMD share of rows.
            const double share = (double)total / kGroup / simds;
            cut = std::max<int64_t>(1024, (int64_t)(0.5 * share));
        }
    }
    int64_t n_short = 0;
    while (n_short < n_seqs && db->len[order[n_short]] <= cut) ++n_short;
    db->long_threshold = cut;
    for (int64_t i = n_seqs - 1; i >= n_short; --i) {
        db->long_ids.push_back(order[i]);
        db->long_res += db->len[order[i]];
    }

    // ---- groups of 128 (lane l: lo = 128g + l, hi = 128g + 64 + l) ----
    const int32_t ng = (int32_t)((n_short + kGroup - 1) / kGroup);
    db->n_groups = ng;
    std::vector<int64_t> gbase(ng);
    std::vector<int32_t> gids((size_t)ng * kGroup, -1);
    db->grp_rows.resize(ng);
    int64_t codes_total = 0;
    for (int32_t g = 0; g < ng; ++g) {
        const int64_t last = std::min<int64_t>(n_short, (int64_t)(g + 1) * kGroup) - 1;
        const int64_t rows = std::max<int64_t>(kChunk, round_up(db->len[order[last]], kChunk));
        db->grp_rows[g] = (int32_t)rows;
        gbase[g] = codes_total;
        codes_total += rows * kWave;
        db->max_rows = std::max<int32_t>(db->max_rows, (int32_t)rows);
        db->inter_padded_rows += rows * kGroup;
        for (int x = 0; x < kGroup; ++x) {
            const int64_t si = (int64_t)g * kGroup + x;
            if (si < n_short) {
                gids[(size_t)g * kGroup + x] = order[si];
                db->inter_res += db->len[order[si]];
            }
        }
    }
    std::vector<uint16_t> codes((size_t)codes_total);
    {
        const int nth = (int)std::max(1, std::min(16, ng / 64));
        std::vector<std::thread> th;
        for (int t = 0; t < nth; ++t)
            th.emplace_back([&, t] {
                const uint16_t padc = (uint16_t)(R - 1);
                for (int32_t g = t; g < ng; g += nth) {
                    const int64_t rows = db->grp_rows[g];
                    uint16_t *dst = codes.data() + gbase[g];
                    for (int l = 0; l < kWave; ++l) {
                        const int32_t lo = gids[(size_t)g * kGroup + l];
                        const int32_t hi = gids[(size_t)g * kGroup + kWave + l];
                        const uint8_t *slo = lo >= 0 ? residues + offsets[lo] : nullptr;
                        const uint8_t *shi = hi >= 0 ? residues + offsets[hi] : nullptr;
                        const int64_t nlo = lo >= 0 ? db->len[lo] : 0, nhi = hi >= 0 ? db->len[hi] : 0;
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
    }

    // ---- upload ----
    if (int rc = db->d_res.reserve((size_t)std::max<int64_t>(total, 1))) return rc;
    if (int rc = db->d_off.reserve((size_t)(n_seqs + 1) * 8)) return rc;
    if (total > 0) HIPX(hipMemcpy(db->d_res.p, residues, (size_t)total, hipMemcpyHostToDevice));
    HIPX(hipMemcpy(db->d_off.p, offsets, (size_t)(n_seqs + 1) * 8, hipMemcpyHostToDevice));
    if (ng > 0) {
        if (int rc = db->d_codes.reserve(codes.size() * 2)) return rc;
        if (int rc = db->d_grp_base.reserve((size_t)ng * 8)) return rc;
        if (int rc = db->d_grp_rows.reserve((size_t)ng * 4)) return rc;
        if (int rc = db->d_grp_ids.reserve(gids.size() * 4)) return rc;
        HIPX(hipMemcpy(db->d_codes.p, codes.data(), codes.size() * 2, hipMemcpyHostToDevice));
        HIPX(hipMemcpy(db->d_grp_base.p, gbase.data(), (size_t)ng * 8, hipMemcpyHostToDevice));
        HIPX(hipMemcpy(db->d_grp_rows.p, db->grp_rows.data(), (size_t)ng * 4, hipMemcpyHostToDevice));
        HIPX(hipMemcpy(db->d_grp_ids.p, gids.data(), gids.size() * 4, hipMemcpyHostToDevice));
    }
    *out = db.release();
    return SW_OK;
}

void sw_db_close(sw_db *db) {
    if (!db) return;
    (void)hipSetDevice(db->device);
    if (db->stream) (void)hipStreamSynchronize(db->stream);
    for (auto &e : db->ev)
        if (e) (void)hipEventDestroy(e);
    if (db->stream) (void)hipStreamDestroy(db->stream);
    delete db;
}

int64_t sw_db_size(const sw_db *db) { return db ? db->n_seqs : -1; }

int sw_db_set_opts(sw_db *db, const sw_search_opts *opts) {
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
    db->opts = *opts;
    return SW_OK;
}

int sw_db_last_stats(sw_db *db, sw_stats *out) {
    if (!db || !out) return fail(SW_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(db->mu);
    *out = db->last;
    return SW_OK;
}

int sw_db_search(sw_db *db, const uint8_t *query, int32_t qlen, const sw_scoring *sc,
                 int32_t *scores, void *hip_stream) {
    g_err.clear();
    if (!db) return fail(SW_EINVAL, "db is NULL");
    if (!scores && db->n_seqs > 0) return fail(SW_EINVAL, "scores is NULL");
    std::lock_guard<std::mutex> lk(db->mu);
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
    const int64_t off[2] = {0, qlen};
    return run_search(db, 1, query, off, sc, 0, nullptr, nullptr, nullptr, scores_dev,
                      (hipStream_t)hip_stream);
}

int sw_db_topk(sw_db *db, const uint8_t *query, int32_t qlen, const sw_scoring *sc, int32_t k,
               int32_t *top_scores, int64_t *top_idx, void *hip_stream) {
    g_err.clear();
    if (!db) return fail(SW_EINVAL, "db is NULL");
    if (k < 1 || k > SW_MAX_K) return fail(SW_EINVAL, "k not in 1..%d", SW_MAX_K);
    if (!top_scores || !top_idx) return fail(SW_EINVAL, "top-k outputs are NULL");
    std::lock_guard<std::mutex> lk(db->mu);
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
    return run_search(db, nq, q_res, q_off, sc, k, top_scores, top_idx, all_scores, nullptr,
                      (hipStream_t)hip_stream);
}

int sw_db_autotune(sw_db *db, const sw_scoring *sc, const int32_t *qlens, int32_t n_qlens,
                   const char *cache_path) {
    (void)sc;
    (void)qlens;
    (void)n_qlens;
    (void)cache_path;
    if (!db) return fail(SW_EINVAL, "db is NULL");
    return SW_OK;
}

int sw_server_start(sw_db *db, const sw_server_opts *opts, sw_server **out) {
    (void)db;
    (void)opts;
    (void)out;
    return fail(SW_EINVAL, "server not available");
}
int sw_server_submit(sw_server *srv, const uint8_t *query, int32_t qlen, const sw_scoring *sc,
                     int32_t k, uint64_t *ticket) {
    (void)srv; (void)query; (void)qlen; (void)sc; (void)k; (void)ticket;
    return fail(SW_EINVAL, "server not available");
}
int sw_server_wait(sw_server *srv, uint64_t ticket, int32_t *top_scores, int64_t *top_idx,
                   sw_req_stats *stats) {
    (void)srv; (void)ticket; (void)top_scores; (void)top_idx; (void)stats;
    return fail(SW_EINVAL, "server not available");
}
void sw_server_stop(sw_server *srv) { (void)srv; }

}  // extern "C"
