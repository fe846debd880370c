// Internal interface between the host library (sw_host.cpp) and the gfx950
// kernels (sw_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swmi {

// Residue code reserved for padding: it scores 0 against every query residue
// (the dummy residue of section III.B.1).  Real codes are 0..alphabet-1, so
// the pad code is `alphabet` and profiles have R = alphabet + 1 rows.
// Lanes per wave on gfx950.
constexpr int kWave = 64;
// Subjects per lane-per-subject group: 64 lanes x 2 packed halves.
constexpr int kGroup = 2 * kWave;
// Rows per residue/boundary chunk of the lane-per-subject kernel.
constexpr int kChunk = 4;
// Query profiles are padded to a multiple of this many columns (a strip of 64
// runs past the end of a profile padded to 32; those columns score 0).
constexpr int kQPad = 32;

// Exactness ceilings of the narrow tiers (see sw_kernels.hip for the proofs).
constexpr int kThrF16 = 1920;    // fp16 holds every integer in [-2048, 2048]
constexpr int kThrI16 = 32767;   // saturating int16
// The fp16 kernels keep values in a frame that moves by alpha per subject
// row and per column within groups of kFrameCols (see sw_kernels.hip).
// Offsets reach (kFrameRows + kFrameCols - 1) * alpha, so the ceiling for a
// query with gap extension alpha is kThrF16 - (kFrameRows + kFrameCols) *
// alpha; the lane-per-subject kernel flags every lane above kLaneFlagAlpha.
// Above kFrameMaxAlpha the planner prefers the int16 tier, and the packed
// wave-per-pair kernel flags every pair.
constexpr int kFrameRows = 32;
constexpr int kFrameCols = 4;
constexpr int kFrameMaxAlpha = 28;
constexpr int kLaneFlagAlpha = (kThrF16 - 1) / (kFrameRows + kFrameCols);   // 53
__host__ __device__ inline int lane_frame_thr(int thr, int alpha) {
    if (alpha > kLaneFlagAlpha) return 0;
    const int c = kThrF16 - (kFrameRows + kFrameCols) * alpha;
    return thr < c ? thr : c;
}

enum Tier : int { TIER_F16X2 = 1, TIER_I16X2 = 2 };

// Per-call description of the queries on the device, indexed by query slot.
// Slot q's profile is R rows x mpad[q] int8 at qp[q]; its scores go to row q
// of the score matrix.
struct QuerySet {
    const int8_t *const *qp;
    // score-profile kernel only: per slot, the A x A matrix followed by the
    // mpad query codes (past the query: the pad letter A); nullptr otherwise
    const uint8_t *const *qc;
    const int32_t *mpad;     // padded length (multiple of kQPad, even)
    const int32_t *qlen;     // real length
    const int32_t *gap;      // alpha, beta of slot q at gap[2q], gap[2q+1]
};

struct InterArgs {
    const uint16_t *codes;   // pair codes lo*R + hi per (chunk, lane, row)
    const int64_t *grp_base; // first code (uint16 index) of each group
    const int32_t *grp_rows; // rows of each group (multiple of kChunk)
    const int32_t *grp_ids;  // caller ids: [g*128 + lane] lo half, [g*128 + 64 + lane] hi half
    int32_t n_groups;
    const int32_t *item_q;   // work item -> query
    const int32_t *item_g;   // work item -> first group of its block of `waves` groups
    int32_t n_items;
    int32_t *counter;        // work-queue head, zero before launch
    QuerySet qs;
    int32_t R;
    int32_t thr;             // a lane whose best reaches thr is flagged (fp16: see lane_frame_thr)
    uint32_t *scratch;       // boundary columns: per (slot, wave) max_rows * 64 * 2 dwords
    int32_t max_rows;
    int32_t *scores;         // [query][n_seqs], caller order
    int64_t n_seqs;
    int32_t *ovf_q, *ovf_id, *ovf_count;
    int64_t ovf_cap;
};

struct IntraArgs {
    const uint8_t *res;      // all residues, caller order
    const int64_t *off;      // n_seqs + 1 offsets
    const int32_t *item_q;   // work item -> query
    const int32_t *item_ids; // work item -> `waves` subject ids (-1 = none)
    int32_t n_items;         // used when n_items_dev == nullptr
    const int32_t *n_items_dev;
    int32_t *counter;
    QuerySet qs;
    int32_t R;
    int32_t *pass_scratch;   // per (slot, wave): (max_len_pad) x 2 int32
    int64_t max_len_pad;     // rows per scratch slot (>= longest subject rounded to 64, + 128)
    int32_t *scores;
    int64_t n_seqs;
    // packed-fp16 variant only: flagged pairs go to the exact recompute list
    int32_t thr;
    int32_t *ovf_q, *ovf_id, *ovf_count;
    int64_t ovf_cap;
};

// Raise the dynamic-LDS limit of every kernel variant (once per device, before
// any launch or stream capture).
hipError_t prepare_kernels();

// Launchers (return hipError_t of the launch).
// The lane-per-subject kernel; with `la` non-null and ti in {4, 8, 16} (fp16
// tier at strip kFuseStrip only) it first works through la's wave-per-pair
// items, one subject per wave (la.item_ids holds `waves` ids per item), with
// the wave-per-pair strip ti, in its own workgroups.
constexpr int kFuseStrip = 32;
hipError_t launch_inter(const InterArgs &a, const IntraArgs *la, int ti, int tier, int strip,
                        int waves, int grid, hipStream_t st);
int inter_lds_bytes(int R, int strip, int ti = 0, int waves = 4);
// resident workgroups that fit (ti as for launch_inter)
int inter_max_grid(int R, int tier, int strip, int waves, int ti = 0);

// Score-profile variant of the lane-per-subject kernel (fp16 tier, strip 32,
// 4 waves per workgroup, alphabets of at most 23 letters); needs qs.qc.
hipError_t launch_inter_sp(const InterArgs &a, int strip, int waves, int grid, hipStream_t st);
int inter_sp_lds_bytes(int R, int waves);
int inter_sp_max_grid(int R, int waves);
constexpr int kSpMaxAlphabet = 23;

hipError_t launch_intra(const IntraArgs &a, int T, int waves, int grid, hipStream_t st);
int intra_lds_bytes(int R, int T);
// LDS of a wave-per-pair workgroup: the profile and one feed ring per wave.
int wpp_lds_bytes(int R, int T, int waves);
// Packed-fp16 wave-per-pair kernel: each wave aligns one query with two
// subjects (item_ids holds 2 * waves ids per item).
hipError_t launch_intra2(const IntraArgs &a, int T, int waves, int grid, hipStream_t st);

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);

// Alignment with traceback for a list of subjects against one query.
struct AlignArgs {
    const uint8_t *res;      // all residues, caller order
    const int64_t *off;      // n_seqs + 1 offsets
    const int64_t *ids;      // n_pairs subject ids
    int32_t n_pairs;
    const int8_t *qp;        // query profile: R rows x mpad columns
    int32_t mpad, qlen, ldq; // ldq: direction row stride, qlen rounded up to 16
    int32_t alpha, beta, R;
    uint8_t *dir;            // direction bytes; pair p's len x ldq block at dir + dir_off[p]
    const int64_t *dir_off;
    int32_t *pass_scratch;   // per (slot, wave): max_len_pad x 2 int32 (H, F of a pass boundary)
    int64_t max_len_pad;
    int32_t *end;            // per pair: score, end row, end column (forward kernel output)
    uint32_t *ops;           // per pair: runs at ops + ops_off[p], capacity len + qlen
    const int64_t *ops_off;
    int32_t *out;            // per pair: score, q_begin, q_end, s_begin, s_end, n_ops
};
constexpr int kAlignWaves = 4;    // pairs per workgroup (they share the query profile)
// Pipelined forward pass (one workgroup per pair, one wave per pass): most
// passes (waves), rows of a pass boundary in the LDS ring, and the lag in
// steps between consecutive passes.
constexpr int kAlignPipeMax = 16;
constexpr int kAlignPipeRing = 256;
constexpr int kAlignPipeLag = 128;
__host__ __device__ constexpr int align_pipe_prof_bytes(int R, int T, int P) {
    return P * R * (64 * T + 16);   // int8 profiles of P passes
}
__host__ __device__ constexpr int align_pipe_lds_bytes(int R, int T, int P) {
    return align_pipe_prof_bytes(R, T, P) + (P - 1) * kAlignPipeRing * 8 + 3 * P * 4;
}
// Columns per lane of the pipelined forward pass for this query (its pass
// count in *P_out), or 0 when the query has one pass or its passes need more
// waves or LDS than a workgroup has.
int align_pipe_plan(int R, int qlen, int *P_out);
hipError_t launch_align(const AlignArgs &a, hipStream_t st);

// Device scratch of the entry point that allocates nothing
// (sw_db_search_dev_noalloc): one fixed array per GPU, held until the process
// ends.  noalloc_scratch_init (called once per device by sw_db_open, with that
// device current) takes the array's device address; noalloc_scratch returns it
// (nullptr before initialisation).
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;
hipError_t noalloc_scratch_init(int device);
uint8_t *noalloc_scratch(int device);

// Arguments of the kernel that writes the per-call state of one no-allocation
// search into the scratch (see noalloc_setup_kernel).
struct NoAllocSetup {
    const uint8_t *q;            // query codes, device memory
    int32_t qlen, mpad, R, A;
    int8_t matrix[32 * 32];      // A x A, row = query residue
    int32_t alpha, beta;
    int8_t *prof;                // R x mpad
    const int8_t **qp;           // one-slot query set
    int32_t *mpad_out, *qlen_out, *gap_out;
    int32_t *it_q, *it_g;        // lane-per-subject items
    int32_t n_inter, waves;
    int32_t *il_q, *il_ids;      // wave-per-pair items, `per` ids each
    int32_t n_intra, per;
    const int32_t *long_static;  // the database's long list (device)
    int32_t n_static;
    const int32_t *grp_ids;      // group slots (device), for groups g_cut..n_groups-1
    int32_t g_cut, n_groups;
};
hipError_t launch_noalloc_setup(const NoAllocSetup &s, hipStream_t st);

// Top-k by (score desc, index asc) over rows of `n` scores, `nq` rows.
struct TopkWork {
    uint32_t *hist;      // nq * 256
    int32_t *state;      // nq * 4: prefix, kleft, cnt_gt, pad
    int32_t *eqcnt;      // nq * kTopkBlocks
    int32_t *cand_s;     // nq * k
    int32_t *cand_i;     // nq * k
};
constexpr int kTopkBlocks = 256;
// rows: nq row indices into `scores` (nullptr = rows 0..nq-1).
hipError_t launch_topk(const int32_t *scores, int64_t n, int32_t nq, const int32_t *rows,
                       int32_t k, const TopkWork &w, int32_t *top_s, int64_t *top_i,
                       hipStream_t st);

}  // namespace swmi
