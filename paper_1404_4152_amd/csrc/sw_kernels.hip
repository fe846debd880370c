// gfx950 kernels for exact affine-gap Smith-Waterman database search.
//
// Recurrence (section II.A, Eq. 1), with i over the subject and j over the
// query, and substitution score M[Q[j]][S[i]]:
//   H(i,j) = max{0, H(i-1,j-1) + M, E(i,j), F(i,j)}
//   E(i,j) = max{E(i-1,j) - alpha, H(i-1,j) - beta}
//   F(i,j) = max{F(i,j-1) - alpha, H(i,j-1) - beta}
// The int32 and int16 paths evaluate it in the per-cell form
//   h = max(hdiag + s, e, f); t = h - beta; e' = max(e - alpha, t, 0);
//   f' = max(f - alpha, t, 0); best = max(best, h)
// Flooring E and F at 0 leaves H unchanged: H = max(0, ...) already, and by
// induction the floored E is max(E, 0) because alpha >= 0.  Sharing
// t = h - beta between E (next row) and F (next column) gives 7.5 VALU ops per
// cell with a 3-input max, the running best taking one max3 per two cells.
// The fp16 tier of the lane-per-subject kernel keeps its values in a frame
// that moves by alpha per subject row and per query column within groups of
// four columns, and needs 5.75 (FrameStrip below).
//
// Kernels:
//  * inter_kernel: one lane per subject, two subjects per 32-bit lane in packed
//    16-bit halves (the inter-sequence model of section III.B).  Subjects are
//    length-sorted into groups of 128; a group is one wavefront.  Each lane
//    keeps a strip of T query columns of H and E in registers and streams its
//    subjects' rows; the column crossing to the next strip (H and F of every
//    row) goes through a per-wave boundary buffer.  This is the tiled SW
//    computation of the conclusion.  The substitution scores of the strip sit
//    in LDS as a pair profile P[a*R + b][j] = (M[q_j][a], M[q_j][b]) so that one
//    dword read feeds both halves of a lane.  Its fused variants (TI > 0) first
//    hand out the long list's wave-per-pair items from the same work queue.
//  * intra_kernel: one wavefront per (query, subject) pair, int32 and exact
//    (the intra-sequence model of section III.C, laid out as a systolic
//    array along anti-diagonals rather than striped).  Lane l owns T query
//    columns; at step t it computes subject row t - l; H and F of its last
//    column move to lane l+1 with a DPP wave shift.  Each lane reads its
//    subject residue, and lane 0 its incoming H and F, from a per-wave LDS
//    ring.  Serves long subjects, small databases and the exact recompute of
//    flagged narrow-tier lanes.
//  * intra2_kernel: the same schedule in packed fp16, two subjects per wave.
//  * align_fwd_kernel / align_pipe_kernel / align_back_kernel: alignment with
//    traceback (the same schedule in int32 storing a direction byte per cell,
//    one wave per pair or one wave per pass of a pair, then a walk back).
//  * topk_*: radix-select top-k of the score rows (one-workgroup bitonic sort
//    for rows of at most 4,096 subjects).
//
// Narrow-tier exactness.  A tier computes exactly while every intermediate
// value is representable; it flags a lane whose best reaches the tier's
// threshold `thr` and the host recomputes that pair in int32.  Claim: if the
// true best is < thr, the tier's result equals it; otherwise the lane is
// flagged.  All values up to the first cell whose true H reaches thr are
// exact (nonnegative values stay below thr + 127, negative values only lose
// magnitude, and floors at 0 hide them), so that cell's computed H is its true
// value >= thr and the running best reaches thr.
//   F16X2: fp16 holds every integer in [-2048, 2048]; thr = 1920 keeps
//          thr - 1 + max(M) <= 2048 for |M| <= 127 (wave-per-pair kernel; the
//          lane-per-subject frame lowers it by 36 alpha).  alpha and beta are
//          clamped to 2048: for lanes below thr a larger penalty gives the same
//          (zero-floored) E and F.  Once flagged, values may round or reach
//          +inf but never NaN (only finite constants are subtracted).
//   I16X2: saturating int16; thr = 32767, the saturation ceiling.
#include "sw_internal.h"

#include <algorithm>
#include <mutex>
#include <type_traits>

namespace swmi {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef short s2 __attribute__((ext_vector_type(2)));
typedef unsigned short u2 __attribute__((ext_vector_type(2)));

template <class V>
__device__ __forceinline__ V as_v(uint32_t x) { return __builtin_bit_cast(V, x); }
template <class V>
__device__ __forceinline__ uint32_t as_u(V v) { return __builtin_bit_cast(uint32_t, v); }

// ---------------------------------------------------------------------------
// Lane arithmetic of the two packed tiers.
// ---------------------------------------------------------------------------
template <int TIER> struct Lane;

// The fp16 tier's cell arithmetic is the frame form (LaneFrame and
// FrameStrip below); this holds the encoding and the epilogue.
template <> struct Lane<TIER_F16X2> {
    typedef h2 V;
    static __device__ __forceinline__ V zero() { return V{(_Float16)0.0f, (_Float16)0.0f}; }
    static __device__ __forceinline__ uint16_t enc(int v) {
        return __builtin_bit_cast(uint16_t, (_Float16)(float)v);
    }
    // (score, flagged) of one half
    static __device__ __forceinline__ int value(V b, int half, int thr, bool *flag) {
        const float x = half ? (float)b.y : (float)b.x;
        *flag = !(x < (float)thr);
        return *flag ? -1 : (int)x;
    }
};

template <> struct Lane<TIER_I16X2> {
    typedef s2 V;
    u2 ua, ub;
    __device__ Lane(int alpha, int beta) {
        ua = u2{(unsigned short)alpha, (unsigned short)alpha};
        ub = u2{(unsigned short)beta, (unsigned short)beta};
    }
    static __device__ __forceinline__ V zero() { return V{0, 0}; }
    static __device__ __forceinline__ uint16_t enc(int v) { return (uint16_t)(int16_t)v; }
    __device__ __forceinline__ V diag(V hd, V s) const { return __builtin_elementwise_add_sat(hd, s); }
    __device__ __forceinline__ V hmax(V hd, V e, V f) const {
        return __builtin_elementwise_max(__builtin_elementwise_max(hd, e), f);
    }
    // h >= 0 here, so the unsigned saturating subtraction is max(h - beta, 0).
    __device__ __forceinline__ V open(V h) const {
        return (V)__builtin_elementwise_sub_sat((u2)h, ub);
    }
    __device__ __forceinline__ V gap(V g, V t) const {
        return __builtin_elementwise_max((V)__builtin_elementwise_sub_sat((u2)g, ua), t);
    }
    __device__ __forceinline__ V best2(V b, V h0, V h1) const {
        return __builtin_elementwise_max(__builtin_elementwise_max(b, h0), h1);
    }
    static __device__ __forceinline__ int value(V b, int half, int thr, bool *flag) {
        const int x = half ? (int)b.y : (int)b.x;
        *flag = x >= thr;
        return *flag ? -1 : x;
    }
};

// a / R for a < R*R <= 1089 via a multiply (checked on the host for every R).
__device__ __forceinline__ int div_r(int a, int magic) { return (a * magic) >> 16; }

// ---------------------------------------------------------------------------
// Lane-per-subject kernel.  Strip evaluates the textbook form and serves the
// int16 tier; the fp16 tier uses FrameStrip.
// ---------------------------------------------------------------------------
template <int T, int TIER>
struct Strip {
    typedef Lane<TIER> L;
    typedef typename L::V V;

    // One subject row across the strip.  Pc holds this row's pair-profile
    // values; the next row's (`nxt`) are loaded into Pn at the start, so the
    // LDS latency hides behind a full row of arithmetic.  The two buffers
    // alternate row by row and stay in fixed registers.
    // hb_prev = H(i-1, j0-1), fin = F(i, j0).  Returns H(i, j0+T-1), F(i, j0+T).
    static __device__ __forceinline__ void row(const L &ops, V (&H)[T], V (&E)[T],
                                               const uint4 (&Pc)[T / 4], uint4 (&Pn)[T / 4],
                                               const uint4 *nxt, uint32_t hb_prev, uint32_t fin,
                                               V &best, uint32_t &hout, uint32_t &fout) {
        V hdiag = as_v<V>(hb_prev);
        V f = as_v<V>(fin);
#pragma unroll
        for (int j4 = 0; j4 < T / 4; ++j4) Pn[j4] = nxt[j4];
#pragma unroll
        for (int j4 = 0; j4 < T / 4; ++j4) {
            const uint32_t pv[4] = {Pc[j4].x, Pc[j4].y, Pc[j4].z, Pc[j4].w};
#pragma unroll
            for (int u = 0; u < 4; u += 2) {
                const int j = j4 * 4 + u;
                V h0, h1;
                {
                    const V hold = H[j];
                    h0 = ops.hmax(ops.diag(hdiag, as_v<V>(pv[u])), E[j], f);
                    const V t = ops.open(h0);
                    E[j] = ops.gap(E[j], t);
                    f = ops.gap(f, t);
                    H[j] = h0;
                    hdiag = hold;
                }
                {
                    const V hold = H[j + 1];
                    h1 = ops.hmax(ops.diag(hdiag, as_v<V>(pv[u + 1])), E[j + 1], f);
                    const V t = ops.open(h1);
                    E[j + 1] = ops.gap(E[j + 1], t);
                    f = ops.gap(f, t);
                    H[j + 1] = h1;
                    hdiag = hold;
                }
                best = ops.best2(best, h0, h1);
            }
        }
        hout = as_u(H[T - 1]);
        fout = as_u(f);
        // Materialise this row's state here: without the fences the compiler
        // sinks E and the running best into the next rows and keeps several
        // rows of H alive, which spills.
#pragma unroll
        for (int j = 0; j < T; ++j) asm volatile("" : "+v"(H[j]), "+v"(E[j]));
        asm volatile("" : "+v"(best));
    }

    // All rows of one group against one strip.  HAS_IN: read the boundary
    // column left by the previous strip; HAS_OUT: write it for the next.
    // Every load is unconditional (addresses clamp at the last chunk) so the
    // compiler can count outstanding loads instead of draining them.
    template <bool HAS_IN, bool HAS_OUT>
    static __device__ __forceinline__ void pass(const L &ops, V &best, const uint16_t *codes,
                                                uint32_t *wsc, int nch, const uint32_t *lds,
                                                int RS) {
        V H[T], E[T];
#pragma unroll
        for (int j = 0; j < T; ++j) { H[j] = L::zero(); E[j] = L::zero(); }
        uint32_t hb_prev = 0;
        const int last = nch - 1;
        uint2 cd = *(const uint2 *)codes;
        uint2 cd_n = *(const uint2 *)(codes + (size_t)(last < 1 ? last : 1) * 256);
        uint4 b0 = make_uint4(0, 0, 0, 0), b1 = make_uint4(0, 0, 0, 0);
        if (HAS_IN) {
            b0 = ((const uint4 *)wsc)[0];
            b1 = ((const uint4 *)wsc)[1];
        }
        uint4 P0[T / 4], P1[T / 4];
        {
            const uint4 *src = (const uint4 *)(lds + (cd.x & 0xffffu) * RS);
#pragma unroll
            for (int j4 = 0; j4 < T / 4; ++j4) P0[j4] = src[j4];
        }
        for (int c = 0; c < nch; ++c) {
            const int c1 = c + 1 < last ? c + 1 : last;
            const int c2 = c + 2 < last ? c + 2 : last;
            const uint2 cd_nn = *(const uint2 *)(codes + (size_t)c2 * 256);
            uint4 b0n = make_uint4(0, 0, 0, 0), b1n = make_uint4(0, 0, 0, 0);
            if (HAS_IN) {
                b0n = ((const uint4 *)(wsc + (size_t)c1 * 512))[0];
                b1n = ((const uint4 *)(wsc + (size_t)c1 * 512))[1];
            }
            const uint4 *n1 = (const uint4 *)(lds + (cd.x >> 16) * RS);
            const uint4 *n2 = (const uint4 *)(lds + (cd.y & 0xffffu) * RS);
            const uint4 *n3 = (const uint4 *)(lds + (cd.y >> 16) * RS);
            const uint4 *n4 = (const uint4 *)(lds + (cd_n.x & 0xffffu) * RS);
            uint32_t o[8];
            row(ops, H, E, P0, P1, n1, hb_prev, b0.y, best, o[0], o[1]);
            hb_prev = b0.x;
            row(ops, H, E, P1, P0, n2, hb_prev, b0.w, best, o[2], o[3]);
            hb_prev = b0.z;
            row(ops, H, E, P0, P1, n3, hb_prev, b1.y, best, o[4], o[5]);
            hb_prev = b1.x;
            row(ops, H, E, P1, P0, n4, hb_prev, b1.w, best, o[6], o[7]);
            hb_prev = b1.z;
            if (HAS_OUT) {
                uint4 *dst = (uint4 *)(wsc + (size_t)c * 512);
                dst[0] = make_uint4(o[0], o[1], o[2], o[3]);
                dst[1] = make_uint4(o[4], o[5], o[6], o[7]);
            }
            cd = cd_n;
            cd_n = cd_nn;
            b0 = b0n;
            b1 = b1n;
        }
    }
};

// ---------------------------------------------------------------------------
// Frame form of the fp16 tier (lane-per-subject kernel).
//
// E loses alpha per subject row and F loses alpha per query column.  Cell
// (r, j) is stored shifted by o(r, j) = c_r + alpha * (j mod G), G =
// kFrameCols, where c_r = r * alpha (r counted from the start of a period of
// kFrameRows rows).  Then E entering row r + 1 sits at o(r, j) + alpha and F
// entering column j + 1 at o(r, j) + alpha unless j + 1 starts a new group of
// G columns, where its offset drops back by (G - 1) alpha:
//   h = max(hdiag + s', e, f);         u = h + (alpha - beta);
//   e' = max(e, u, fl[j mod G]);       f' = max(f, u)  [- G alpha after class G-1]
// is Eq. 1, with the diagonal's offset change folded into the profile
// (s' = s + 2 alpha, or s + (2 - G) alpha into a class-0 column, whose
// diagonal comes from class G - 1 of the row above).  One subtraction per G
// columns serves F and none serves E: 5.75 VALU ops per cell with the running
// best at G = 4, against 7.5 for the textbook form.  Only E is floored (fl[c]
// = true 0 at offset o(r + 1, j) for class c); F may go negative, which H never
// sees because E >= 0 (H = max(0, ...) needs one floored operand).
//
// Running best: cells (r, j) and (r - 1, j + 1) for even j share the offset
// c_r + alpha * (j mod G) (j mod G < G - 1), and H(r - 1, j + 1) is the
// diagonal operand left over after column j + 1, so one max3 per two cells
// covers row r's even columns and row r - 1's odd ones into one register per
// even class, each kept in the frame of the current row (+alpha per row).  The
// last row's odd columns are taken after the last row.  Each period the carried
// H, E, floors and bests drop by kFrameRows * alpha.
//
// Exactness: until the first cell whose true H reaches thr, every true value
// lies in [-2048, thr + 126] and offsets add at most (kFrameRows + G - 1) alpha,
// so thr = kThrF16 - (kFrameRows + G) alpha keeps all values exact integers in
// fp16; that cell's offset H is exact and >= thr + its offset.  Rounding is
// monotone and every offset applied is an exactly representable constant, so
// the running best stays >= thr + its offset and the converted best >= thr:
// the lane is flagged.  For alpha > kLaneFlagAlpha the ceiling is 0 and every
// lane is flagged (alpha is clamped there, so values stay finite).
// ---------------------------------------------------------------------------
struct LaneFrame {
    h2 nalpha;    // -alpha
    h2 palpha;    // +alpha
    h2 nu;        // alpha - beta
    h2 rebase;    // -kFrameRows * alpha
    h2 ngroup;    // -kFrameCols * alpha
    int alpha;
    int bias0;    // profile bias of a class-0 column: (2 - kFrameCols) * alpha
    int bias1;    // of any other column: 2 * alpha
    __device__ LaneFrame(int alpha_, int beta) {
        alpha = min(alpha_, kLaneFlagAlpha);
        beta = min(beta, 2048);
        nalpha = k(-1);
        palpha = k(1);
        const _Float16 u = (_Float16)(float)(alpha - beta);
        nu = h2{u, u};
        rebase = k(-kFrameRows);
        ngroup = k(-kFrameCols);
        bias0 = (2 - kFrameCols) * alpha;
        bias1 = 2 * alpha;
    }
    // n * alpha in both halves (exact: |n * alpha| <= (kFrameRows + kFrameCols) * 53)
    __device__ h2 k(int n) const {
        const _Float16 v = (_Float16)(float)(n * alpha);
        return h2{v, v};
    }
};

template <int T>
struct FrameStrip {
    static_assert(kFrameCols == 4 && T % kFrameCols == 0, "a profile quad is one column group");
    typedef h2 V;
    static __device__ __forceinline__ V max3(V a, V b, V c) {
        return __builtin_elementwise_maximum(__builtin_elementwise_maximum(a, b), c);
    }

    // One cell of column class C; hdiag and f carry along the row.
    template <int C>
    static __device__ __forceinline__ V cell(const LaneFrame &ops, V &H, V &E, uint32_t s, V &hdiag,
                                             V &f, V fl) {
        const V hold = H;
        const V h = max3(hdiag + as_v<V>(s), E, f);
        const V t = h + ops.nu;
        E = max3(E, t, fl);
        f = __builtin_elementwise_maximum(f, t);
        if (C == kFrameCols - 1) f += ops.ngroup;
        H = h;
        hdiag = hold;
        return h;
    }

    // One subject row across the strip: Pc holds this row's pair-profile
    // values, and the next row's are loaded into Pn at the start so the LDS
    // latency hides behind the row.  Alternating the two buffers row by row
    // keeps every value in fixed registers (a single buffer refilled in place
    // makes the compiler copy it back at every loop edge).
    // hb_prev = H(r-1, j0-1) at offset c_r + (G-2) alpha, fin = F(r, j0) at
    // offset c_r, FL[c] = c_r + (c+1) alpha (the E floor of class c); B[0],
    // B[1] = running bests of classes 0 and 2, at offsets c_r and c_r + 2 alpha.
    static __device__ __forceinline__ void row(const LaneFrame &ops, V (&H)[T], V (&E)[T],
                                               const uint4 (&Pc)[T / 4], uint4 (&Pn)[T / 4],
                                               const uint4 *nxt, uint32_t hb_prev, uint32_t fin,
                                               const V *FL, V (&B)[2], uint32_t &hout,
                                               uint32_t &fout) {
        V f = as_v<V>(fin);
#pragma unroll
        for (int j4 = 0; j4 < T / 4; ++j4) Pn[j4] = nxt[j4];
        // The cells of FrameStrip::cell, in an order that puts independent
        // work between each column's dependent steps h -> t -> f: gfx950 needs
        // a wait state before a packed fp16 instruction that reads the result
        // of the packed fp16 instruction just before it.  Between h and t goes
        // the next column's diagonal sum (H[j] still holds row r - 1 there);
        // between t and f the running best of an even column, and the E
        // update of the column before (E[j] is next read by the row below).
        V d = as_v<V>(hb_prev) + as_v<V>(Pc[0].x);
        V tp = d;
#pragma unroll
        for (int j = 0; j < T; ++j) {
            const V h = max3(d, E[j], f);
            if (j + 1 < T) d = H[j] + as_v<V>(pval(Pc, j + 1));
            const V t = h + ops.nu;
            // classes 0 and 2: (r, j) and (r - 1, j + 1) share an offset
            if (!(j & 1)) B[(j >> 1) & 1] = max3(B[(j >> 1) & 1], h, H[j + 1]);
            if (j > 0) E[j - 1] = max3(E[j - 1], tp, FL[(j - 1) & 3]);
            f = __builtin_elementwise_maximum(f, t);
            if ((j & 3) == 3) f += ops.ngroup;
            H[j] = h;
            tp = t;
        }
        E[T - 1] = max3(E[T - 1], tp, FL[(T - 1) & 3]);
        hout = as_u(H[T - 1]);
        fout = as_u(f);
#pragma unroll
        for (int j = 0; j < T; ++j) asm volatile("" : "+v"(H[j]), "+v"(E[j]));
        asm volatile("" : "+v"(B[0]), "+v"(B[1]));
    }

    // Column j's value of a row of profile quads.
    static __device__ __forceinline__ uint32_t pval(const uint4 (&P)[T / 4], int j) {
        const uint4 &q = P[j >> 2];
        return (j & 3) == 0 ? q.x : (j & 3) == 1 ? q.y : (j & 3) == 2 ? q.z : q.w;
    }

    // All rows of one group against one strip; `best_io` is a true value on
    // entry and exit.  Loads as in Strip::pass.
    template <bool HAS_IN, bool HAS_OUT>
    static __device__ __forceinline__ void pass(const LaneFrame &ops, V &best_io,
                                                const uint16_t *codes, uint32_t *wsc, int nch,
                                                const uint32_t *lds, int RS) {
        constexpr int kPeriodChunks = kFrameRows / kChunk;
        V H[T], E[T];
        // Row -1: H is the true 0 boundary at offset o(-1, j), E the true 0
        // floor at o(0, j).
#pragma unroll
        for (int j = 0; j < T; ++j) {
            H[j] = ops.k((j & 3) - 1);
            E[j] = ops.k(j & 3);
        }
        // E floors: class c of chunk row x uses FL[x + c] = c_r + (x + c + 1) alpha
        // (row r + 1's class c floor is row r's class c + 1 floor), so the
        // seven floors of a chunk move once per chunk.
        constexpr int kFloors = kChunk + kFrameCols - 1;
        V FL[kFloors];
#pragma unroll
        for (int x = 0; x < kFloors; ++x) FL[x] = ops.k(x + 1);
        const V chunk_step = ops.k(kChunk);
        V B[2] = {best_io, ops.k(0)};
        // true 0 at the offset of a class-0 column's diagonal: left edge of the
        // first strip, and the row above the first row
        V z = ops.k(kFrameCols - 2);
        uint32_t hb_prev = as_u(z);
        // F left of the first strip: any true value <= 0 will do (H >= E >= 0)
        const uint32_t f_edge = as_u(ops.nalpha);
        const int last = nch - 1;
        uint2 cd = *(const uint2 *)codes;
        uint2 cd_n = *(const uint2 *)(codes + (size_t)(last < 1 ? last : 1) * 256);
        uint4 b0 = make_uint4(0, 0, 0, 0), b1 = make_uint4(0, 0, 0, 0);
        if (HAS_IN) {
            b0 = ((const uint4 *)wsc)[0];
            b1 = ((const uint4 *)wsc)[1];
        }
        uint4 P0[T / 4], P1[T / 4];
        {
            const uint4 *src = (const uint4 *)(lds + (cd.x & 0xffffu) * RS);
#pragma unroll
            for (int j4 = 0; j4 < T / 4; ++j4) P0[j4] = src[j4];
        }
        for (int c = 0; c < nch; ++c) {
            if (c != 0 && c % kPeriodChunks == 0) {
#pragma unroll
                for (int j = 0; j < T; ++j) { H[j] += ops.rebase; E[j] += ops.rebase; }
#pragma unroll
                for (int x = 0; x < kFloors; ++x) FL[x] += ops.rebase;
                B[0] += ops.rebase;
                B[1] += ops.rebase;
                if (HAS_IN) hb_prev = as_u(as_v<V>(hb_prev) + ops.rebase);
                else z += ops.rebase;
            }
            const int c1 = c + 1 < last ? c + 1 : last;
            const int c2 = c + 2 < last ? c + 2 : last;
            const uint2 cd_nn = *(const uint2 *)(codes + (size_t)c2 * 256);
            uint4 b0n = make_uint4(0, 0, 0, 0), b1n = make_uint4(0, 0, 0, 0);
            if (HAS_IN) {
                b0n = ((const uint4 *)(wsc + (size_t)c1 * 512))[0];
                b1n = ((const uint4 *)(wsc + (size_t)c1 * 512))[1];
            }
            const uint4 *nx[4] = {(const uint4 *)(lds + (cd.x >> 16) * RS),
                                  (const uint4 *)(lds + (cd.y & 0xffffu) * RS),
                                  (const uint4 *)(lds + (cd.y >> 16) * RS),
                                  (const uint4 *)(lds + (cd_n.x & 0xffffu) * RS)};
            const uint32_t hb_in[4] = {hb_prev, b0.x, b0.z, b1.x};
            const uint32_t f_in[4] = {b0.y, b0.w, b1.y, b1.w};
            uint32_t o[8];
#pragma unroll
            for (int x = 0; x < kChunk; ++x) {
                const uint32_t hb = HAS_IN ? hb_in[x] : as_u(z), fi = HAS_IN ? f_in[x] : f_edge;
                if (x & 1) row(ops, H, E, P1, P0, nx[x], hb, fi, FL + x, B, o[2 * x], o[2 * x + 1]);
                else row(ops, H, E, P0, P1, nx[x], hb, fi, FL + x, B, o[2 * x], o[2 * x + 1]);
                B[0] += ops.palpha;
                B[1] += ops.palpha;
                if (!HAS_IN) z += ops.palpha;
            }
#pragma unroll
            for (int x = 0; x < kFloors; ++x) FL[x] += chunk_step;
            hb_prev = b1.z;
            if (HAS_OUT) {
                uint4 *dst = (uint4 *)(wsc + (size_t)c * 512);
                dst[0] = make_uint4(o[0], o[1], o[2], o[3]);
                dst[1] = make_uint4(o[4], o[5], o[6], o[7]);
            }
            cd = cd_n;
            cd_n = cd_nn;
            b0 = b0n;
            b1 = b1n;
        }
        // The last row's odd columns (classes 1 and 3), at the offsets of B[0]
        // and B[1] after the last row's step.
#pragma unroll
        for (int j = 0; j < T; j += 4) {
            B[0] = __builtin_elementwise_maximum(B[0], H[j + 1]);
            B[1] = __builtin_elementwise_maximum(B[1], H[j + 3]);
        }
        // B[0] sits at offset FL[0] - alpha, B[1] at FL[0] + alpha
        best_io = __builtin_elementwise_maximum(B[0] - (FL[0] + ops.nalpha),
                                                B[1] - (FL[0] + ops.palpha));
    }
};

// Occupancy the register budget is sized for (waves per SIMD).
// The fp16 frame form needs a few more registers than 128 at strip 16.
template <int T, int TIER> struct InterOcc {
    static constexpr int value = T <= 16 ? (TIER == TIER_F16X2 ? 3 : 4) : (T <= 32 ? 2 : 1);
};

template <int T, int W>
__device__ __forceinline__ void intra_item(const IntraArgs &a, int it, uint32_t *lds,
                                           int32_t *wsc);

// TI > 0: the work queue first hands out the long list's wave-per-pair items
// (`la`, one subject per wave, strip TI), then the lane-per-subject items, so
// the long list runs in this kernel's own workgroup slots.
template <int T, int W, int TIER, int TI>
__global__ void __launch_bounds__(W * 64, (InterOcc<T, TIER>::value))
    inter_kernel(InterArgs a, IntraArgs la, int magic) {
    typedef Lane<TIER> L;
    typedef typename L::V V;
    constexpr int RS = T + 4;                 // dwords per pair-profile row (padded)
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const int R = a.R;
    const int RR = R * R;
    uint32_t *stage = lds + RR * RS;          // R x T/2 dwords: the strip's profile, 16-bit
    __shared__ int s_item;

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    // Penalties above the tier's range only change values that are floored
    // to 0 anyway, so they are clamped to it.
    constexpr int kCap = TIER == TIER_I16X2 ? 32767 : 2048;
    uint32_t *wsc = a.scratch + ((size_t)(blockIdx.x * W + w) * (size_t)a.max_rows) * 128 + lane * 8;
    const int n_long = TI > 0 ? la.n_items : 0;

    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        int it = s_item;
        if constexpr (TI > 0) {
            if (it < n_long) {
                const int wv = __builtin_amdgcn_readfirstlane(w);
                int32_t *lwsc = la.pass_scratch + (size_t)(blockIdx.x * W + wv) * (size_t)la.max_len_pad * 2;
                intra_item<TI, W>(la, it, lds, lwsc);   // its first barrier orders the read of s_item
                continue;
            }
            it -= n_long;
        }
        if (it >= a.n_items) break;
        const int q = a.item_q[it];
        const int alpha = a.qs.gap[2 * q], beta = a.qs.gap[2 * q + 1];
        typedef typename std::conditional<TIER == TIER_F16X2, LaneFrame, L>::type Ops;
        const Ops ops(min(alpha, kCap), min(beta, kCap));
        int bias0 = 0, bias1 = 0, thr = a.thr;
        if constexpr (TIER == TIER_F16X2) {
            bias0 = ops.bias0;
            bias1 = ops.bias1;
            thr = lane_frame_thr(a.thr, alpha);
        }
        const int g = a.item_g[it] + w;
        const bool active = g < a.n_groups;
        const int rows = active ? a.grp_rows[g] : 0;
        const int mp = a.qs.mpad[q];
        const int nstrips = (mp + T - 1) / T;   // the last strip may run past mp (scores 0)
        const int8_t *qp = a.qs.qp[q];
        const uint16_t *codes = a.codes + (active ? a.grp_base[g] : 0) + lane * 4;
        V best = L::zero();

        for (int k = 0; k < nstrips; ++k) {
            __syncthreads();   // previous table no longer read; s_item consumed
            for (int e = threadIdx.x; e < R * (T / 2); e += W * 64) {
                const int r = e / (T / 2), jj = e - r * (T / 2);
                const int col = k * T + 2 * jj;    // mp is even, so col < mp covers col + 1
                const int8_t *src = qp + (size_t)r * mp + col;
                const int s0 = col < mp ? src[0] : 0, s1 = col < mp ? src[1] : 0;
                const int b0 = col % kFrameCols == 0 ? bias0 : bias1;   // col + 1 is odd
                stage[e] = (uint32_t)L::enc(s0 + b0) | ((uint32_t)L::enc(s1 + bias1) << 16);
            }
            __syncthreads();
            for (int e = threadIdx.x; e < RR * (T / 2); e += W * 64) {
                const int row = e / (T / 2), jj = e - row * (T / 2);
                const int ra = div_r(row, magic), rb = row - ra * R;
                const uint32_t pa = stage[ra * (T / 2) + jj], pb = stage[rb * (T / 2) + jj];
                uint2 v;
                v.x = (pa & 0xffffu) | (pb << 16);
                v.y = (pa >> 16) | (pb & 0xffff0000u);
                *(uint2 *)(lds + row * RS + 2 * jj) = v;
            }
            __syncthreads();
            if (!active) continue;

            const int nch = rows / kChunk;
            typedef typename std::conditional<TIER == TIER_F16X2, FrameStrip<T>, Strip<T, TIER>>::type S;
            if (k == 0) {
                if (nstrips == 1) S::template pass<false, false>(ops, best, codes, wsc, nch, lds, RS);
                else S::template pass<false, true>(ops, best, codes, wsc, nch, lds, RS);
            } else {
                if (k + 1 == nstrips) S::template pass<true, false>(ops, best, codes, wsc, nch, lds, RS);
                else S::template pass<true, true>(ops, best, codes, wsc, nch, lds, RS);
            }
        }
        if (active) {
            const int ids[2] = {a.grp_ids[g * kGroup + lane], a.grp_ids[g * kGroup + kWave + lane]};
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int id = ids[half];
                if (id < 0) continue;
                bool flag;
                const int v = L::value(best, half, thr, &flag);
                a.scores[(size_t)q * a.n_seqs + id] = v;
                if (flag) {
                    const int pos = atomicAdd(a.ovf_count, 1);
                    if (pos < a.ovf_cap) {
                        a.ovf_q[pos] = q;
                        a.ovf_id[pos] = id;
                    }
                }
            }
        }
    }
}

int inter_lds_bytes(int R, int strip, int ti, int waves) {
    const int lane = (R * R * (strip + 4) + R * (strip / 2)) * 4;
    return ti > 0 ? std::max(lane, wpp_lds_bytes(R, ti, waves)) : lane;
}

static int lds_per_cu() { return 160 * 1024; }

template <int T, int W, int TIER, int TI>
static int inter_resident_t(int R) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, inter_kernel<T, W, TIER, TI>, W * 64,
                                                     inter_lds_bytes(R, T, TI, W)) != hipSuccess)
        per_cu = 0;
    return per_cu;
}

template <int T, int W, int TIER>
static int inter_resident_ti(int R, int ti) {
    if (ti == 0) return inter_resident_t<T, W, TIER, 0>(R);
    if constexpr (T == kFuseStrip && TIER == TIER_F16X2) {
        if (ti == 4) return inter_resident_t<T, W, TIER, 4>(R);
        if (ti == 8) return inter_resident_t<T, W, TIER, 8>(R);
        if (ti == 16) return inter_resident_t<T, W, TIER, 16>(R);
    }
    return 0;
}

int inter_max_grid(int R, int tier, int strip, int waves, int ti) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    }
    // workgroups of this variant that fit on one CU (registers, LDS, waves)
    int per_cu = 0;
#define SWMI_RES_CASE(T_, W_)                                                              \
    if (strip == T_ && waves == W_)                                                        \
        per_cu = tier == TIER_I16X2 ? inter_resident_ti<T_, W_, TIER_I16X2>(R, ti)        \
                                    : inter_resident_ti<T_, W_, TIER_F16X2>(R, ti);
    SWMI_RES_CASE(16, 4) SWMI_RES_CASE(16, 8)
    SWMI_RES_CASE(32, 4) SWMI_RES_CASE(32, 6) SWMI_RES_CASE(32, 8)
    SWMI_RES_CASE(64, 4)
#undef SWMI_RES_CASE
    if (per_cu < 1) {
        // runtime query unavailable: bound by LDS and 8 waves per SIMD
        const int by_lds = lds_per_cu() / (inter_lds_bytes(R, strip, ti, waves) + 64);
        const int by_waves = 32 / waves;
        per_cu = by_lds < by_waves ? by_lds : by_waves;
        if (per_cu < 1) per_cu = 1;
    }
    return per_cu * cus;
}

template <int T, int W, int TIER, int TI>
static hipError_t launch_inter_t(const InterArgs &a, const IntraArgs &la, int grid, hipStream_t st) {
    int magic = (65536 + a.R - 1) / a.R;
    const int lds = inter_lds_bytes(a.R, T, TI, W);
    hipLaunchKernelGGL((inter_kernel<T, W, TIER, TI>), dim3(grid), dim3(W * 64), lds, st, a, la,
                       magic);
    return hipGetLastError();
}

template <int T, int W, int TIER>
static hipError_t launch_inter_ti(const InterArgs &a, const IntraArgs *la, int ti, int grid,
                                  hipStream_t st) {
    if (!la || ti == 0) return launch_inter_t<T, W, TIER, 0>(a, IntraArgs{}, grid, st);
    if constexpr (T == kFuseStrip && TIER == TIER_F16X2) {
        if (ti == 4) return launch_inter_t<T, W, TIER, 4>(a, *la, grid, st);
        if (ti == 8) return launch_inter_t<T, W, TIER, 8>(a, *la, grid, st);
        if (ti == 16) return launch_inter_t<T, W, TIER, 16>(a, *la, grid, st);
    }
    return hipErrorInvalidValue;
}

template <int TIER>
static hipError_t launch_inter_tier(const InterArgs &a, const IntraArgs *la, int ti, int strip,
                                    int waves, int grid, hipStream_t st) {
#define SWMI_INTER_CASE(T_, W_) \
    if (strip == T_ && waves == W_) return launch_inter_ti<T_, W_, TIER>(a, la, ti, grid, st);
    SWMI_INTER_CASE(16, 4) SWMI_INTER_CASE(16, 8)
    SWMI_INTER_CASE(32, 4) SWMI_INTER_CASE(32, 6) SWMI_INTER_CASE(32, 8)
    SWMI_INTER_CASE(64, 4)
#undef SWMI_INTER_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_inter(const InterArgs &a, const IntraArgs *la, int ti, int tier, int strip,
                        int waves, int grid, hipStream_t st) {
    if (tier == TIER_F16X2) return launch_inter_tier<TIER_F16X2>(a, la, ti, strip, waves, grid, st);
    if (tier == TIER_I16X2) return launch_inter_tier<TIER_I16X2>(a, la, ti, strip, waves, grid, st);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Score-profile variant of the lane-per-subject kernel (section III.B.3).
//
// The paper's score profile holds, for the subject residues under the vector
// lanes, their scores against every query letter, so the inner loop over
// query positions reads it at the query letter instead of gathering.  Here
// each lane keeps the score-profile row of its own two subjects' residues at
// one subject row: SP[c][lane] = (M[c][s_lo] + 2 alpha, M[c][s_hi] + 2 alpha)
// for every query letter c, one dword per letter, lane-contiguous in LDS, so
// the read for query column j (letter q_j, the same for the whole wave) is
// conflict-free.  The row is copied, one row ahead, from a letter-pair table
// LPT[a * R + b][c] built once per query in the workgroup's LDS (it depends
// only on the matrix and alpha).  Each lane's T column addresses
// (letter q_j x 256 + lane x 4) are set once per strip.  The pad letter A
// scores 0 (columns past the query).  The arithmetic is FrameStrip's; a
// class-0 column takes its diagonal bias (2 - G) alpha as the table's 2 alpha
// plus -G alpha on the diagonal operand.
// ---------------------------------------------------------------------------
constexpr int kSpLetters = 24;   // letters per table row: query alphabet + pad letter, <= 24

template <int T>
struct FrameStripSP {
    static_assert(kFrameCols == 4 && T % kFrameCols == 0, "column classes");
    typedef h2 V;
    typedef FrameStrip<T> F;

    // Write one profile row (the table row `t` of a subject row's pair code)
    // into this lane's column of the wave's profile buffer.
    static __device__ __forceinline__ void put(uint32_t *spw, const uint4 *t) {
        uint4 L[kSpLetters / 4];
#pragma unroll
        for (int c4 = 0; c4 < kSpLetters / 4; ++c4) L[c4] = t[c4];
#pragma unroll
        for (int c4 = 0; c4 < kSpLetters / 4; ++c4) {
            spw[(4 * c4 + 0) * kWave] = L[c4].x;
            spw[(4 * c4 + 1) * kWave] = L[c4].y;
            spw[(4 * c4 + 2) * kWave] = L[c4].z;
            spw[(4 * c4 + 3) * kWave] = L[c4].w;
        }
    }

    // One subject row: P holds its T values.  First the next row's profile
    // row is put in the buffer (table row `tn`); the row is computed; then P
    // is refilled with the next row's values.  The LDS latencies of the copy
    // and the refill are covered by the SIMD's other wave.
    static __device__ __forceinline__ void row(const LaneFrame &ops, V (&H)[T], V (&E)[T],
                                               uint32_t (&P)[T], const uint4 *tn, uint32_t *spw,
                                               const uint32_t (&addr)[T], const uint8_t *lds8,
                                               uint32_t hb_prev, uint32_t fin, const V *FL,
                                               V (&B)[2], uint32_t &hout, uint32_t &fout) {
        put(spw, tn);
        V f = as_v<V>(fin);
        // The steps in FrameStrip::row's order; a class-0 column's diagonal
        // operand also takes -G alpha before its table value is added.
        V d = (as_v<V>(hb_prev) + ops.ngroup) + as_v<V>(P[0]);
        V tp = d;
#pragma unroll
        for (int j = 0; j < T; ++j) {
            const V h = F::max3(d, E[j], f);
            if (j + 1 < T) d = (((j + 1) & 3) == 0 ? H[j] + ops.ngroup : H[j]) + as_v<V>(P[j + 1]);
            const V t = h + ops.nu;
            if (!(j & 1)) B[(j >> 1) & 1] = F::max3(B[(j >> 1) & 1], h, H[j + 1]);
            if (j > 0) E[j - 1] = F::max3(E[j - 1], tp, FL[(j - 1) & 3]);
            f = __builtin_elementwise_maximum(f, t);
            if ((j & 3) == 3) f += ops.ngroup;
            H[j] = h;
            tp = t;
        }
        E[T - 1] = F::max3(E[T - 1], tp, FL[(T - 1) & 3]);
        hout = as_u(H[T - 1]);
        fout = as_u(f);
#pragma unroll
        for (int j = 0; j < T; ++j) asm volatile("" : "+v"(H[j]), "+v"(E[j]));
        asm volatile("" : "+v"(B[0]), "+v"(B[1]));
#pragma unroll
        for (int j = 0; j < T; ++j) P[j] = *(const uint32_t *)(lds8 + addr[j]);
    }

    // All rows of one group against one strip, as FrameStrip::pass.
    template <bool HAS_IN, bool HAS_OUT>
    static __device__ __forceinline__ void pass(const LaneFrame &ops, V &best_io,
                                                const uint16_t *codes, uint32_t *wsc, int nch,
                                                const uint32_t *lpt, uint32_t *spw,
                                                const uint32_t (&addr)[T], const uint8_t *lds8) {
        constexpr int kPeriodChunks = kFrameRows / kChunk;
        V H[T], E[T];
#pragma unroll
        for (int j = 0; j < T; ++j) {
            H[j] = ops.k((j & 3) - 1);
            E[j] = ops.k(j & 3);
        }
        constexpr int kFloors = kChunk + kFrameCols - 1;
        V FL[kFloors];
#pragma unroll
        for (int x = 0; x < kFloors; ++x) FL[x] = ops.k(x + 1);
        const V chunk_step = ops.k(kChunk);
        V B[2] = {best_io, ops.k(0)};
        V z = ops.k(kFrameCols - 2);
        uint32_t hb_prev = as_u(z);
        const uint32_t f_edge = as_u(ops.nalpha);
        const int last = nch - 1;
        uint2 cd = *(const uint2 *)codes;
        uint2 cd_n = *(const uint2 *)(codes + (size_t)(last < 1 ? last : 1) * 256);
        uint4 b0 = make_uint4(0, 0, 0, 0), b1 = make_uint4(0, 0, 0, 0);
        if (HAS_IN) {
            b0 = ((const uint4 *)wsc)[0];
            b1 = ((const uint4 *)wsc)[1];
        }
        // prologue: row 0's profile row written and read
        put(spw, (const uint4 *)(lpt + (cd.x & 0xffffu) * kSpLetters));
        uint32_t P[T];
#pragma unroll
        for (int j = 0; j < T; ++j) P[j] = *(const uint32_t *)(lds8 + addr[j]);
        for (int c = 0; c < nch; ++c) {
            if (c != 0 && c % kPeriodChunks == 0) {
#pragma unroll
                for (int j = 0; j < T; ++j) { H[j] += ops.rebase; E[j] += ops.rebase; }
#pragma unroll
                for (int x = 0; x < kFloors; ++x) FL[x] += ops.rebase;
                B[0] += ops.rebase;
                B[1] += ops.rebase;
                if (HAS_IN) hb_prev = as_u(as_v<V>(hb_prev) + ops.rebase);
                else z += ops.rebase;
            }
            const int c1 = c + 1 < last ? c + 1 : last;
            const int c2 = c + 2 < last ? c + 2 : last;
            const uint2 cd_nn = *(const uint2 *)(codes + (size_t)c2 * 256);
            uint4 b0n = make_uint4(0, 0, 0, 0), b1n = make_uint4(0, 0, 0, 0);
            if (HAS_IN) {
                b0n = ((const uint4 *)(wsc + (size_t)c1 * 512))[0];
                b1n = ((const uint4 *)(wsc + (size_t)c1 * 512))[1];
            }
            // table rows of rows x + 1: rows 1, 2, 3 of this chunk and row 0 of the next
            const uint32_t tn[4] = {cd.x >> 16, cd.y & 0xffffu, cd.y >> 16, cd_n.x & 0xffffu};
            const uint32_t hb_in[4] = {hb_prev, b0.x, b0.z, b1.x};
            const uint32_t f_in[4] = {b0.y, b0.w, b1.y, b1.w};
            uint32_t o[8];
#pragma unroll
            for (int x = 0; x < kChunk; ++x) {
                const uint32_t hb = HAS_IN ? hb_in[x] : as_u(z), fi = HAS_IN ? f_in[x] : f_edge;
                row(ops, H, E, P, (const uint4 *)(lpt + tn[x] * kSpLetters), spw, addr, lds8, hb, fi,
                    FL + x, B, o[2 * x], o[2 * x + 1]);
                B[0] += ops.palpha;
                B[1] += ops.palpha;
                if (!HAS_IN) z += ops.palpha;
            }
#pragma unroll
            for (int x = 0; x < kFloors; ++x) FL[x] += chunk_step;
            hb_prev = b1.z;
            if (HAS_OUT) {
                uint4 *dst = (uint4 *)(wsc + (size_t)c * 512);
                dst[0] = make_uint4(o[0], o[1], o[2], o[3]);
                dst[1] = make_uint4(o[4], o[5], o[6], o[7]);
            }
            cd = cd_n;
            cd_n = cd_nn;
            b0 = b0n;
            b1 = b1n;
        }
#pragma unroll
        for (int j = 0; j < T; j += 4) {
            B[0] = __builtin_elementwise_maximum(B[0], H[j + 1]);
            B[1] = __builtin_elementwise_maximum(B[1], H[j + 3]);
        }
        best_io = __builtin_elementwise_maximum(B[0] - (FL[0] + ops.nalpha),
                                                B[1] - (FL[0] + ops.palpha));
    }
};

int inter_sp_lds_bytes(int R, int waves) {
    return (R * R * kSpLetters + waves * kSpLetters * kWave) * 4;
}

template <int T, int W>
__global__ void __launch_bounds__(W * 64, 2) inter_sp_kernel(InterArgs a, int magic) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const int R = a.R;
    const int RR = R * R;
    uint32_t *lpt = lds;                                   // RR x kSpLetters
    uint32_t *spbase = lds + RR * kSpLetters;              // W x kSpLetters x 64
    __shared__ int s_item;
    __shared__ int s_q;   // query whose table is in LDS (-1: none)
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    uint32_t *wsc = a.scratch + ((size_t)(blockIdx.x * W + w) * (size_t)a.max_rows) * 128 + lane * 8;
    uint32_t *spw = spbase + (size_t)w * kSpLetters * kWave + lane;
    const uint8_t *lds8 = (const uint8_t *)lds;
    if (threadIdx.x == 0) s_q = -1;

    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        const int last_q = __builtin_amdgcn_readfirstlane(s_q);
        __syncthreads();   // s_item and s_q read by every wave before either changes
        if (it >= a.n_items) break;
        const int q = __builtin_amdgcn_readfirstlane(a.item_q[it]);
        const int alpha = a.qs.gap[2 * q], beta = a.qs.gap[2 * q + 1];
        const LaneFrame ops(min(alpha, 2048), min(beta, 2048));
        const int thr = lane_frame_thr(a.thr, alpha);
        const int A = R - 1;
        const uint8_t *blk = a.qs.qc[q];        // A x A matrix, then the mpad query codes
        const uint8_t *qcodes = blk + A * A;
        if (q != last_q) {
            // every wave has finished its previous item (the loop-top barrier)
            const int8_t *M = (const int8_t *)blk;
            for (int e = threadIdx.x; e < RR * kSpLetters; e += W * 64) {
                const int pair = e / kSpLetters, c = e - pair * kSpLetters;
                const int ra = div_r(pair, magic), rb = pair - ra * R;
                const int va = c < A && ra < A ? M[c * A + ra] : 0;
                const int vb = c < A && rb < A ? M[c * A + rb] : 0;
                lpt[e] = (uint32_t)Lane<TIER_F16X2>::enc(va + ops.bias1) |
                         ((uint32_t)Lane<TIER_F16X2>::enc(vb + ops.bias1) << 16);
            }
            if (threadIdx.x == 0) s_q = q;
            __syncthreads();
        }
        const int g = a.item_g[it] + w;
        const bool active = g < a.n_groups;
        if (active) {
            const int rows = a.grp_rows[g];
            const int mp = a.qs.mpad[q];
            const int nstrips = (mp + T - 1) / T;
            const uint16_t *codes = a.codes + a.grp_base[g] + lane * 4;
            const int nch = rows / kChunk;
            const uint32_t spw_off = (uint32_t)((spw - lds) * 4) - (uint32_t)lane * 4;
            h2 best = Lane<TIER_F16X2>::zero();
            for (int k = 0; k < nstrips; ++k) {
                uint32_t addr[T];
#pragma unroll
                for (int j = 0; j < T; ++j) {
                    const int col = k * T + j;
                    const int letter = col < mp ? qcodes[col] : A;
                    addr[j] = spw_off + (uint32_t)letter * (kWave * 4) + (uint32_t)lane * 4;
                }
                typedef FrameStripSP<T> S;
                if (k == 0) {
                    if (nstrips == 1) S::template pass<false, false>(ops, best, codes, wsc, nch, lpt, spw, addr, lds8);
                    else S::template pass<false, true>(ops, best, codes, wsc, nch, lpt, spw, addr, lds8);
                } else {
                    if (k + 1 == nstrips) S::template pass<true, false>(ops, best, codes, wsc, nch, lpt, spw, addr, lds8);
                    else S::template pass<true, true>(ops, best, codes, wsc, nch, lpt, spw, addr, lds8);
                }
            }
            const int ids[2] = {a.grp_ids[g * kGroup + lane], a.grp_ids[g * kGroup + kWave + lane]};
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                const int id = ids[half];
                if (id < 0) continue;
                bool flag;
                const int v = Lane<TIER_F16X2>::value(best, half, thr, &flag);
                a.scores[(size_t)q * a.n_seqs + id] = v;
                if (flag) {
                    const int pos = atomicAdd(a.ovf_count, 1);
                    if (pos < a.ovf_cap) {
                        a.ovf_q[pos] = q;
                        a.ovf_id[pos] = id;
                    }
                }
            }
        }
    }
}

int inter_sp_max_grid(int R, int waves) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    }
    int per_cu = 0;
    if (waves == 4 &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, inter_sp_kernel<32, 4>, 4 * 64,
                                                     inter_sp_lds_bytes(R, 4)) != hipSuccess)
        per_cu = 0;
    if (per_cu < 1) per_cu = 1;
    return per_cu * cus;
}

hipError_t launch_inter_sp(const InterArgs &a, int strip, int waves, int grid, hipStream_t st) {
    if (strip != 32 || waves != 4 || a.R - 1 >= kSpLetters) return hipErrorInvalidValue;
    const int magic = (65536 + a.R - 1) / a.R;
    hipLaunchKernelGGL((inter_sp_kernel<32, 4>), dim3(grid), dim3(4 * 64), inter_sp_lds_bytes(a.R, 4),
                       st, a, magic);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Wave-per-pair kernel (int32, exact).
// ---------------------------------------------------------------------------
// DPP wave shifts: lane i takes lane i-1 (shr) or i+1 (shl); the lane with no
// source keeps `old`.
__device__ __forceinline__ int shr1(int old, int src) {
    return __builtin_amdgcn_update_dpp(old, src, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int shl1(int old, int src) {
    return __builtin_amdgcn_update_dpp(old, src, 0x130, 0xf, 0xf, false);
}

// Per-wave LDS ring of the wave-per-pair kernels, 638 words after the
// profile.  Entry x (0 <= x < 128) of the residue-code arrays A and B covers
// row 64(b - 1) + x during block b of 64 steps; the lane-0 feeds H and F keep
// only the current block (entries 64..127); the output arrays OH and OF take
// entries 1..127.  Reads of entries that an array does not keep land, in
// bounds, on another array and only feed lanes whose value is discarded.
// (The int32 kernel, one subject per wave, leaves B unused.)
constexpr int kRingA = 0, kRingB = 128, kRingH = 192, kRingF = 256, kRingOH = 383, kRingOF = 510;
constexpr int kRing2Bytes = 638 * 4;

int wpp_lds_bytes(int R, int T, int waves) { return intra_lds_bytes(R, T) + waves * kRing2Bytes; }

template <int T>
__device__ __forceinline__ void intra_row(int (&H)[T], int (&E)[T], const uint2 *pr, int hb_prev,
                                          int fin, int alpha, int beta, int &best, int &hout,
                                          int &fout) {
    int hdiag = hb_prev, f = fin;
#pragma unroll
    for (int j4 = 0; j4 < T / 4; ++j4) {
        const uint2 p = pr[j4];
        const uint32_t pv[2] = {p.x, p.y};
#pragma unroll
        for (int u = 0; u < 4; u += 2) {
            const int j = j4 * 4 + u;
            const uint32_t wd = pv[u >> 1];
            int h0, h1;
            {
                const int hold = H[j];
                h0 = __builtin_elementwise_max(
                    __builtin_elementwise_max(hdiag + (int)(short)(wd & 0xffffu), E[j]), f);
                const int t = h0 - beta;
                E[j] = __builtin_elementwise_max(__builtin_elementwise_max(E[j] - alpha, t), 0);
                f = __builtin_elementwise_max(__builtin_elementwise_max(f - alpha, t), 0);
                H[j] = h0;
                hdiag = hold;
            }
            {
                const int hold = H[j + 1];
                h1 = __builtin_elementwise_max(
                    __builtin_elementwise_max(hdiag + (int)(short)(wd >> 16), E[j + 1]), f);
                const int t = h1 - beta;
                E[j + 1] = __builtin_elementwise_max(__builtin_elementwise_max(E[j + 1] - alpha, t), 0);
                f = __builtin_elementwise_max(__builtin_elementwise_max(f - alpha, t), 0);
                H[j + 1] = h1;
                hdiag = hold;
            }
            best = __builtin_elementwise_max(__builtin_elementwise_max(best, h0), h1);
        }
    }
    hout = H[T - 1];
    fout = f;
}

// One query against one subject per wave (id < 0: none): the W waves of the
// workgroup share the query's profile (built per pass in `lds`).  Every wave
// reaches every barrier (waves without a subject skip the rows); q must be
// the same for the whole workgroup.
template <int T, int W>
__device__ __forceinline__ void intra_pair(const IntraArgs &a, int q, int id, uint32_t *lds,
                                           int32_t *wsc) {
    constexpr int PW = 64 * T;          // query columns per pass
    constexpr int RS = PW + 8;          // int16 per profile row (padded)
    int16_t *prof = (int16_t *)lds;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    uint32_t *ring = lds + (a.R * RS * 2 + w * kRing2Bytes) / 4;   // after the profile
    const int pad = a.R - 1;
    const int64_t n64 = id >= 0 ? a.off[id + 1] - a.off[id] : 0;
    const int n = (int)n64;
    const uint8_t *s = id >= 0 ? a.res + a.off[id] : a.res;
    const int mp = a.qs.mpad[q];
    const int npass = (a.qs.qlen[q] + PW - 1) / PW;
    const int alpha = a.qs.gap[2 * q], beta = a.qs.gap[2 * q + 1];
    const int8_t *qp = a.qs.qp[q];
    int best = 0;

    for (int p = 0; p < npass; ++p) {
        __syncthreads();
        for (int e = threadIdx.x; e < a.R * PW; e += W * 64) {
            const int r = e / PW, c = e - r * PW;
            const int col = p * PW + c;
            prof[r * RS + c] = col < mp ? (int16_t)qp[(size_t)r * mp + col] : (int16_t)0;
        }
        __syncthreads();
        if (n <= 0) continue;

        const bool has_in = p > 0, has_out = p + 1 < npass;
        const int nblk = (n + 63) / 64;
        // with outputs, the last block's read-back needs step 64 * nblk + 63
        const int steps = has_out ? nblk * 64 + 64 : n + 63;
        int H[T], E[T];
#pragma unroll
        for (int j = 0; j < T; ++j) { H[j] = 0; E[j] = 0; }
        int hb_prev = 0, hout = 0, fout = 0;
        // Lane l fills entry 64 + l of the ring's A, H and F with row 64b + l
        // of block b (A: residue code, H and F: the previous pass's last
        // column, 0 on the first pass).  At step 64b + u lane l reads entry
        // 64 + u - l; every lane writes its outputs to that entry of OH and
        // OF, and entry u + 1 ends the block holding lane 63's.
        auto feed = [&](int row, uint32_t &fa, uint32_t &fh, uint32_t &ff) {
            fa = row < n ? s[row] : pad;
            fh = (has_in && row < n) ? (uint32_t)wsc[2 * row] : 0u;
            ff = (has_in && row < n) ? (uint32_t)wsc[2 * row + 1] : 0u;
        };
        uint32_t cA, cHf, cFf, nA, nH, nF;
        feed(lane, cA, cHf, cFf);   // only until they are in the ring
        feed(64 + lane, nA, nH, nF);
        ring[kRingA + lane] = pad;
        ring[kRingA + 64 + lane] = cA;
        ring[kRingH + 64 + lane] = cHf;
        ring[kRingF + 64 + lane] = cFf;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint32_t *rl = ring + 64 - lane;
        for (int tb = 0; tb < steps; tb += 64) {
            if (tb > 0) {
                // block tb/64 - 1 moves down, block tb/64 comes in
                ring[kRingA + lane] = cA;
                ring[kRingA + 64 + lane] = nA;
                ring[kRingH + 64 + lane] = nH;
                ring[kRingF + 64 + lane] = nF;
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                cA = nA;
                feed(tb + 64 + lane, nA, nH, nF);
            }
            const int ue = __builtin_amdgcn_readfirstlane(steps - tb < 64 ? steps - tb : 64);
            for (int u = 0; u < ue; ++u) {
                uint32_t *e = rl + u;
                const int hin = shr1((int)e[kRingH], hout);
                const int fin = shr1((int)e[kRingF], fout);
                // residue codes are below 2^24, so the 24-bit multiply is exact
                const uint2 *pr = (const uint2 *)(prof + (__umul24(e[kRingA], RS) + lane * T));
                intra_row<T>(H, E, pr, hb_prev, fin, alpha, beta, best, hout, fout);
                hb_prev = hin;
                if (has_out) {
                    e[kRingOH] = (uint32_t)hout;
                    e[kRingOF] = (uint32_t)fout;
                }
            }
            if (has_out) {
                // the block's last step t = tb + 63 has passed; entries 1..64
                // hold lane 63's rows t - 126 .. t - 63 (steps with outputs run
                // whole blocks)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const int row = tb + 63 - 126 + lane;
                const uint32_t oh = ring[kRingOH + 1 + lane], of = ring[kRingOF + 1 + lane];
                if (row >= 0 && row < n) {
                    wsc[2 * row] = (int)oh;
                    wsc[2 * row + 1] = (int)of;
                }
            }
        }
    }
    if (id >= 0) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o, 64));
        if (lane == 0) a.scores[(size_t)q * a.n_seqs + id] = best;
    }
}

// One wave-per-pair item: one subject per wave, all against the item's query.
template <int T, int W>
__device__ __forceinline__ void intra_item(const IntraArgs &a, int it, uint32_t *lds,
                                           int32_t *wsc) {
    const int w = threadIdx.x >> 6;
    intra_pair<T, W>(a, a.item_q[it], a.item_ids[(size_t)it * W + w], lds, wsc);
}

template <int T, int W>
__global__ void __launch_bounds__(W * 64) intra_kernel(IntraArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ int s_item;
    const int w = threadIdx.x >> 6;
    int32_t *wsc = a.pass_scratch + (size_t)(blockIdx.x * W + w) * (size_t)a.max_len_pad * 2;
    const int n_items = a.n_items_dev ? *a.n_items_dev : a.n_items;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= n_items) break;
        // one wave per workgroup (the recompute list): skip entries the packed
        // kernel has already recomputed (id -1) without building a profile
        if (W == 1 && a.item_ids[it] < 0) continue;
        intra_item<T, W>(a, it, lds, wsc);   // its first barrier orders the read of s_item
    }
}

int intra_lds_bytes(int R, int T) { return R * (64 * T + 8) * 2; }

// ---------------------------------------------------------------------------
// Packed-fp16 wave-per-pair kernel: the systolic schedule above with one
// subject in each 16-bit half of every lane (same query), so one instruction
// advances two alignments.  The two halves read their substitution scores from
// two profile rows; one v_perm per column pair packs them.
//
// It evaluates the frame form of the lane-per-subject fp16 tier (LaneFrame).
// Lane l works on subject row t - l at step t, so the offset of that row is
// taken as alpha * ((t mod kFrameRows) - l): it grows by alpha per step, so E
// needs no decay, it is the same for every lane that handles the row (H and F
// cross to lane l+1 one step later), and it drops by kFrameRows * alpha for
// every lane at once at the end of each block of kFrameRows steps, outputs
// included.  A lane's T columns start on a multiple of kFrameCols, so column
// j of the lane adds alpha * (j mod kFrameCols) as in FrameStrip: F decays
// once per group of columns (its hand-off to lane l+1 is in class 0), the E
// floors and the two running bests are per class, and the profile carries
// the diagonal's offset change per column class.  Offsets span
// [-63 alpha, 35 alpha]; for alpha <= kFrameMaxAlpha every value that can
// matter stays an exact fp16 integer with thr = 1920 - 36 alpha, and a value
// below -2048 rounds to one that is still below the frame's zero.  Larger
// alpha flags every half for the exact recompute.  Pass boundaries are stored
// as true values and converted on the way in and out.
//
// What enters at lane 0 (and the residue codes every lane needs) comes from a
// per-wave LDS ring, filled once per 64 rows: at step t lane l reads entry
// t - l, so no register shifts feeder values along the wave each step.  The
// last lane's outputs go through the same ring, read back once per 64 rows.
// ---------------------------------------------------------------------------
// Steps of the packed kernel run in groups of G2 steps; row X of a group
// takes, in column class c, the floor FW[X + c].  The loads of a group's steps
// are issued together, so a group pays the two dependent LDS round trips
// (ring, then profile rows) once.  The kernel at 4 columns per lane, whose
// steps are short and which often runs one wave per SIMD (small databases),
// takes groups of 8, halving that exposed latency per step; elsewhere groups
// of 4 keep the registers within the occupancy the kernel is built for.
template <int T, int X, int G2>
__device__ __forceinline__ void intra2_row(h2 (&H)[T], h2 (&E)[T], const uint2 *pa,
                                           const uint2 *pb, const LaneFrame &ops, h2 hdiag, h2 f,
                                           const h2 (&FW)[kFrameCols + G2 - 1], h2 (&B)[2],
                                           h2 &hout, h2 &fout) {
    static_assert(kFrameCols == 4 && T % kFrameCols == 0, "a lane holds whole column groups");
    // (low half from subject a's row, high half from subject b's row)
    uint32_t sv[T];
#pragma unroll
    for (int j4 = 0; j4 < T / 4; ++j4) {
        const uint2 A = pa[j4], Bv = pb[j4];
        sv[4 * j4 + 0] = __builtin_amdgcn_perm(Bv.x, A.x, 0x05040100u);
        sv[4 * j4 + 1] = __builtin_amdgcn_perm(Bv.x, A.x, 0x07060302u);
        sv[4 * j4 + 2] = __builtin_amdgcn_perm(Bv.y, A.y, 0x05040100u);
        sv[4 * j4 + 3] = __builtin_amdgcn_perm(Bv.y, A.y, 0x07060302u);
    }
    // The diagonal operand of column j+1 is taken from H[j] before H[j] is
    // overwritten, so each new H goes into the register of the old one.  The
    // steps are ordered as in FrameStrip::row, with independent work between
    // each column's dependent packed steps h -> t -> f.
    h2 d = hdiag + as_v<h2>(sv[0]);
    h2 tp = d;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        const h2 h = FrameStrip<4>::max3(d, E[j], f);
        if (j + 1 < T) d = H[j] + as_v<h2>(sv[j + 1]);
        const h2 t = h + ops.nu;
        // (r, j) and (r - 1, j + 1) share an offset for even j; H[j + 1]
        // still holds row r - 1
        if (!(j & 1)) B[(j & 2) >> 1] = FrameStrip<4>::max3(B[(j & 2) >> 1], h, H[j + 1]);
        if (j > 0) E[j - 1] = FrameStrip<4>::max3(E[j - 1], tp, FW[X + ((j - 1) & 3)]);
        f = __builtin_elementwise_maximum(f, t);
        if ((j & 3) == 3) f += ops.ngroup;
        H[j] = h;
        tp = t;
    }
    E[T - 1] = FrameStrip<4>::max3(E[T - 1], tp, FW[X + ((T - 1) & 3)]);
    hout = H[T - 1];
    fout = f;
}


template <int T, bool HAS_IN, bool HAS_OUT, int G2 = 4>
__device__ __forceinline__ void intra2_pass(const IntraArgs &a, const LaneFrame &ops,
                                            const uint16_t *prof, int RS, int32_t *wsc,
                                            uint32_t *ring, const uint8_t *sa, const uint8_t *sb,
                                            int na, int nb, int pad, h2 &best_io) {
    const int lane = threadIdx.x & 63;
    const int n = __builtin_amdgcn_readfirstlane(na > nb ? na : nb);
    const int nblk = (n + 63) / 64;
    // with outputs, the last block's collection needs step 64 * nblk + 63;
    // steps run in whole groups (past the last row every lane reads pad
    // rows, whose zero scores raise no best)
    constexpr int kGrp2 = G2;
    const int steps = HAS_OUT ? nblk * 64 + 64 : (n + 63 + kGrp2 - 1) / kGrp2 * kGrp2;
    const h2 pa2 = ops.palpha, pag = ops.k(kGrp2);
    const float alpha = (float)ops.alpha;
    constexpr int G = kFrameCols;
    // Offset of this lane at step 0, and the per-lane conversions of the
    // lane-0 feeds (row consumed at step row: alpha * (row mod 32); H comes
    // from the previous pass's last column, class G - 1) and of the collected
    // last-lane outputs (lane l stores the row lane 63 produced at a step
    // congruent to l mod 64, at offset alpha * ((l mod 32) - 63)).
    const _Float16 o0 = (_Float16)(-alpha * lane);
    const _Float16 fc = (_Float16)(alpha * (lane & (kFrameRows - 1)));
    const _Float16 fch = (_Float16)(alpha * ((lane & (kFrameRows - 1)) + G - 1));
    const _Float16 wc = (_Float16)(alpha * ((lane & (kFrameRows - 1)) - 63));
    const _Float16 wch = (_Float16)(alpha * ((lane & (kFrameRows - 1)) - 63 + G - 1));
    const h2 off0 = h2{o0, o0}, fconv = h2{fc, fc}, fconv_h = h2{fch, fch};
    const h2 wconv = h2{wc, wc}, wconv_h = h2{wch, wch};
    h2 H[T], E[T];
#pragma unroll
    for (int j = 0; j < T; ++j) {
        H[j] = off0 + ops.k((j & 3) - 1);
        E[j] = off0 + ops.k(j & 3);
    }
    // E floors (true 0) of the steps of a group: step x of the group, class
    // c, is at FW[x + c]; the window moves by kGrp2 * alpha per group
    h2 FW[G + kGrp2 - 1];
#pragma unroll
    for (int i = 0; i < G + kGrp2 - 1; ++i) FW[i] = off0 + ops.k(i + 1);
    h2 B[2] = {best_io + off0, off0 + ops.k(2)};
    h2 hb_prev = off0 + ops.k(G - 2);
    // outputs handed to lane l+1 before step 0 stand for step -1 of lane l:
    // true 0 at offset -alpha * (l + 1), plus the class offset of H's column
    h2 hout = off0 + ops.k(G - 2), fout = off0 + ops.nalpha;
    // Lane l fills entry 64 + l of each ring array with row 64b + l of block
    // b.  At step 64b + u lane l reads entry 64 + u - l: its own row's
    // residue codes and, for lane 0, the H and F that enter the pass at row
    // 64b + u.  Every lane writes its outputs of that step to the same entry
    // of OH and OF; entry u + 1 is lane 63's, and no later write of the block
    // reaches it (lane l writes it at step u + 1 - 64 + l).
    auto feed = [&](int row, uint32_t &fa, uint32_t &fb, uint32_t &fh, uint32_t &ff) {
        fa = row < na ? sa[row] : pad;
        fb = row < nb ? sb[row] : pad;
        h2 vh = fconv_h, vf = fconv;
        if (HAS_IN && row < n) {
            vh += as_v<h2>((uint32_t)wsc[2 * row]);
            vf += as_v<h2>((uint32_t)wsc[2 * row + 1]);
        }
        fh = as_u(vh);
        ff = as_u(vf);
    };
    uint32_t cA, cB, cHf, cFf, nA, nB, nH, nF;
    feed(lane, cA, cB, cHf, cFf);
    feed(64 + lane, nA, nB, nH, nF);
    ring[kRingA + lane] = pad;
    ring[kRingB + lane] = pad;
    ring[kRingA + 64 + lane] = cA;
    ring[kRingB + 64 + lane] = cB;
    ring[kRingH + 64 + lane] = cHf;
    ring[kRingF + 64 + lane] = cFf;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t *rl = ring + 64 - lane;
    for (int tb = 0; tb < steps; tb += kFrameRows) {
        if (tb > 0 && (tb & 63) == 0) {
            // block tb/64 - 1 moves down, block tb/64 comes in
            ring[kRingA + lane] = cA;
            ring[kRingB + lane] = cB;
            ring[kRingA + 64 + lane] = nA;
            ring[kRingB + 64 + lane] = nB;
            ring[kRingH + 64 + lane] = nH;
            ring[kRingF + 64 + lane] = nF;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            cA = nA;
            cB = nB;
            feed(tb + 64 + lane, nA, nB, nH, nF);
        }
        const int ue =
            __builtin_amdgcn_readfirstlane(steps - tb < kFrameRows ? steps - tb : kFrameRows);
        uint32_t *rb0 = rl + (tb & 63);
        for (int u = 0; u < ue; u += kGrp2) {
#pragma unroll
            for (int x = 0; x < kGrp2; ++x) {
                uint32_t *e = rb0 + u + x;
                const h2 hin = as_v<h2>((uint32_t)shr1((int)e[kRingH], (int)as_u(hout)));
                const h2 fin = as_v<h2>((uint32_t)shr1((int)e[kRingF], (int)as_u(fout)));
                // residue codes are below 2^24, so the 24-bit multiply is exact
                const uint2 *pa = (const uint2 *)(prof + (__umul24(e[kRingA], RS) + lane * T));
                const uint2 *pb = (const uint2 *)(prof + (__umul24(e[kRingB], RS) + lane * T));
                switch (x) {
                case 0: intra2_row<T, 0, kGrp2>(H, E, pa, pb, ops, hb_prev, fin, FW, B, hout, fout); break;
                case 1: intra2_row<T, 1 % kGrp2, kGrp2>(H, E, pa, pb, ops, hb_prev, fin, FW, B, hout, fout); break;
                case 2: intra2_row<T, 2 % kGrp2, kGrp2>(H, E, pa, pb, ops, hb_prev, fin, FW, B, hout, fout); break;
                case 3: intra2_row<T, 3 % kGrp2, kGrp2>(H, E, pa, pb, ops, hb_prev, fin, FW, B, hout, fout); break;
                case 4: intra2_row<T, 4 % kGrp2, kGrp2>(H, E, pa, pb, ops, hb_prev, fin, FW, B, hout, fout); break;
                case 5: intra2_row<T, 5 % kGrp2, kGrp2>(H, E, pa, pb, ops, hb_prev, fin, FW, B, hout, fout); break;
                case 6: intra2_row<T, 6 % kGrp2, kGrp2>(H, E, pa, pb, ops, hb_prev, fin, FW, B, hout, fout); break;
                default: intra2_row<T, 7 % kGrp2, kGrp2>(H, E, pa, pb, ops, hb_prev, fin, FW, B, hout, fout); break;
                }
                hb_prev = hin;
                B[0] += pa2;
                B[1] += pa2;
                if (HAS_OUT) {
                    e[kRingOH] = as_u(hout);
                    e[kRingOF] = as_u(fout);
                }
            }
#pragma unroll
            for (int i = 0; i < G + kGrp2 - 1; ++i) FW[i] += pag;
        }
        if (HAS_OUT && (tb & 63) == 32) {
            // the block's last step t = tb + 31 has passed; entries 1..64 hold
            // lane 63's rows t - 126 .. t - 63 (steps with outputs run whole
            // blocks of 64)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int row = tb + 31 - 126 + lane;
            const uint32_t oh = ring[kRingOH + 1 + lane], of = ring[kRingOF + 1 + lane];
            if (row >= 0 && row < n) {
                wsc[2 * row] = (int)as_u(as_v<h2>(oh) - wconv_h);
                wsc[2 * row + 1] = (int)as_u(as_v<h2>(of) - wconv);
            }
        }
        if (ue == kFrameRows) {
#pragma unroll
            for (int j = 0; j < T; ++j) {
                H[j] += ops.rebase;
                E[j] += ops.rebase;
            }
#pragma unroll
            for (int i = 0; i < G + kGrp2 - 1; ++i) FW[i] += ops.rebase;
            B[0] += ops.rebase;
            B[1] += ops.rebase;
            hb_prev += ops.rebase;
            hout += ops.rebase;
            fout += ops.rebase;
        }
    }
    // The last step's odd columns (classes 1 and 3), at the offsets of B[0]
    // and B[1] after that step.
#pragma unroll
    for (int j = 0; j < T; j += 4) {
        B[0] = __builtin_elementwise_maximum(B[0], H[j + 1]);
        B[1] = __builtin_elementwise_maximum(B[1], H[j + 3]);
    }
    // B[0] is at the offset of step `steps`, B[1] two alpha above it
    const _Float16 oe = (_Float16)(alpha * ((steps & (kFrameRows - 1)) - lane));
    const h2 oe2 = h2{oe, oe};
    best_io = __builtin_elementwise_maximum(B[0] - oe2, B[1] - (oe2 + ops.k(2)));
}

// At T = 16 the protein-sized profile already holds a CU to three of these
// workgroups, so the kernel may use the registers of three waves per SIMD; at
// T = 4 its groups of 8 steps need them (see intra2_row).
template <int T, int W>
__global__ void __launch_bounds__(W * 64, T == 8 ? 4 : 3) intra2_kernel(IntraArgs a) {
    typedef Lane<TIER_F16X2> L;
    constexpr int PW = 64 * T;          // query columns per pass
    constexpr int RS = PW + 8;          // fp16 entries per profile row (padded)
    constexpr int kG2 = T == 4 ? 8 : 4; // steps per group of the T-wide passes
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    uint16_t *prof = (uint16_t *)lds;
    __shared__ int s_item, s_nflag;
    __shared__ int s_flag[2 * W];

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int pad = a.R - 1;
    int32_t *wsc = a.pass_scratch + (size_t)(blockIdx.x * W + w) * (size_t)a.max_len_pad * 2;
    uint32_t *ring = lds + (a.R * (PW + 8) * 2 + w * kRing2Bytes) / 4;   // after the profile
    const int n_items = a.n_items_dev ? *a.n_items_dev : a.n_items;

    for (;;) {
        if (threadIdx.x == 0) {
            s_item = atomicAdd(a.counter, 1);
            s_nflag = 0;
        }
        __syncthreads();
        const int it = s_item;
        if (it >= n_items) break;
        const int q = a.item_q[it];
        const int id_a = a.item_ids[(size_t)it * 2 * W + 2 * w];
        const int id_b = a.item_ids[(size_t)it * 2 * W + 2 * w + 1];
        const int na = id_a >= 0 ? (int)(a.off[id_a + 1] - a.off[id_a]) : 0;
        const int nb = id_b >= 0 ? (int)(a.off[id_b + 1] - a.off[id_b]) : 0;
        const int n = na > nb ? na : nb;
        const uint8_t *sa = id_a >= 0 ? a.res + a.off[id_a] : a.res;
        const uint8_t *sb = id_b >= 0 ? a.res + a.off[id_b] : a.res;
        const int mp = a.qs.mpad[q];
        const int qlen = a.qs.qlen[q];
        const int npass = (qlen + PW - 1) / PW;
        // The last pass takes the fewest columns per lane that hold its
        // columns: every step costs all of a lane's columns, used or not.
        const int rem = qlen - (npass - 1) * PW;
        const int tl = T == 16 ? (rem <= 256 ? 4 : rem <= 512 ? 8 : rem <= 768 ? 12 : 16) : T;
        const int8_t *qp = a.qs.qp[q];
        const int alpha = a.qs.gap[2 * q];
        const LaneFrame ops(min(alpha, kFrameMaxAlpha), a.qs.gap[2 * q + 1]);
        const int thr = alpha > kFrameMaxAlpha ? 0 : lane_frame_thr(a.thr, alpha);
        h2 best = L::zero();

        for (int p = 0; p < npass; ++p) {
            const bool last = p + 1 == npass;
            const int pw = 64 * (last ? tl : T), rs = pw + 8;   // this pass's width and row stride
            __syncthreads();
            for (int e = threadIdx.x; e < a.R * pw; e += W * 64) {
                const int r = e / pw, c = e - r * pw;
                const int col = p * PW + c;
                const int bias = col % kFrameCols == 0 ? ops.bias0 : ops.bias1;
                prof[r * rs + c] = L::enc((col < mp ? (int)qp[(size_t)r * mp + col] : 0) + bias);
            }
            __syncthreads();
            if (n <= 0) continue;
            const bool has_in = p > 0, has_out = !last;
            if constexpr (T == 16) {
                if (last && tl == 4) {
                    if (has_in) intra2_pass<4, true, false>(a, ops, prof, rs, wsc, ring, sa, sb, na, nb, pad, best);
                    else intra2_pass<4, false, false>(a, ops, prof, rs, wsc, ring, sa, sb, na, nb, pad, best);
                    continue;
                }
                if (last && tl == 8) {
                    if (has_in) intra2_pass<8, true, false>(a, ops, prof, rs, wsc, ring, sa, sb, na, nb, pad, best);
                    else intra2_pass<8, false, false>(a, ops, prof, rs, wsc, ring, sa, sb, na, nb, pad, best);
                    continue;
                }
                if (last && tl == 12) {
                    if (has_in) intra2_pass<12, true, false>(a, ops, prof, rs, wsc, ring, sa, sb, na, nb, pad, best);
                    else intra2_pass<12, false, false>(a, ops, prof, rs, wsc, ring, sa, sb, na, nb, pad, best);
                    continue;
                }
            }
            if (has_in) {
                if (has_out) intra2_pass<T, true, true, kG2>(a, ops, prof, RS, wsc, ring, sa, sb, na, nb, pad, best);
                else intra2_pass<T, true, false, kG2>(a, ops, prof, RS, wsc, ring, sa, sb, na, nb, pad, best);
            } else {
                if (has_out) intra2_pass<T, false, true, kG2>(a, ops, prof, RS, wsc, ring, sa, sb, na, nb, pad, best);
                else intra2_pass<T, false, false, kG2>(a, ops, prof, RS, wsc, ring, sa, sb, na, nb, pad, best);
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const h2 other = as_v<h2>((uint32_t)__shfl_xor((int)as_u(best), o, 64));
            best = __builtin_elementwise_maximum(best, other);
        }
        // A flagged half is recomputed exactly (int32) by this workgroup at
        // once, one subject per wave, while the other workgroups go on with
        // the queue; it is still counted in the recompute list, with id -1
        // so that the recompute launch after this one skips it.
        if (lane == 0) {
            const int ids[2] = {id_a, id_b};
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                if (ids[half] < 0) continue;
                bool flag;
                const int v = L::value(best, half, thr, &flag);
                if (!flag) {
                    a.scores[(size_t)q * a.n_seqs + ids[half]] = v;
                    continue;
                }
                s_flag[atomicAdd(&s_nflag, 1)] = ids[half];
                const int pos = atomicAdd(a.ovf_count, 1);
                if (pos < a.ovf_cap) {
                    a.ovf_q[pos] = q;
                    a.ovf_id[pos] = -1;
                }
            }
        }
        __syncthreads();
        const int nflag = s_nflag;      // the same in every wave: the loop below meets
        for (int b = 0; b < nflag; b += W)   // the same barriers in all of them
            intra_pair<T, W>(a, q, b + w < nflag ? s_flag[b + w] : -1, lds, wsc);
        // every wave has read s_nflag and s_flag before thread 0 resets the
        // count for the next item
        __syncthreads();
    }
}

template <int T, int W>
static hipError_t launch_intra2_t(const IntraArgs &a, int grid, hipStream_t st) {
    const int lds = wpp_lds_bytes(a.R, T, W);
    hipLaunchKernelGGL((intra2_kernel<T, W>), dim3(grid), dim3(W * 64), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_intra2(const IntraArgs &a, int T, int waves, int grid, hipStream_t st) {
    if (waves != 4) return hipErrorInvalidValue;
    if (T == 4) return launch_intra2_t<4, 4>(a, grid, st);
    if (T == 8) return launch_intra2_t<8, 4>(a, grid, st);
    if (T == 16) return launch_intra2_t<16, 4>(a, grid, st);
    return hipErrorInvalidValue;
}

template <int T, int W>
static hipError_t launch_intra_t(const IntraArgs &a, int grid, hipStream_t st) {
    const int lds = wpp_lds_bytes(a.R, T, W);
    hipLaunchKernelGGL((intra_kernel<T, W>), dim3(grid), dim3(W * 64), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_intra(const IntraArgs &a, int T, int waves, int grid, hipStream_t st) {
#define SWMI_INTRA_CASE(T_, W_) \
    if (T == T_ && waves == W_) return launch_intra_t<T_, W_>(a, grid, st);
    SWMI_INTRA_CASE(4, 1) SWMI_INTRA_CASE(8, 1) SWMI_INTRA_CASE(16, 1)
    SWMI_INTRA_CASE(4, 4) SWMI_INTRA_CASE(8, 4) SWMI_INTRA_CASE(16, 4)
#undef SWMI_INTRA_CASE
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Utilities and top-k (stage iv: scores in descending order; equal scores by
// ascending database index).  Exact radix select over the 32-bit scores in
// four 8-bit passes, then an ordered gather of the ties at the threshold.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Alignment with traceback (the conclusion leaves alignment reconstruction to
// future work).  Scores are Eq. 1's; among equal-scoring alignments:
//   - the alignment ends at the first cell, subject row then query column,
//     whose H equals the score;
//   - walking back, H comes from the diagonal before E before F, and E and F
//     from the gap opening (H - beta) before the extension;
//   - it starts at the first diagonal step whose predecessor H is 0 (or on the
//     boundary).
// Forward pass: the systolic wave-per-pair schedule of intra_item, in int32
// on the recurrence as written (E and F start at 0 and are not floored, so
// every tie is decided on exact values), storing one direction byte per cell:
// bits 0-1 the source of H (0 diagonal, 1 E, 2 F), bit 2 H == 0, bit 3 E
// opened, bit 4 F opened.  A lane hands H and F of its last column to the
// lane on its right, which computes F of its first column (and that cell's
// bit) itself.  A lane's T columns (4, 8 or 16, by query length) are T bytes
// of a row whose stride is qlen rounded up to 16, so each step stores one
// aligned T-byte vector.  Each lane keeps its first strict maximum (within a
// pass rows and columns come in order; across passes a tie keeps the smaller
// row); the wave reduces by (score desc, row asc, column asc).
// Traceback: one thread per pair walks back from the end cell, every read
// bounds-checked.
// ---------------------------------------------------------------------------
// One subject row of a lane's T columns in the forward pass.  FILL: a step
// in which lanes before row 0 keep the zero boundary (the first 63).  Each
// lane keeps the first strict maximum of the pass in its own (row, column)
// order, as (step, column); cells outside the subject or the query score 0 on
// their diagonal and gap moves only lower a value, so none of them exceeds
// the value of a real cell that precedes it.
// The lane's T scores of one profile row, int16 or int8, read as whole
// 4-, 8- or 16-byte LDS words.
template <int T, typename S>
__device__ __forceinline__ void load_scores(const S *pr, uint32_t (&pw)[T * sizeof(S) / 4]) {
    constexpr int NW = T * (int)sizeof(S) / 4;
    if constexpr (NW >= 4) {
#pragma unroll
        for (int k = 0; k < NW / 4; ++k) {
            const uint4 v = ((const uint4 *)pr)[k];
            pw[4 * k] = v.x;
            pw[4 * k + 1] = v.y;
            pw[4 * k + 2] = v.z;
            pw[4 * k + 3] = v.w;
        }
    } else if constexpr (NW == 2) {
        const uint2 v = *(const uint2 *)pr;
        pw[0] = v.x;
        pw[1] = v.y;
    } else {
        pw[0] = *(const uint32_t *)pr;
    }
}

template <int T, typename S>
__device__ __forceinline__ int score_at(const uint32_t (&pw)[T * sizeof(S) / 4], int j) {
    // sign extension folds into SDWA operands of the add that uses it
    if constexpr (sizeof(S) == 2)
        return (j & 1) ? ((int)pw[j >> 1] >> 16) : (int)(int16_t)(pw[j >> 1] & 0xffffu);
    else
        return (int)(int8_t)((pw[j >> 2] >> (8 * (j & 3))) & 0xffu);
}

template <int T, bool FILL, typename S>
__device__ __forceinline__ void align_row(const AlignArgs &a, int (&H)[T], int (&E)[T],
                                          const S *pr, int t, int i, int hdiag, int hleft,
                                          int fprev, int &pbest, int &pt, int &pj, uint32_t (&cw)[T / 4],
                                          int &hout, int &fout) {
    static_assert(T % 4 == 0, "a lane stores whole 32-bit direction words");
    uint32_t pw[T * sizeof(S) / 4];
    load_scores<T, S>(pr, pw);
    const bool real_row = i >= 0;
#pragma unroll
    for (int k = 0; k < T / 4; ++k) cw[k] = 0;
#pragma unroll
    for (int j = 0; j < T; ++j) {
        const int sc = score_at<T, S>(pw, j);
        const int hup = H[j];
        const int e_ext = E[j] - a.alpha, e_open = hup - a.beta;
        const int e = max(e_ext, e_open);
        const int f_ext = fprev - a.alpha, f_open = hleft - a.beta;
        const int fv = max(f_ext, f_open);
        const int d = hdiag + sc;
        const int h = max(max(0, d), max(e, fv));
        uint32_t code = h == 0 ? 4u : (h == d ? 0u : (h == e ? 1u : 2u));
        code |= (e_open >= e_ext ? 8u : 0u) | (f_open >= f_ext ? 16u : 0u);
        cw[j >> 2] |= code << (8 * (j & 3));
        const bool gt = h > pbest;
        pbest = gt ? h : pbest;
        pt = gt ? t : pt;
        pj = gt ? j : pj;
        hdiag = hup;
        if (FILL) {
            H[j] = real_row ? h : 0;
            E[j] = real_row ? e : 0;
            fprev = real_row ? fv : 0;
        } else {
            H[j] = h;
            E[j] = e;
            fprev = fv;
        }
        hleft = H[j];
    }
    hout = H[T - 1];
    fout = fprev;
}

template <int T, int W>
__global__ void __launch_bounds__(W * 64) align_fwd_kernel(AlignArgs a) {
    constexpr int PW = 64 * T;          // query columns per pass
    constexpr int RS = PW + 8;          // int16 per profile row (padded)
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    int16_t *prof = (int16_t *)lds;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int pad = a.R - 1;
    const int pair = blockIdx.x * W + w;
    const int64_t id = pair < a.n_pairs ? a.ids[pair] : -1;
    const int n = id >= 0 ? (int)(a.off[id + 1] - a.off[id]) : 0;
    const uint8_t *s = id >= 0 ? a.res + a.off[id] : a.res;
    uint8_t *dir = a.dir + (id >= 0 ? a.dir_off[pair] : 0);
    int32_t *wsc = a.pass_scratch + (size_t)(blockIdx.x * W + w) * (size_t)a.max_len_pad * 2;
    const int npass = (a.qlen + PW - 1) / PW;
    int best = 0, bi = 0x7fffffff, bj = 0x7fffffff;

    for (int p = 0; p < npass; ++p) {
        __syncthreads();
        for (int e = threadIdx.x; e < a.R * PW; e += W * 64) {
            const int r = e / PW, c = e - r * PW;
            const int col = p * PW + c;
            prof[r * RS + c] = col < a.qlen ? (int16_t)a.qp[(size_t)r * a.mpad + col] : (int16_t)0;
        }
        __syncthreads();
        if (n <= 0) continue;
        const bool has_in = p > 0, has_out = p + 1 < npass;
        const int nblk = (n + 63) / 64;
        const int steps = has_out ? nblk * 64 + 63 : n + 63;
        const int col0 = p * PW + lane * T;             // first query column of this lane
        const bool cols_in_row = col0 < a.ldq;          // its T bytes lie inside the row
        int H[T], E[T];
#pragma unroll
        for (int j = 0; j < T; ++j) { H[j] = 0; E[j] = 0; }
        int hb_prev = 0, hout = 0, fout = 0, r = pad, cH = 0, cF = 0;
        int pbest = 0, pt = -1, pj = 0;
        // Feeders: lane k holds the data of subject row 64*b + k: its residue
        // and H, F of the previous pass's last column (0 on the first pass).
        int fR, fH, fF, nR, nH, nF;
        {
            const int row = lane;
            fR = row < n ? s[row] : pad;
            fH = (has_in && row < n) ? wsc[2 * row] : 0;
            fF = (has_in && row < n) ? wsc[2 * row + 1] : 0;
            const int row2 = 64 + lane;
            nR = row2 < n ? s[row2] : pad;
            nH = (has_in && row2 < n) ? wsc[2 * row2] : 0;
            nF = (has_in && row2 < n) ? wsc[2 * row2 + 1] : 0;
        }
        auto step = [&](int t, auto fill) {
            if (t > 0 && (t & 63) == 0) {
                fR = nR; fH = nH; fF = nF;
                const int row = t + 64 + lane;
                nR = row < n ? s[row] : pad;
                nH = (has_in && row < n) ? wsc[2 * row] : 0;
                nF = (has_in && row < n) ? wsc[2 * row + 1] : 0;
            }
            r = shr1(fR, r);
            const int hin = shr1(fH, hout);     // H(i, col0 - 1)
            const int fin = shr1(fF, fout);     // F(i, col0 - 1)
            fR = shl1(fR, fR);
            fH = shl1(fH, fH);
            fF = shl1(fF, fF);
            const int i = t - lane;             // this lane's subject row at this step
            uint32_t cw[T / 4];
            align_row<T, decltype(fill)::value>(a, H, E, prof + r * RS + lane * T, t, i, hb_prev,
                                                hin, fin, pbest, pt, pj, cw, hout, fout);
            if (i >= 0 && i < n && cols_in_row) {
                uint8_t *dst = dir + (size_t)i * (size_t)a.ldq + col0;
                if constexpr (T == 16) *(uint4 *)dst = make_uint4(cw[0], cw[1], cw[2], cw[3]);
                else if constexpr (T == 8) *(uint2 *)dst = make_uint2(cw[0], cw[1]);
                else *(uint32_t *)dst = cw[0];
            }
            hb_prev = hin;
            if (has_out) {
                cH = shl1(hout, cH);
                cF = shl1(fout, cF);
                if ((t & 63) == 62 && t >= 126) {
                    const int row = t - 126 + lane;
                    wsc[2 * row] = cH;
                    wsc[2 * row + 1] = cF;
                }
            }
        };
        const int fill_end = steps < 63 ? steps : 63;
        for (int t = 0; t < fill_end; ++t) step(t, std::true_type{});
        for (int t = fill_end; t < steps; ++t) step(t, std::false_type{});
        // merge the pass: a tie with an earlier pass keeps the smaller row
        if (pt >= 0) {
            const int pi = pt - lane;
            if (pbest > best || (pbest == best && pi < bi)) {
                best = pbest;
                bi = pi;
                bj = col0 + pj;
            }
        }
    }
    // (score desc, row asc, column asc) over the wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int ob = __shfl_xor(best, o, 64), oi = __shfl_xor(bi, o, 64), oj = __shfl_xor(bj, o, 64);
        if (ob > best || (ob == best && (oi < bi || (oi == bi && oj < bj)))) {
            best = ob;
            bi = oi;
            bj = oj;
        }
    }
    if (lane == 0 && pair < a.n_pairs) {
        a.end[3 * pair] = best;
        a.end[3 * pair + 1] = bi;
        a.end[3 * pair + 2] = bj;
    }
}

// Pipelined forward pass: one workgroup per pair and one wave per pass of T
// columns per lane, all passes at once, each with its int8 profile in LDS.
// Wave w runs pass w kAlignPipeLag steps behind wave w - 1: lane 63 of wave
// w - 1 writes H and F of the pass's last column, row by row, to an LDS ring
// that wave w reads at the start of each block of 64 steps.  Every wave meets a barrier after every
// global block of 64 steps (the trip count is the same for all of them), so a
// row written in one block is read in a later one, and a ring slot is read
// before it is written again (the ring holds 256 rows, the lag is 128).
template <int T>
__global__ void __launch_bounds__(kAlignPipeMax * 64) align_pipe_kernel(AlignArgs a, int P) {
    constexpr int PW = 64 * T;          // query columns per pass
    constexpr int RS = PW + 16;         // int8 per profile row (padded)
    constexpr int RING = kAlignPipeRing;
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // this wave's pass
    const int pad = a.R - 1;
    const int pair = blockIdx.x;
    const int64_t id = a.ids[pair];
    const int n = id >= 0 ? (int)(a.off[id + 1] - a.off[id]) : 0;
    const uint8_t *s = id >= 0 ? a.res + a.off[id] : a.res;
    uint8_t *dir = a.dir + (id >= 0 ? a.dir_off[pair] : 0);
    int8_t *profs = (int8_t *)lds;
    uint2 *rings = (uint2 *)(lds + align_pipe_prof_bytes(a.R, T, P) / 4);
    int *red = (int *)(rings + (P - 1) * RING);

    for (int e = threadIdx.x; e < P * a.R * PW; e += blockDim.x) {
        const int pass = e / (a.R * PW), rc = e - pass * (a.R * PW);
        const int r = rc / PW, c = rc - r * PW;
        const int col = pass * PW + c;
        profs[(pass * a.R + r) * RS + c] = col < a.qlen ? a.qp[(size_t)r * a.mpad + col] : (int8_t)0;
    }
    __syncthreads();

    const int8_t *prof = profs + w * a.R * RS;
    const bool has_in = w > 0, has_out = w + 1 < P;
    const uint2 *in_ring = rings + (has_in ? w - 1 : 0) * RING;
    uint2 *out_ring = rings + (has_out ? w : 0) * RING;
    const int steps = n + 63;
    const int nlb = n > 0 ? (steps + 63) / 64 : 0;          // blocks of this wave
    constexpr int lagb = kAlignPipeLag / 64;
    const int total = nlb > 0 ? nlb + (P - 1) * lagb : 0;   // same for every wave
    const int col0 = w * PW + lane * T;
    const bool cols_in_row = col0 < a.ldq;
    int H[T], E[T];
#pragma unroll
    for (int j = 0; j < T; ++j) { H[j] = 0; E[j] = 0; }
    int hb_prev = 0, hout = 0, fout = 0, r = pad;
    int pbest = 0, pt = -1, pj = 0;
    // residues of the next block, loaded one block ahead
    int nR = lane < n ? s[lane] : pad;

    for (int gb = 0; gb < total; ++gb) {
        const int lb = gb - w * lagb;
        if (lb >= 0 && lb < nlb) {
            const int row = 64 * lb + lane;
            int fR = nR;
            nR = row + 64 < n ? s[row + 64] : pad;
            int fH = 0, fF = 0;
            if (has_in && row < n) {
                const uint2 v = in_ring[row & (RING - 1)];
                fH = (int)v.x;
                fF = (int)v.y;
            }
            const int ue = steps - 64 * lb < 64 ? steps - 64 * lb : 64;
            auto step = [&](int t, auto fill) {
                r = shr1(fR, r);
                const int hin = shr1(fH, hout);
                const int fin = shr1(fF, fout);
                fR = shl1(fR, fR);
                fH = shl1(fH, fH);
                fF = shl1(fF, fF);
                const int i = t - lane;
                uint32_t cw[T / 4];
                align_row<T, decltype(fill)::value>(a, H, E, prof + r * RS + lane * T, t, i,
                                                    hb_prev, hin, fin, pbest, pt, pj, cw, hout,
                                                    fout);   // int8 scores
                if (i >= 0 && i < n && cols_in_row) {
                    uint8_t *dst = dir + (size_t)i * (size_t)a.ldq + col0;
                    if constexpr (T == 16) *(uint4 *)dst = make_uint4(cw[0], cw[1], cw[2], cw[3]);
                    else if constexpr (T == 8) *(uint2 *)dst = make_uint2(cw[0], cw[1]);
                    else *(uint32_t *)dst = cw[0];
                }
                hb_prev = hin;
                // lane 63 hands row t - 63 of the pass's last column on
                if (has_out && lane == 63 && t >= 63)
                    out_ring[(t - 63) & (RING - 1)] = make_uint2((uint32_t)hout, (uint32_t)fout);
            };
            for (int u = 0; u < ue; ++u) {
                const int t = 64 * lb + u;
                if (t < 63) step(t, std::true_type{});
                else step(t, std::false_type{});
            }
        }
        __syncthreads();
    }
    // this wave's candidate, then (score desc, row asc, column asc) over the
    // wave and over the passes
    int best = 0, bi = 0x7fffffff, bj = 0x7fffffff;
    if (pt >= 0) {
        best = pbest;
        bi = pt - lane;
        bj = col0 + pj;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int ob = __shfl_xor(best, o, 64), oi = __shfl_xor(bi, o, 64), oj = __shfl_xor(bj, o, 64);
        if (ob > best || (ob == best && (oi < bi || (oi == bi && oj < bj)))) {
            best = ob;
            bi = oi;
            bj = oj;
        }
    }
    if (lane == 0) {
        red[3 * w] = best;
        red[3 * w + 1] = bi;
        red[3 * w + 2] = bj;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int b = red[0], ri = red[1], rj = red[2];
        for (int k = 1; k < P; ++k) {
            const int ob = red[3 * k], oi = red[3 * k + 1], oj = red[3 * k + 2];
            if (ob > b || (ob == b && (oi < ri || (oi == ri && oj < rj)))) {
                b = ob;
                ri = oi;
                rj = oj;
            }
        }
        a.end[3 * pair] = b;
        a.end[3 * pair + 1] = ri;
        a.end[3 * pair + 2] = rj;
    }
}

__global__ void align_back_kernel(AlignArgs a) {
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= a.n_pairs) return;
    int32_t *out = a.out + 6 * (size_t)pair;
    const int64_t id = a.ids[pair];
    const int score = a.end[3 * pair];
    out[0] = score;
    out[1] = out[2] = out[3] = out[4] = -1;
    out[5] = 0;
    if (id < 0 || score <= 0) return;
    const int n = (int)(a.off[id + 1] - a.off[id]), m = a.qlen;
    const int end_i = a.end[3 * pair + 1], end_j = a.end[3 * pair + 2];
    const uint8_t *dir = a.dir + a.dir_off[pair];
    const size_t ld = (size_t)a.ldq;
    uint32_t *ops = a.ops + a.ops_off[pair];
    const int64_t cap = (int64_t)n + m;
    int i = end_i, j = end_j, state = 0;
    uint32_t run_op = 3, run_len = 0;
    int64_t nrev = 0, guard = 0;
    bool ok = true;
    auto push = [&](uint32_t v) {
        if (nrev < cap) ops[nrev++] = v;
        else ok = false;
    };
    for (;;) {
        // every move lowers i or j, and a step that only enters E or F is
        // followed by a move: at most 2 (n + m) + 1 steps
        if (i < 0 || j < 0 || i >= n || j >= m || ++guard > 2 * cap + 2) {
            ok = false;
            break;
        }
        const uint32_t code = dir[(size_t)i * ld + j];
        if (state == 0) {
            const uint32_t src = code & 3u;
            if (src == 0) {
                if (run_op == 0) {
                    ++run_len;
                } else {
                    if (run_len) push((run_len << 2) | run_op);
                    run_op = 0;
                    run_len = 1;
                }
                if (i == 0 || j == 0 || (dir[(size_t)(i - 1) * ld + (j - 1)] & 4u)) break;
                --i;
                --j;
            } else if (src == 1 || src == 2) {
                if (run_len) push((run_len << 2) | run_op);
                state = (int)src;
                run_op = src == 1 ? 2u : 1u;
                run_len = 0;
            } else {
                ok = false;
                break;
            }
        } else if (state == 1) {   // subject residue i against a gap
            ++run_len;
            const bool opened = (code >> 3) & 1u;
            --i;
            if (opened) {
                push((run_len << 2) | run_op);
                run_op = 3;
                run_len = 0;
                state = 0;
            }
        } else {                   // query residue j against a gap
            ++run_len;
            const bool opened = (code >> 4) & 1u;
            --j;
            if (opened) {
                push((run_len << 2) | run_op);
                run_op = 3;
                run_len = 0;
                state = 0;
            }
        }
    }
    if (ok && run_len) push((run_len << 2) | run_op);
    if (!ok) {
        out[5] = -1;
        return;
    }
    for (int64_t k = 0; k < nrev / 2; ++k) {
        const uint32_t x = ops[k];
        ops[k] = ops[nrev - 1 - k];
        ops[nrev - 1 - k] = x;
    }
    out[1] = j;
    out[2] = end_j;
    out[3] = i;
    out[4] = end_i;
    out[5] = (int32_t)nrev;
}

// Columns per lane of the forward pass: the fewest passes, then the fewest
// columns per lane (a short query leaves most of a wide pass idle while every
// step still costs all of a lane's columns).
int align_T_for(int qlen) {
    if (qlen <= 256) return 4;
    if (qlen <= 512) return 8;
    return 16;
}

// The pipelined forward pass takes the fewest columns per lane (4 or 8; at 16
// the kernel would not fit 128 VGPRs) whose passes fit a workgroup (waves and
// LDS); a query of one pass stays on the kernel that puts several pairs in a
// workgroup.
int align_pipe_plan(int R, int qlen, int *P_out) {
    for (int T = 4; T <= 8; T *= 2) {
        const int P = (qlen + 64 * T - 1) / (64 * T);
        if (P < 2) return 0;
        if (P <= kAlignPipeMax && align_pipe_lds_bytes(R, T, P) <= 160 * 1024 - 64) {
            *P_out = P;
            return T;
        }
    }
    return 0;
}

hipError_t launch_align(const AlignArgs &a, hipStream_t st) {
    if (a.n_pairs <= 0) return hipSuccess;
    int P = 0;
    if (const int Tp = align_pipe_plan(a.R, a.qlen, &P)) {
        const int lds = align_pipe_lds_bytes(a.R, Tp, P);
        if (Tp == 4)
            hipLaunchKernelGGL(align_pipe_kernel<4>, dim3(a.n_pairs), dim3(P * 64), lds, st, a, P);
        else
            hipLaunchKernelGGL(align_pipe_kernel<8>, dim3(a.n_pairs), dim3(P * 64), lds, st, a, P);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(align_back_kernel, dim3((a.n_pairs + 63) / 64), dim3(64), 0, st, a);
        return hipGetLastError();
    }
    const int grid = (a.n_pairs + kAlignWaves - 1) / kAlignWaves;
    const int T = align_T_for(a.qlen);
    const int lds = intra_lds_bytes(a.R, T);
    if (T == 4)
        hipLaunchKernelGGL((align_fwd_kernel<4, kAlignWaves>), dim3(grid), dim3(kAlignWaves * 64), lds, st, a);
    else if (T == 8)
        hipLaunchKernelGGL((align_fwd_kernel<8, kAlignWaves>), dim3(grid), dim3(kAlignWaves * 64), lds, st, a);
    else
        hipLaunchKernelGGL((align_fwd_kernel<16, kAlignWaves>), dim3(grid), dim3(kAlignWaves * 64), lds, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(align_back_kernel, dim3((a.n_pairs + 63) / 64), dim3(64), 0, st, a);
    return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed device scratch for sw_db_search_dev_noalloc (callers that cannot
// allocate).  Host code never passes `scratch` itself to a kernel: in host
// code the name is a host-side stand-in.  Its device address, one per GPU, is
// taken once per device by noalloc_scratch_init and handed out by
// noalloc_scratch.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the device must be current
    uint8_t *ptr = nullptr;
    e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

uint8_t *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

// Per-call state of sw_db_search_dev_noalloc, written on the device: the
// query profile (section III.B.2: row r holds the whole query's scores
// against residue r; the pad row, columns past the query and query codes
// outside the alphabet score 0), the one-slot query set, the work counters
// and both work lists.  Lane-per-subject items: blocks of `waves` groups,
// longest (highest) first.  Wave-per-pair items: the database's long list,
// then every subject of groups g_cut.. in descending group order, `per` ids
// per item (-1 past the end).
__global__ void noalloc_setup_kernel(NoAllocSetup s) {
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    const int64_t np = (int64_t)s.R * s.mpad;
    for (int64_t e = tid; e < np; e += step) {
        const int r = (int)(e / s.mpad), j = (int)(e - (int64_t)r * s.mpad);
        int v = 0;
        if (r < s.A && j < s.qlen) {
            const int c = s.q[j];
            if (c < s.A) v = s.matrix[c * s.A + r];
        }
        s.prof[e] = (int8_t)v;
    }
    if (tid == 0) {
        s.qp[0] = s.prof;
        s.mpad_out[0] = s.mpad;
        s.qlen_out[0] = s.qlen;
        s.gap_out[0] = s.alpha;
        s.gap_out[1] = s.beta;
    }
    for (int64_t i = tid; i < s.n_inter; i += step) {
        s.it_q[i] = 0;
        s.it_g[i] = (int32_t)((s.n_inter - 1 - i) * s.waves);
    }
    const int64_t n_long = (int64_t)s.n_static + (int64_t)(s.n_groups - s.g_cut) * kGroup;
    for (int64_t i = tid; i < (int64_t)s.n_intra * s.per; i += step) {
        if (i % s.per == 0) s.il_q[i / s.per] = 0;
        int32_t id = -1;
        if (i < s.n_static) {
            id = s.long_static[i];
        } else if (i < n_long) {
            const int64_t x = i - s.n_static;
            const int64_t g = s.n_groups - 1 - x / kGroup;
            id = s.grp_ids[g * kGroup + (kGroup - 1 - x % kGroup)];
        }
        s.il_ids[i] = id;
    }
}

hipError_t launch_noalloc_setup(const NoAllocSetup &s, hipStream_t st) {
    const int64_t work = std::max<int64_t>((int64_t)s.R * s.mpad,
                                           std::max<int64_t>(s.n_inter, (int64_t)s.n_intra * s.per));
    int64_t blocks = (work + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3((unsigned)blocks), dim3(256), 0, st, s);
    return hipGetLastError();
}

__global__ void topk_init(int32_t *state, uint32_t *hist, int32_t k) {
    const int q = blockIdx.x;
    for (int b = threadIdx.x; b < 256; b += blockDim.x) hist[q * 256 + b] = 0;
    if (threadIdx.x == 0) {
        state[q * 4 + 0] = 0;   // prefix of the threshold found so far
        state[q * 4 + 1] = k;   // entries still needed at or below the prefix
        state[q * 4 + 2] = 0;   // entries strictly above the threshold
        state[q * 4 + 3] = 0;   // write cursor of those entries
    }
}

__global__ void topk_hist(const int32_t *scores, int64_t n, const int32_t *rows, int pass,
                          const int32_t *state, uint32_t *hist) {
    __shared__ uint32_t h[256];
    const int q = blockIdx.y;
    for (int b = threadIdx.x; b < 256; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const uint32_t prefix = (uint32_t)state[q * 4 + 0];
    const int shift = 24 - 8 * pass;
    const int32_t *row = scores + (size_t)(rows ? rows[q] : q) * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)row[i];
        if (pass == 0 || (v >> (shift + 8)) == prefix) atomicAdd(&h[(v >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < 256; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[q * 256 + b], h[b]);
}

__global__ void topk_select(int32_t *state, uint32_t *hist, int nq) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    uint32_t *h = hist + q * 256;
    const int64_t kleft = state[q * 4 + 1];
    int64_t cum = 0, above = -1;
    int chosen = 0;
    for (int b = 255; b >= 0; --b) {
        if (above < 0 && cum + h[b] >= kleft) {
            chosen = b;
            above = cum;
        }
        cum += h[b];
    }
    if (above < 0) above = cum - h[0];   // fewer entries than k: take all
    state[q * 4 + 0] = (int32_t)(((uint32_t)state[q * 4 + 0] << 8) | (uint32_t)chosen);
    state[q * 4 + 1] = (int32_t)(kleft - above);
    state[q * 4 + 2] += (int32_t)above;
    for (int b = 0; b < 256; ++b) h[b] = 0;
}

__global__ void topk_gather(const int32_t *scores, int64_t n, const int32_t *rows, int32_t *state,
                            int32_t *eqcnt, int32_t *cs, int32_t *ci, int32_t k) {
    __shared__ int32_t red[32];
    const int q = blockIdx.y;
    const uint32_t theta = (uint32_t)state[q * 4 + 0];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    const int32_t *row = scores + (size_t)(rows ? rows[q] : q) * n;
    int cnt = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const uint32_t v = (uint32_t)row[i];
        if (v > theta) {
            const int pos = atomicAdd(&state[q * 4 + 3], 1);
            if (pos < k) {
                cs[q * k + pos] = (int32_t)v;
                ci[q * k + pos] = (int32_t)i;
            }
        } else if (v == theta) {
            ++cnt;
        }
    }
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
        eqcnt[q * gridDim.x + blockIdx.x] = s;
    }
}

__global__ void topk_gather_eq(const int32_t *scores, int64_t n, const int32_t *rows,
                               const int32_t *state, const int32_t *eqcnt, int32_t *cs,
                               int32_t *ci, int32_t k) {
    __shared__ int32_t wsum[16];
    __shared__ int32_t s_base;
    const int q = blockIdx.y;
    const uint32_t theta = (uint32_t)state[q * 4 + 0];
    const int need = state[q * 4 + 1];
    const int cnt_gt = state[q * 4 + 2];
    if (threadIdx.x == 0) {
        int s = 0;
        for (unsigned b = 0; b < blockIdx.x; ++b) s += eqcnt[q * gridDim.x + b];
        s_base = s;
    }
    __syncthreads();
    int base = s_base;
    if (base >= need) return;
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    const int32_t *row = scores + (size_t)(rows ? rows[q] : q) * n;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int64_t t0 = lo; t0 < hi; t0 += blockDim.x) {
        const int64_t i = t0 + threadIdx.x;
        const bool hit = i < hi && (uint32_t)row[i] == theta;
        const uint64_t bal = __ballot(hit);
        const int below = __popcll(bal & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
        if (lane == 0) wsum[wv] = __popcll(bal);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int x = 0; x < nw; ++x) {
            if (x < wv) woff += wsum[x];
            tot += wsum[x];
        }
        const int rank = base + woff + below;
        if (hit && rank < need) {
            cs[q * k + cnt_gt + rank] = (int32_t)theta;
            ci[q * k + cnt_gt + rank] = (int32_t)i;
        }
        base += tot;
        __syncthreads();
        if (base >= need) break;
    }
}

__global__ void topk_final(const int32_t *state, const int32_t *eqcnt, int nblk,
                           const int32_t *cs, const int32_t *ci, int32_t k, int32_t *top_s,
                           int64_t *top_i) {
    extern __shared__ __attribute__((aligned(16))) int32_t sm[];
    int32_t *ks = sm, *ki = sm + k;
    __shared__ int32_t s_cnt;
    const int q = blockIdx.x;
    if (threadIdx.x == 0) {
        int eq = 0;
        for (int b = 0; b < nblk; ++b) eq += eqcnt[q * nblk + b];
        const int need = state[q * 4 + 1];
        int c = state[q * 4 + 2] + (eq < need ? eq : need);
        s_cnt = c < k ? c : k;
    }
    __syncthreads();
    const int cnt = s_cnt;
    for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
        ks[x] = cs[q * k + x];
        ki[x] = ci[q * k + x];
    }
    __syncthreads();
    for (int x = threadIdx.x; x < cnt; x += blockDim.x) {
        const int sx = ks[x], ix = ki[x];
        int rank = 0;
        for (int y = 0; y < cnt; ++y)
            rank += (ks[y] > sx) || (ks[y] == sx && ki[y] < ix);
        top_s[(size_t)q * k + rank] = sx;
        top_i[(size_t)q * k + rank] = ix;
    }
    for (int x = cnt + threadIdx.x; x < k; x += blockDim.x) {
        top_s[(size_t)q * k + x] = -1;
        top_i[(size_t)q * k + x] = -1;
    }
}

// Top-k of a short score row in one workgroup per query: a bitonic sort of
// 64-bit keys (2^31 - 1 - score, index) in LDS, ascending, so the first k are
// the scores in descending order with equal scores by ascending index.  The
// radix select above takes eleven launches, which cost more than the sort at
// this size.
constexpr int kTopkSmallN = 4096;

__global__ void __launch_bounds__(1024) topk_small(const int32_t *scores, int64_t n,
                                                   const int32_t *rows, int32_t k,
                                                   int32_t *top_s, int64_t *top_i) {
    __shared__ uint64_t key[kTopkSmallN];
    const int q = blockIdx.x;
    const int32_t *row = scores + (size_t)(rows ? rows[q] : q) * n;
    int N = 1;
    while (N < n) N <<= 1;
    for (int x = threadIdx.x; x < N; x += blockDim.x)
        key[x] = x < n ? ((uint64_t)(uint32_t)(0x7fffffff - row[x]) << 32) | (uint32_t)x
                       : ~(uint64_t)0;
    __syncthreads();
    for (int size = 2; size <= N; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int x = threadIdx.x; x < N; x += blockDim.x) {
                const int y = x ^ stride;
                if (y > x) {
                    const bool up = (x & size) == 0;
                    const uint64_t a = key[x], b = key[y];
                    if ((a > b) == up) {
                        key[x] = b;
                        key[y] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int x = threadIdx.x; x < k; x += blockDim.x) {
        const bool real = x < n;
        const uint64_t v = real ? key[x] : 0;
        top_s[(size_t)q * k + x] = real ? 0x7fffffff - (int32_t)(v >> 32) : -1;
        top_i[(size_t)q * k + x] = real ? (int64_t)(uint32_t)v : -1;
    }
}

hipError_t launch_topk(const int32_t *scores, int64_t n, int32_t nq, const int32_t *rows,
                       int32_t k, const TopkWork &w, int32_t *top_s, int64_t *top_i,
                       hipStream_t st) {
    if (nq <= 0) return hipSuccess;
    if (n <= kTopkSmallN) {
        hipLaunchKernelGGL(topk_small, dim3(nq), dim3(1024), 0, st, scores, n, rows, k, top_s, top_i);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(topk_init, dim3(nq), dim3(256), 0, st, w.state, w.hist, k);
    int64_t hb = (n + 2047) / 2048;
    if (hb < 1) hb = 1;
    if (hb > 128) hb = 128;
    for (int pass = 0; pass < 4; ++pass) {
        hipLaunchKernelGGL(topk_hist, dim3((unsigned)hb, nq), dim3(256), 0, st, scores, n, rows,
                           pass, w.state, w.hist);
        hipLaunchKernelGGL(topk_select, dim3((nq + 63) / 64), dim3(64), 0, st, w.state, w.hist, nq);
    }
    hipLaunchKernelGGL(topk_gather, dim3(kTopkBlocks, nq), dim3(256), 0, st, scores, n, rows,
                       w.state, w.eqcnt, w.cand_s, w.cand_i, k);
    hipLaunchKernelGGL(topk_gather_eq, dim3(kTopkBlocks, nq), dim3(256), 0, st, scores, n, rows,
                       w.state, w.eqcnt, w.cand_s, w.cand_i, k);
    hipLaunchKernelGGL(topk_final, dim3(nq), dim3(256), (size_t)k * 8, st, w.state, w.eqcnt,
                       kTopkBlocks, w.cand_s, w.cand_i, k, top_s, top_i);
    return hipGetLastError();
}

hipError_t prepare_kernels() {
#define SWMI_K(T_, W_, TIER_, TI_) (const void *)inter_kernel<T_, W_, TIER_, TI_>
#define SWMI_FUSED(W_, TIER_) \
    SWMI_K(kFuseStrip, W_, TIER_, 4), SWMI_K(kFuseStrip, W_, TIER_, 8), SWMI_K(kFuseStrip, W_, TIER_, 16)
    const void *ks[] = {
        SWMI_K(16, 4, TIER_F16X2, 0), SWMI_K(16, 8, TIER_F16X2, 0), SWMI_K(32, 4, TIER_F16X2, 0),
        SWMI_K(32, 6, TIER_F16X2, 0), SWMI_K(32, 8, TIER_F16X2, 0), SWMI_K(64, 4, TIER_F16X2, 0),
        SWMI_K(16, 4, TIER_I16X2, 0), SWMI_K(16, 8, TIER_I16X2, 0), SWMI_K(32, 4, TIER_I16X2, 0),
        SWMI_K(32, 6, TIER_I16X2, 0), SWMI_K(32, 8, TIER_I16X2, 0), SWMI_K(64, 4, TIER_I16X2, 0),
        SWMI_FUSED(4, TIER_F16X2), SWMI_FUSED(6, TIER_F16X2), SWMI_FUSED(8, TIER_F16X2),
        (const void *)intra_kernel<4, 1>,  (const void *)intra_kernel<8, 1>,
        (const void *)intra_kernel<16, 1>, (const void *)intra_kernel<4, 4>,
        (const void *)intra_kernel<8, 4>,  (const void *)intra_kernel<16, 4>,
        (const void *)intra2_kernel<4, 4>, (const void *)intra2_kernel<8, 4>,
        (const void *)intra2_kernel<16, 4>,
        (const void *)align_fwd_kernel<4, kAlignWaves>, (const void *)align_fwd_kernel<8, kAlignWaves>,
        (const void *)align_fwd_kernel<16, kAlignWaves>, (const void *)align_pipe_kernel<4>,
        (const void *)align_pipe_kernel<8>, (const void *)inter_sp_kernel<32, 4>,
    };
#undef SWMI_FUSED
#undef SWMI_K
    for (const void *k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024 - 64);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace swmi
