/*
 * CPU oracle for Smith-Waterman protein database search — TEST INFRASTRUCTURE.
 *
 * This file is the parity authority for the GPU library: a plain, scalar,
 * obviously correct evaluation of the affine-gap Smith-Waterman score.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or table with the GPU path.
 *
 * What it computes (section II.A, Eq. 1 and the initialisation that follows it):
 *
 *   H(i,j) = max{ 0, H(i-1,j-1) + sbt(i,j), E(i,j), F(i,j) }
 *   E(i,j) = max{ E(i-1,j) - alpha, H(i-1,j) - beta }
 *   F(i,j) = max{ F(i,j-1) - alpha, H(i,j-1) - beta }
 *   H(i,0) = H(0,j) = E(0,j) = F(i,0) = 0,   score = max over all H(i,j).
 *
 * alpha is the gap-extension penalty and beta the sum of gap-open and
 * extension penalties (section II.A).  Readings taken where the paper is not
 * explicit:
 *   - i runs over the database (subject) sequence and j over the query: the
 *     paper's alignment kernels stream subject residues in the outer loop and
 *     query positions in the inner loop (Fig. 3), and keep one row of H and E
 *     whose size follows the query length (section III.A).
 *   - sbt(i,j) = matrix[q[j] * alphabet + s[i]]: the matrix row is the QUERY
 *     residue, as in the query profile, whose column r holds the scores of the
 *     whole query against residue r (section III.B.2).
 *   - E and F start from 0 exactly as written (not minus infinity).
 *
 * Linear space (section II.A, last sentence; section III.A): one row of H and
 * one row of E, plus scalars for the diagonal, the left neighbour and F.
 *
 * Integer width: int32, the paper's lane width (section III).  Values stay in
 * range for lengths <= 2^24, |matrix| <= 127 and 0 <= alpha <= beta <= 2^30:
 * E and F never drop below -beta because H >= 0, and H <= 127 * min(m, n).
 *
 * Built with -O2 -fno-tree-vectorize; OpenMP only spreads whole subjects over
 * threads (dynamic schedule, chunks of 64), never inside one alignment.
 */
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }

/* Score of one query (length m) against one subject (length n).
 * Returns -1 if the row buffers cannot be allocated. */
int32_t oracle_sw_score(const uint8_t *q, int32_t m, const uint8_t *s, int64_t n,
                        const int8_t *matrix, int32_t alphabet,
                        int32_t alpha, int32_t beta)
{
    if (m <= 0 || n <= 0)
        return 0;                       /* H is all zeros: max H = 0 */

    /* Row i-1 of H and of E, indexed by query position j = 0..m. */
    int32_t *h_row = (int32_t *)calloc((size_t)m + 1, sizeof(int32_t));
    int32_t *e_row = (int32_t *)calloc((size_t)m + 1, sizeof(int32_t));
    if (!h_row || !e_row) {
        free(h_row);
        free(e_row);
        return -1;
    }
    /* calloc: H(0,j) = 0 and E(0,j) = 0 */

    int32_t best = 0;
    for (int64_t i = 1; i <= n; ++i) {
        const int32_t s_res = s[i - 1];
        int32_t h_diag = 0;             /* H(i-1, 0) */
        int32_t h_left = 0;             /* H(i, 0)   */
        int32_t f = 0;                  /* F(i, 0)   */
        for (int32_t j = 1; j <= m; ++j) {
            const int32_t sbt = matrix[(int32_t)q[j - 1] * alphabet + s_res];
            const int32_t e = imax(e_row[j] - alpha, h_row[j] - beta);   /* E(i,j) */
            f = imax(f - alpha, h_left - beta);                          /* F(i,j) */
            int32_t h = 0;
            h = imax(h, h_diag + sbt);
            h = imax(h, e);
            h = imax(h, f);                                              /* H(i,j) */
            h_diag = h_row[j];          /* H(i-1, j) is the next column's diagonal */
            h_row[j] = h;
            e_row[j] = e;
            h_left = h;
            if (h > best)
                best = h;
        }
    }
    free(h_row);
    free(e_row);
    return best;
}

/* Score one query against every sequence of a database given as concatenated
 * residues plus n_seqs+1 offsets.  scores[k] is the score of sequence k, in the
 * database's own order.  nthreads <= 0 lets OpenMP choose. */
void oracle_search(const uint8_t *q, int32_t m,
                   const uint8_t *residues, const int64_t *offsets, int64_t n_seqs,
                   const int8_t *matrix, int32_t alphabet, int32_t alpha, int32_t beta,
                   int32_t *scores, int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) {
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
        for (int64_t k = 0; k < n_seqs; ++k)
            scores[k] = oracle_sw_score(q, m, residues + offsets[k], offsets[k + 1] - offsets[k],
                                        matrix, alphabet, alpha, beta);
        return;
    }
#pragma omp parallel for schedule(dynamic, 64)
#else
    (void)nthreads;
#endif
    for (int64_t k = 0; k < n_seqs; ++k)
        scores[k] = oracle_sw_score(q, m, residues + offsets[k], offsets[k + 1] - offsets[k],
                                    matrix, alphabet, alpha, beta);
}

/* Same, for a list of subject indices only (sampled checks at full size). */
void oracle_search_subset(const uint8_t *q, int32_t m,
                          const uint8_t *residues, const int64_t *offsets,
                          const int64_t *which, int64_t n_which,
                          const int8_t *matrix, int32_t alphabet, int32_t alpha, int32_t beta,
                          int32_t *scores, int32_t nthreads)
{
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
#endif
    for (int64_t k = 0; k < n_which; ++k) {
        const int64_t x = which[k];
        scores[k] = oracle_sw_score(q, m, residues + offsets[x], offsets[x + 1] - offsets[x],
                                    matrix, alphabet, alpha, beta);
    }
}

/* Optimal local alignment of one query against one subject, with traceback
 * (the conclusion names alignment reconstruction as future work; the scores
 * are those of Eq. 1 above, the choice among equal-scoring alignments is a
 * reading of this implementation).  Readings:
 *   - the alignment ends at the first cell, in the order i then j (subject row
 *     outer, query column inner, as above), whose H equals the score;
 *   - walking back from there, H takes its value from the diagonal before E
 *     before F; E and F take theirs from the gap opening (H - beta) before the
 *     extension (E or F - alpha);
 *   - the alignment starts at the first diagonal step whose predecessor
 *     H(i-1, j-1) is 0 (or on the boundary).
 * Output: res[0] = score, res[1] = q_begin, res[2] = q_end; sres[0] =
 * s_begin, sres[1] = s_end (0-based, inclusive; -1 when the score is 0).
 * ops: runs in forward order, (length << 2) | op with op 0 = aligned pair,
 * 1 = query residue against a gap, 2 = subject residue against a gap; every
 * gap (one opening and its extensions) is its own run, aligned pairs in a
 * row share one.  Returns the number of runs, -1 if memory runs out and -2
 * if ops_cap is too small.  Keeps one byte per cell: n * m bytes. */
int64_t oracle_sw_align(const uint8_t *q, int32_t m, const uint8_t *s, int64_t n,
                        const int8_t *matrix, int32_t alphabet, int32_t alpha, int32_t beta,
                        int32_t *res, int64_t *sres, uint32_t *ops, int64_t ops_cap)
{
    res[0] = 0;
    res[1] = res[2] = -1;
    sres[0] = sres[1] = -1;
    if (m <= 0 || n <= 0)
        return 0;
    /* dir[(i-1) * m + (j-1)] for cell (i, j): bits 0-1 where H came from
     * (0 diagonal, 1 E, 2 F), bit 2 H == 0, bit 3 E opened, bit 4 F opened */
    uint8_t *dir = (uint8_t *)malloc((size_t)n * (size_t)m);
    int32_t *h_row = (int32_t *)calloc((size_t)m + 1, sizeof(int32_t));
    int32_t *e_row = (int32_t *)calloc((size_t)m + 1, sizeof(int32_t));
    uint32_t *rev = (uint32_t *)malloc(((size_t)n + (size_t)m + 1) * sizeof(uint32_t));
    if (!dir || !h_row || !e_row || !rev) {
        free(dir);
        free(h_row);
        free(e_row);
        free(rev);
        return -1;
    }
    int32_t best = 0;
    int64_t bi = 0, bj = 0;
    for (int64_t i = 1; i <= n; ++i) {
        const int32_t s_res = s[i - 1];
        int32_t h_diag = 0, h_left = 0, f = 0;
        for (int32_t j = 1; j <= m; ++j) {
            const int32_t sbt = matrix[(int32_t)q[j - 1] * alphabet + s_res];
            const int32_t e_ext = e_row[j] - alpha, e_open = h_row[j] - beta;
            const int32_t e = imax(e_ext, e_open);
            const int32_t f_ext = f - alpha, f_open = h_left - beta;
            f = imax(f_ext, f_open);
            const int32_t d = h_diag + sbt;
            int32_t h = imax(imax(0, d), imax(e, f));
            uint8_t code;
            if (h == 0) code = 4;
            else if (h == d) code = 0;
            else if (h == e) code = 1;
            else code = 2;
            if (e_open >= e_ext) code |= 8;
            if (f_open >= f_ext) code |= 16;
            dir[(size_t)(i - 1) * (size_t)m + (size_t)(j - 1)] = code;
            h_diag = h_row[j];
            h_row[j] = h;
            e_row[j] = e;
            h_left = h;
            if (h > best) {
                best = h;
                bi = i;
                bj = j;
            }
        }
    }
    free(h_row);
    free(e_row);
    res[0] = best;
    if (best == 0) {
        free(dir);
        free(rev);
        return 0;
    }
    /* walk back: state 0 in H, 1 in E, 2 in F; ops collected in reverse */
    int64_t i = bi, j = bj, nrev = 0;
    int state = 0;
    uint32_t run_op = 3, run_len = 0;
    for (;;) {
        const uint8_t code = dir[(size_t)(i - 1) * (size_t)m + (size_t)(j - 1)];
        if (state == 0) {
            const int src = code & 3;
            if (src == 0) {
                if (run_op == 0) {
                    ++run_len;
                } else {
                    if (run_len) rev[nrev++] = (run_len << 2) | run_op;
                    run_op = 0;
                    run_len = 1;
                }
                const int at_start = i == 1 || j == 1 ||
                                     (dir[(size_t)(i - 2) * (size_t)m + (size_t)(j - 2)] & 4);
                if (at_start)
                    break;
                --i;
                --j;
            } else {
                state = src;   /* 1: E, 2: F; the gap run starts here */
                if (run_len) rev[nrev++] = (run_len << 2) | run_op;
                run_op = src == 1 ? 2u : 1u;
                run_len = 0;
            }
        } else if (state == 1) {   /* subject residue i against a gap */
            ++run_len;
            const int opened = (code >> 3) & 1;
            --i;
            if (opened) {
                rev[nrev++] = (run_len << 2) | run_op;
                run_op = 3;
                run_len = 0;
                state = 0;
            }
        } else {                   /* query residue j against a gap */
            ++run_len;
            const int opened = (code >> 4) & 1;
            --j;
            if (opened) {
                rev[nrev++] = (run_len << 2) | run_op;
                run_op = 3;
                run_len = 0;
                state = 0;
            }
        }
    }
    if (run_len) rev[nrev++] = (run_len << 2) | run_op;
    free(dir);
    res[1] = (int32_t)(j - 1);
    res[2] = (int32_t)(bj - 1);
    sres[0] = i - 1;
    sres[1] = bi - 1;
    if (nrev > ops_cap) {
        free(rev);
        return -2;
    }
    for (int64_t k = 0; k < nrev; ++k)
        ops[k] = rev[nrev - 1 - k];
    free(rev);
    return nrev;
}

/* Number of threads OpenMP would use (1 without OpenMP). */
int32_t oracle_max_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
