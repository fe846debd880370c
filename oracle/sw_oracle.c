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

/* Number of threads OpenMP would use (1 without OpenMP). */
int32_t oracle_max_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}
