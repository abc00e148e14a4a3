/*
 * xc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of the correlator of
 * van Nieuwpoort & Romein, "Correlating Radio Astronomy Signals with
 * Many-Core Hardware" (Section 2, the correlation equation).  Only tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or helper with the GPU library and depends only on the
 * written definition.
 *
 * Definition (Section 2, correlation equation): for every channel c, every
 * station pair 0 <= i <= j < S (autocorrelations included) and every
 * polarisation pair p, q in {X=0, Y=1},
 *
 *   V[c][b(i,j)][p][q] = sum_{t=0}^{T-1} x[c][t][i][p] * conj(x[c][t][j][q]),
 *   b(i,j) = j(j+1)/2 + i.
 *
 * Written out here as linear algebra: number the rows of one time step's
 * samples r = s P + p (station-major, polarisation inner), so that a time
 * step is a vector a_t of S P complex numbers.  Then the correlation of a
 * channel is the Hermitian Gram matrix G = sum_t a_t a_t^H, and V holds its
 * 2x2 blocks on and above the block diagonal: V[b(i,j)][p][q] = G[iP+p][jP+q].
 * The code accumulates G one time step at a time (a rank-one update, time
 * ascending, of the entries whose column station is not below the row's
 * station) and then packs those blocks into V.
 *
 * Readings where the paper is silent or ambiguous:
 *   - The conjugated factor belongs to the higher-numbered station j (the
 *     equation conjugates the second station's sample).
 *   - The baseline number is b(i,j) = j(j+1)/2 + i: the pairs numbered
 *     densely, column by column of the upper triangle.
 *   - Samples are time-major x[c][t][s][p] (Section 4.4's GPU layout); the
 *     output is channel-major V[c][b][p][q] (the paper's output order is the
 *     same data with the first two axes swapped).
 *   - The integration is a plain sum: no 1/T normalisation, weights or flags.
 *
 * Arithmetic: floating-point inputs are widened (exactly) to double by the
 * caller and summed in double; complex-int8 inputs are summed in int64
 * (exact).  A complex multiply-accumulate u * conj(w) is split into its real
 * and imaginary parts (Section 2):
 *     re += u_r w_r + u_i w_i
 *     im += u_i w_r - u_r w_i
 * Build with -ffp-contract=off so that the two products of a diagonal
 * entry's imaginary part round identically and cancel exactly.  Channels are
 * independent (Section 2), so an OpenMP loop over channels is the only
 * parallelism.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Dense number of the station pair i <= j. */
static int64_t pair_number(int64_t i, int64_t j)
{
    return j * (j + 1) / 2 + i;
}

int64_t oracle_n_baselines(int32_t n_stations)
{
    return (int64_t)n_stations * (n_stations + 1) / 2;
}

/*
 * Gram accumulation of one channel, double precision.
 *   xc : double [T][S*P][2]   the channel's samples, one row vector per time step
 *   gr, gi : double [S*P][S*P] real and imaginary parts of G (zeroed here)
 * Only entries G[r][u] whose column station u / P is >= the row station r / P
 * are formed; the others are left at zero and never read.
 */
static void gram_f64(const double *xc, int64_t S, int64_t P, int64_t T, double *gr, double *gi)
{
    const int64_t n = S * P;
    memset(gr, 0, sizeof(double) * n * n);
    memset(gi, 0, sizeof(double) * n * n);
    for (int64_t t = 0; t < T; t++) {
        const double *at = xc + 2 * t * n;
        for (int64_t r = 0; r < n; r++) {
            const double ur = at[2 * r], ui = at[2 * r + 1];
            for (int64_t u = (r / P) * P; u < n; u++) {
                const double wr = at[2 * u], wi = at[2 * u + 1];
                /* a[r] * conj(a[u]) */
                gr[r * n + u] += ur * wr + ui * wi;
                gi[r * n + u] += ui * wr - ur * wi;
            }
        }
    }
}

/* Same in int64 for complex-int8 samples xc : int8 [T][S*P][2]. */
static void gram_i64(const int8_t *xc, int64_t S, int64_t P, int64_t T, int64_t *gr, int64_t *gi)
{
    const int64_t n = S * P;
    memset(gr, 0, sizeof(int64_t) * n * n);
    memset(gi, 0, sizeof(int64_t) * n * n);
    for (int64_t t = 0; t < T; t++) {
        const int8_t *at = xc + 2 * t * n;
        for (int64_t r = 0; r < n; r++) {
            const int64_t ur = at[2 * r], ui = at[2 * r + 1];
            for (int64_t u = (r / P) * P; u < n; u++) {
                const int64_t wr = at[2 * u], wi = at[2 * u + 1];
                /* a[r] * conj(a[u]) */
                gr[r * n + u] += ur * wr + ui * wi;
                gi[r * n + u] += ui * wr - ur * wi;
            }
        }
    }
}

/*
 * x   : double [C][T][S][P][2]  (re, im)
 * vis : double [C][B][P][P][2]  (re, im), B = S(S+1)/2, fully overwritten
 */
void oracle_correlate_f64(const double *x, int32_t S, int32_t P, int32_t C,
                          int32_t T, double *vis)
{
    const int64_t B = oracle_n_baselines(S);
    const int64_t n = (int64_t)S * P;
    int64_t c;
#pragma omp parallel for schedule(dynamic, 1)
    for (c = 0; c < C; c++) {
        double *gr = malloc(sizeof(double) * n * n);
        double *gi = malloc(sizeof(double) * n * n);
        if (!gr || !gi)
            abort();
        gram_f64(x + 2 * c * T * n, S, P, T, gr, gi);
        /* pack the blocks on and above the block diagonal */
        for (int64_t j = 0; j < S; j++)
            for (int64_t i = 0; i <= j; i++)
                for (int64_t p = 0; p < P; p++)
                    for (int64_t q = 0; q < P; q++) {
                        const int64_t g = (i * P + p) * n + (j * P + q);
                        double *v = vis + 2 * (((c * B + pair_number(i, j)) * P + p) * P + q);
                        v[0] = gr[g];
                        v[1] = gi[g];
                    }
        free(gr);
        free(gi);
    }
}

/*
 * x   : int8  [C][T][S][P][2]  (re, im)
 * vis : int64 [C][B][P][P][2]  (re, im), fully overwritten
 */
void oracle_correlate_i64(const int8_t *x, int32_t S, int32_t P, int32_t C,
                          int32_t T, int64_t *vis)
{
    const int64_t B = oracle_n_baselines(S);
    const int64_t n = (int64_t)S * P;
    int64_t c;
#pragma omp parallel for schedule(dynamic, 1)
    for (c = 0; c < C; c++) {
        int64_t *gr = malloc(sizeof(int64_t) * n * n);
        int64_t *gi = malloc(sizeof(int64_t) * n * n);
        if (!gr || !gi)
            abort();
        gram_i64(x + 2 * c * T * n, S, P, T, gr, gi);
        for (int64_t j = 0; j < S; j++)
            for (int64_t i = 0; i <= j; i++)
                for (int64_t p = 0; p < P; p++)
                    for (int64_t q = 0; q < P; q++) {
                        const int64_t g = (i * P + p) * n + (j * P + q);
                        int64_t *v = vis + 2 * (((c * B + pair_number(i, j)) * P + p) * P + q);
                        v[0] = gr[g];
                        v[1] = gi[g];
                    }
        free(gr);
        free(gi);
    }
}
