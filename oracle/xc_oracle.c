/*
 * xc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of the correlator that
 * van Nieuwpoort & Romein describe ("Correlating Radio Astronomy Signals with
 * Many-Core Hardware", Section 2: the correlation equation and the pseudo-code
 * of Figure 2).  Only tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header, table or helper with the GPU
 * library: it depends only on the written definition.
 *
 * What it computes (Section 2, correlation equation):
 *
 *   V[c][b(i,j)][p][q] = sum_{t=0}^{T-1} x[c][t][i][p] * conj(x[c][t][j][q])
 *
 * for every channel c, every station pair 0 <= i <= j < S (autocorrelations
 * included, Section 2), and every polarisation pair p, q in {X=0, Y=1}.
 * The conjugated factor is the higher-index station j (the equation puts the
 * conjugate on s2 >= s1; Figure 2 conjugates station2's sample).
 *
 * Readings taken where the paper is silent:
 *   - computeBaseline(i, j) of Figure 2 is b(i,j) = j(j+1)/2 + i: dense, in the
 *     order in which Figure 2 enumerates the pairs (station2 outer, station1
 *     inner).
 *   - Samples are stored time-major, x[c][t][s][p] (the layout Section 4.4
 *     describes as "all stations for each time step together"); the output is
 *     channel-major, V[c][b][p][q] (Figure 2 writes correlation[b][c][p][q];
 *     the two differ by a permutation of the first two axes).
 *   - The sum is plain: no 1/T normalisation, weights or flags (Section 2,
 *     "accumulating all products").
 *
 * Arithmetic: floating-point inputs are widened (exactly) to double by the
 * caller and summed in double; complex-int8 inputs are summed in int64 (exact).
 * The complex multiply-accumulate is split into real and imaginary parts as
 * Section 2 derives it:
 *     re += a_r b_r + a_i b_i
 *     im += a_i b_r - a_r b_i
 * Build with -ffp-contract=off so that the two products of an
 * autocorrelation's imaginary part round identically and cancel exactly.
 *
 * Loop order is that of Figure 2 (channel, station2, station1 <= station2,
 * pol1, pol2, time), so outputs are produced in storage order.  The only
 * parallelism is an OpenMP loop over channels, which are independent
 * (Section 2, "trivially parallel").
 */
#include <stdint.h>
#include <stddef.h>

/* b(i,j) for 0 <= i <= j: the dense baseline number of Figure 2. */
static int64_t oracle_baseline(int64_t i, int64_t j)
{
    return j * (j + 1) / 2 + i;
}

int64_t oracle_n_baselines(int32_t n_stations)
{
    return (int64_t)n_stations * (n_stations + 1) / 2;
}

/*
 * x   : double [C][T][S][P][2]  (re, im)
 * vis : double [C][B][P][P][2]  (re, im), B = S(S+1)/2, fully overwritten
 */
void oracle_correlate_f64(const double *x, int32_t S, int32_t P, int32_t C,
                          int32_t T, double *vis)
{
    const int64_t B = oracle_n_baselines(S);
    int64_t ch;
#pragma omp parallel for schedule(dynamic, 1)
    for (ch = 0; ch < C; ch++) {
        for (int64_t station2 = 0; station2 < S; station2++) {
            for (int64_t station1 = 0; station1 <= station2; station1++) {
                for (int64_t pol1 = 0; pol1 < P; pol1++) {
                    for (int64_t pol2 = 0; pol2 < P; pol2++) {
                        double sum_re = 0.0, sum_im = 0.0;
                        for (int64_t t = 0; t < T; t++) {
                            const double *a = x + 2 * (((ch * T + t) * S + station1) * P + pol1);
                            const double *b = x + 2 * (((ch * T + t) * S + station2) * P + pol2);
                            /* a * conj(b) */
                            sum_re += a[0] * b[0] + a[1] * b[1];
                            sum_im += a[1] * b[0] - a[0] * b[1];
                        }
                        int64_t bl = oracle_baseline(station1, station2);
                        double *v = vis + 2 * (((ch * B + bl) * P + pol1) * P + pol2);
                        v[0] = sum_re;
                        v[1] = sum_im;
                    }
                }
            }
        }
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
    int64_t ch;
#pragma omp parallel for schedule(dynamic, 1)
    for (ch = 0; ch < C; ch++) {
        for (int64_t station2 = 0; station2 < S; station2++) {
            for (int64_t station1 = 0; station1 <= station2; station1++) {
                for (int64_t pol1 = 0; pol1 < P; pol1++) {
                    for (int64_t pol2 = 0; pol2 < P; pol2++) {
                        int64_t sum_re = 0, sum_im = 0;
                        for (int64_t t = 0; t < T; t++) {
                            const int8_t *a = x + 2 * (((ch * T + t) * S + station1) * P + pol1);
                            const int8_t *b = x + 2 * (((ch * T + t) * S + station2) * P + pol2);
                            int64_t ar = a[0], ai = a[1], br = b[0], bi = b[1];
                            /* a * conj(b) */
                            sum_re += ar * br + ai * bi;
                            sum_im += ai * br - ar * bi;
                        }
                        int64_t bl = oracle_baseline(station1, station2);
                        int64_t *v = vis + 2 * (((ch * B + bl) * P + pol1) * P + pol2);
                        v[0] = sum_re;
                        v[1] = sum_im;
                    }
                }
            }
        }
    }
}
