/* Calls every exported oracle function on small inputs, plus two argument
 * errors, under AddressSanitizer / UndefinedBehaviorSanitizer (CPU only). */
#include <stdio.h>
#include <stdlib.h>
int oracle_threej_row(int l1, int l2, int m, double *out, int n_out);
int oracle_threej_row_forward(int l1, int l2, int m, int l3_hi, double *out, int n_out);
int oracle_coupling_rows(int lmax, const double *W_TT, const double *W_TP, const double *W_PP,
                         int w_len, int l3_lo, int l3_hi, const int *rows, int n_rows,
                         unsigned spectra, double *K_out, double *A_out, int n_threads);
int oracle_coupling_rows_upper(int lmax, const double *W_TT, const double *W_TP, const double *W_PP,
                         int w_len, int l3_lo, int l3_hi, const int *rows, int n_rows,
                         unsigned spectra, double *K_out, double *A_out, int n_threads, int upper);
int oracle_band_rows(int lmax, const double *W_TT, const double *W_TP, const double *W_PP,
                         int w_len, int l3_lo, int l3_hi, const int *rows, int n_rows,
                         unsigned spectra, double *K_out, double *A_out, int n_threads);
int main(void) {
    enum { L = 40, N = 2 * L + 1 };
    double w[N], row[2 * L + 1];
    int rows[L + 1], i, rc = 0;
    for (i = 0; i < N; ++i) w[i] = 1.0 / (1.0 + i);
    for (i = 0; i <= L; ++i) rows[i] = i;
    double *K = malloc(sizeof(double) * 5 * (L + 1) * (L + 1)), *A = malloc(sizeof(double) * 5 * (L + 1) * (L + 1));
    for (i = 0; i <= 2; ++i) rc |= oracle_threej_row(17, 23, -i, row, 2 * L + 1) != 35;
    rc |= oracle_threej_row_forward(30, 25, -2, 20, row, 2 * L + 1) != 16;
    rc |= oracle_coupling_rows(L, w, w, w, N, 0, 1 << 30, rows, L + 1, 31u, K, A, 2) != 0;
    rc |= oracle_coupling_rows_upper(L, w, w, w, N, 0, 1 << 30, rows, L + 1, 31u, K, A, 2, 1) != 0;
    rc |= oracle_band_rows(L, w, w, w, N, 0, 12, rows, L + 1, 31u, K, A, 2) != 0;
    rc |= oracle_coupling_rows(L, w, w, w, N - 1, 0, 1 << 30, rows, L + 1, 31u, K, A, 2) != -1;   /* short W */
    rc |= oracle_threej_row(17, 23, 0, row, 3) != -1;                                          /* short out */
    free(K); free(A);
    printf("oracle driver %s\n", rc ? "FAILED" : "ok");
    return rc;
}
