/*
 * Bulk tier of the CPU oracle for the MASTER mode-coupling matrices.
 * TEST INFRASTRUCTURE ONLY: linked by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product library.
 *
 * What it computes (Sec. 2, eqs. K_TT and K_EE; App. A):
 *
 *   K^X_{l1 l2} = (2 l2 + 1)/(4 pi) sum_{l3} (2 l3 + 1) W^X_{l3} S^X(l1,l2,l3)
 *
 *   S^TT = (l1 l2 l3; 0 0 0)^2
 *   S^TE = [(1+(-1)^L)/2]   (l1 l2 l3; 0 0 0)(l1 l2 l3; -2 2 0)
 *   S^EE = S^BB = [(1+(-1)^L)/2]^2 (l1 l2 l3; -2 2 0)^2
 *   S^EB = [(1-(-1)^L)/2]^2 (l1 l2 l3; -2 2 0)^2,     L = l1 + l2 + l3.
 *
 * How: for every requested (l1, l2) the two rows of 3j symbols over
 * l3 = |l1-l2| .. l1+l2 are produced in long double (x87, 64-bit mantissa)
 * by the Schulten--Gordon three-term recursion in l3, run forward from the
 * lower end and backward from the upper end and joined in the middle, then
 * normalised by the orthogonality sum  sum_l3 (2 l3 + 1) f^2 = 1  and given
 * the sign of the Racah sum at the stretched end l3 = l1 + l2.  The l3 sum of
 * the definition is then taken term by term, in long double.  Each (l1, l2)
 * is evaluated independently; nothing is shared between elements and no
 * symmetry of K is used.  There are no g(p) tables and no closed-form
 * reduction of the (-2 2 0) symbol here: that is the method under test.
 *
 * The recursion.  Write the symbol with the m = 0 column first (an even,
 * cyclic permutation, Sec. 2 eq. permutation):
 *   (l1 l2 l3; m -m 0) = (l3 l1 l2; 0 m -m)  =: f(l3).
 * Schulten & Gordon's recursion in the first argument j of (j j2 j3; m1 m2 m3),
 *   j A(j+1) f(j+1) + B(j) f(j) + (j+1) A(j) f(j-1) = 0,
 *   A(j) = sqrt[(j^2 - (j2-j3)^2)((j2+j3+1)^2 - j^2)(j^2 - m1^2)],
 *   B(j) = -(2j+1)[j2(j2+1) m1 - j3(j3+1) m1 - j(j+1)(m3 - m2)],
 * with m1 = 0, divided through by j(j+1), reads
 *   P(j+1) f(j+1) + Q(j) f(j) + P(j) f(j-1) = 0,
 *   P(j) = sqrt[(j^2 - d^2)(s^2 - j^2)],  d = l1 - l2,  s = l1 + l2 + 1,
 *   Q(j) = (2j+1)(m3 - m2) = -2 m (2j+1),
 * which also holds at j = 0 (the divided form is the one checked against the
 * Racah sum in the tests, including the l1 = l2 rows that start at j = 0).
 *
 * Stretched-end sign: at l3 = l1 + l2 the Racah sum has a single term and the
 * symbol (l3 l1 l2; 0 m -m) has sign (-1)^(l1 + l2).
 *
 * Error metric support: alongside each K element the oracle returns
 * A = (2 l2 + 1)/(4 pi) sum_l3 (2 l3 + 1) |W S|, the scale a relative error
 * is measured against (for TE the terms change sign).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef long double ld;

#define ORACLE_TT 1u
#define ORACLE_TE 2u
#define ORACLE_EE 4u
#define ORACLE_BB 8u
#define ORACLE_EB 16u

static const ld PI_L = 3.141592653589793238462643383279502884L;

/* P(j) of the divided recursion, zero outside the triangle. */
static ld sg_p(long j, long d, long s)
{
    ld a = (ld)j * (ld)j - (ld)d * (ld)d;
    ld b = (ld)s * (ld)s - (ld)j * (ld)j;
    if (a <= 0 || b <= 0) return 0.0L;
    return sqrtl(a * b);
}

/*
 * f[i] = (l1 l2 jmin+i; m -m 0) for i = 0 .. l1+l2-jmin, jmin = |l1-l2|.
 * fw/bw: scratch of the same length.  Returns the row length n.
 */
static long sg_row(int l1, int l2, int m, ld *f, ld *fw, ld *bw)
{
    const long jmin = labs((long)l1 - l2), jmax = (long)l1 + l2;
    const long n = jmax - jmin + 1;
    const long d = (long)l1 - l2, s = (long)l1 + l2 + 1;
    long i;
    if (abs(m) > l1 || abs(m) > l2) {
        for (i = 0; i < n; ++i) f[i] = 0.0L;
        return n;
    }
    if (n == 1) {
        f[0] = 1.0L;
    } else {
        const long im = (n - 1) / 2 - (((n - 1) / 2) & 1); /* even offset: same parity as jmin */
        const long lo = im - 2 < 0 ? 0 : im - 2;
        const long hi = im + 2 > n - 1 ? n - 1 : im + 2;
        for (i = 0; i < n; ++i) fw[i] = bw[i] = 0.0L;
        if (m == 0) {
            /* Q = 0: the recursion links l3 and l3 + 2 only (odd L vanish) */
            fw[0] = 1.0L;
            for (i = 0; i + 2 <= hi; i += 2) {
                long j = jmin + i + 1;
                fw[i + 2] = -sg_p(j, d, s) * fw[i] / sg_p(j + 1, d, s);
            }
            bw[n - 1] = 1.0L;
            for (i = n - 1; i - 2 >= lo; i -= 2) {
                long j = jmin + i - 1;
                bw[i - 2] = -sg_p(j + 1, d, s) * bw[i] / sg_p(j, d, s);
            }
        } else {
            ld prev = 0.0L, cur = 1.0L, p_j = 0.0L, p_j1;
            const ld qm = -2.0L * (ld)m;
            /* forward from jmin; P(jmin) = 0 */
            fw[0] = 1.0L;
            for (i = 0; i < hi; ++i) {
                long j = jmin + i;
                ld nxt;
                p_j1 = sg_p(j + 1, d, s);
                nxt = -(qm * (ld)(2 * j + 1) * cur + p_j * prev) / p_j1;
                fw[i + 1] = nxt;
                prev = cur;
                cur = nxt;
                p_j = p_j1;
            }
            /* backward from jmax; P(jmax + 1) = 0 */
            prev = 0.0L;
            cur = 1.0L;
            p_j1 = 0.0L;
            bw[n - 1] = 1.0L;
            for (i = n - 1; i > lo; --i) {
                long j = jmin + i;
                ld nxt;
                p_j = sg_p(j, d, s);
                nxt = -(qm * (ld)(2 * j + 1) * cur + p_j1 * prev) / p_j;
                bw[i - 1] = nxt;
                prev = cur;
                cur = nxt;
                p_j1 = p_j;
            }
        }
        /* join: least-squares scale of bw onto fw over the points lo..hi */
        {
            ld num = 0.0L, den = 0.0L, scale;
            for (i = lo; i <= hi; ++i) {
                num += fw[i] * bw[i];
                den += bw[i] * bw[i];
            }
            scale = num / den;
            for (i = 0; i <= im; ++i) f[i] = fw[i];
            for (i = im + 1; i < n; ++i) f[i] = scale * bw[i];
        }
    }
    /* normalise: sum (2 l3 + 1) f^2 = 1 over the whole row */
    {
        ld norm = 0.0L;
        for (i = 0; i < n; ++i) norm += (ld)(2 * (jmin + i) + 1) * f[i] * f[i];
        norm = 1.0L / sqrtl(norm);
        /* sign at the stretched end: (-1)^(l1 + l2) */
        if ((((l1 + l2) & 1) ? -1.0L : 1.0L) * f[n - 1] < 0) norm = -norm;
        for (i = 0; i < n; ++i) f[i] *= norm;
    }
    return n;
}

/* (l1 l2 l3; m -m 0) for l3 = |l1-l2| .. l1+l2 into out[0 .. n_out-1] (float64). */
int oracle_threej_row(int l1, int l2, int m, double *out, int n_out)
{
    long n, i;
    ld *buf;
    if (l1 < 0 || l2 < 0 || !out) return -1;
    n = (long)l1 + l2 - labs((long)l1 - l2) + 1;
    if (n_out < n) return -1;
    buf = (ld *)malloc(sizeof(ld) * 3 * (size_t)n);
    if (!buf) return -2;
    sg_row(l1, l2, m, buf, buf + n, buf + 2 * n);
    for (i = 0; i < n; ++i) out[i] = (double)buf[i];
    free(buf);
    return (int)n;
}

static int popcount5(unsigned x)
{
    int c = 0;
    for (; x; x >>= 1) c += (int)(x & 1u);
    return c;
}

/*
 * One K element for every selected spectrum: acc[k] and aab[k] (k in the
 * order TT, TE, EE, BB, EB) receive sum_l3 (2 l3 + 1) W S and the sum of the
 * absolute values of those terms, over l3 in [l3_lo, l3_hi].  x, z: rows of
 * length 2 lmax + 2; fw, bw: scratch of the same length.
 */
static void coupling_element(int l1, int l2, const double *W_TT, const double *W_TP, const double *W_PP,
                             int l3_lo, int l3_hi, unsigned spectra, ld *x, ld *z, ld *fw, ld *bw,
                             ld *acc, ld *aab)
{
    const int need_pol = (spectra & (ORACLE_TE | ORACLE_EE | ORACLE_BB | ORACLE_EB)) != 0;
    const long jmin = labs((long)l1 - l2);
    long n, i;
    int k;
    for (k = 0; k < 5; ++k) acc[k] = aab[k] = 0.0L;
    n = sg_row(l1, l2, 0, x, fw, bw);
    if (need_pol) sg_row(l1, l2, -2, z, fw, bw);
    for (i = 0; i < n; ++i) {
        const long l3 = jmin + i;
        const ld w3 = (ld)(2 * l3 + 1);
        const int even = ((l1 + l2 + l3) & 1L) == 0;
        ld t;
        if (l3 < l3_lo || l3 > l3_hi) continue;
        if (spectra & ORACLE_TT) {
            t = w3 * (ld)W_TT[l3] * x[i] * x[i];
            acc[0] += t; aab[0] += fabsl(t);
        }
        if ((spectra & ORACLE_TE) && even) {
            t = w3 * (ld)W_TP[l3] * x[i] * z[i];
            acc[1] += t; aab[1] += fabsl(t);
        }
        if ((spectra & ORACLE_EE) && even) {
            t = w3 * (ld)W_PP[l3] * z[i] * z[i];
            acc[2] += t; aab[2] += fabsl(t);
        }
        if ((spectra & ORACLE_BB) && even) {
            t = w3 * (ld)W_PP[l3] * z[i] * z[i];
            acc[3] += t; aab[3] += fabsl(t);
        }
        if ((spectra & ORACLE_EB) && !even) {
            t = w3 * (ld)W_PP[l3] * z[i] * z[i];
            acc[4] += t; aab[4] += fabsl(t);
        }
    }
}

/*
 * K rows.  rows[0..n_rows-1] are the l1 values; every l2 in 0..lmax is
 * evaluated, or with `upper` set only l2 >= l1 (the other entries are left
 * 0).  Only l3 in [l3_lo, l3_hi] enter the sum (pass 0 and a large value for
 * the full sum).  Output K_out and A_out (may be NULL) are
 * [n_sel][n_rows][lmax+1] float64, n_sel = popcount(spectra), in the order
 * TT, TE, EE, BB, EB.  Returns 0, or a negative value on bad arguments.
 */
int oracle_coupling_rows_upper(int lmax, const double *W_TT, const double *W_TP, const double *W_PP,
                               int w_len, int l3_lo, int l3_hi, const int *rows, int n_rows,
                               unsigned spectra, double *K_out, double *A_out, int n_threads, int upper)
{
    const int n_sel = popcount5(spectra & 31u);
    const long ncol = (long)lmax + 1;
    int r, err = 0;
    if (lmax < 0 || n_rows < 0 || !rows || !K_out || n_sel == 0) return -1;
    if (w_len < 2 * lmax + 1) return -1;
    if ((spectra & ORACLE_TT) && !W_TT) return -1;
    if ((spectra & ORACLE_TE) && !W_TP) return -1;
    if ((spectra & (ORACLE_EE | ORACLE_BB | ORACLE_EB)) && !W_PP) return -1;
    for (r = 0; r < n_rows; ++r)
        if (rows[r] < 0 || rows[r] > lmax) return -1;
    if (n_threads > 0) omp_set_num_threads(n_threads);
    if (upper) {
        memset(K_out, 0, sizeof(double) * (size_t)n_sel * n_rows * ncol);
        if (A_out) memset(A_out, 0, sizeof(double) * (size_t)n_sel * n_rows * ncol);
    }

#pragma omp parallel reduction(| : err)
    {
        const long len = 2L * lmax + 2;
        ld *x = (ld *)malloc(sizeof(ld) * 3 * (size_t)len);
        ld *z = (ld *)malloc(sizeof(ld) * (size_t)len);
        long task;
        if (!x || !z) err |= 1;
#pragma omp for schedule(dynamic, 4)
        for (task = 0; task < (long)n_rows * ncol; ++task) {
            const int l1 = rows[task / ncol];
            const int l2 = (int)(task % ncol);
            const long ri = task / ncol;
            ld acc[5], aab[5];
            ld pref;
            int k, o;
            if (err || (upper && l2 < l1)) continue;
            coupling_element(l1, l2, W_TT, W_TP, W_PP, l3_lo, l3_hi, spectra, x, z, x + len, x + 2 * len,
                             acc, aab);
            pref = (ld)(2 * l2 + 1) / (4.0L * PI_L);
            for (k = 0, o = 0; k < 5; ++k) {
                if (!(spectra & (1u << k))) continue;
                K_out[((long)o * n_rows + ri) * ncol + l2] = (double)(pref * acc[k]);
                if (A_out) A_out[((long)o * n_rows + ri) * ncol + l2] = (double)(pref * aab[k]);
                ++o;
            }
        }
        free(x);
        free(z);
    }
    return err ? -2 : 0;
}

int oracle_coupling_rows(int lmax, const double *W_TT, const double *W_TP, const double *W_PP,
                         int w_len, int l3_lo, int l3_hi, const int *rows, int n_rows,
                         unsigned spectra, double *K_out, double *A_out, int n_threads)
{
    return oracle_coupling_rows_upper(lmax, W_TT, W_TP, W_PP, w_len, l3_lo, l3_hi, rows, n_rows, spectra,
                                      K_out, A_out, n_threads, 0);
}

/* ------------------------------------------------------------------------
 * Band-limited rows (Sec. 4.3): only l3 <= l3_hi enters the sum, so the row
 * is needed from its lower end jmin = |l1 - l2| up to min(jmax, l3_hi) only.
 * The row is started at jmin with the exact value of the Racah sum there --
 * at the lower end the sum has a single term, evaluated here in log form with
 * lgammal -- and continued upwards by the same Schulten--Gordon recursion
 * (forward is the stable direction out of the lower end).  No normalisation
 * is needed: the seed carries the absolute scale.
 */

/* log|term| and sign of the single-term Racah sum of (j1 j2 j3; m1 m2 m3), or
 * 0 if the sum does not have exactly one term. */
static int racah_single_term(long j1, long j2, long j3, long m1, long m2, long m3, ld *logabs, int *sign)
{
    long t_lo = 0, t_hi, t;
    ld lg;
    if (j2 - j3 - m1 > t_lo) t_lo = j2 - j3 - m1;
    if (j1 - j3 + m2 > t_lo) t_lo = j1 - j3 + m2;
    t_hi = j1 + j2 - j3;
    if (j1 - m1 < t_hi) t_hi = j1 - m1;
    if (j2 + m2 < t_hi) t_hi = j2 + m2;
    if (t_lo != t_hi) return 0;
    t = t_lo;
    /* sqrt(Delta) sqrt(prod (j +- m)!) / denominator factorials */
    lg = 0.5L * (lgammal((ld)(j1 + j2 - j3 + 1)) + lgammal((ld)(j1 - j2 + j3 + 1)) +
                 lgammal((ld)(-j1 + j2 + j3 + 1)) - lgammal((ld)(j1 + j2 + j3 + 2)));
    lg += 0.5L * (lgammal((ld)(j1 + m1 + 1)) + lgammal((ld)(j1 - m1 + 1)) + lgammal((ld)(j2 + m2 + 1)) +
                  lgammal((ld)(j2 - m2 + 1)) + lgammal((ld)(j3 + m3 + 1)) + lgammal((ld)(j3 - m3 + 1)));
    lg -= lgammal((ld)(t + 1)) + lgammal((ld)(j3 - j2 + t + m1 + 1)) + lgammal((ld)(j3 - j1 + t - m2 + 1)) +
          lgammal((ld)(j1 + j2 - j3 - t + 1)) + lgammal((ld)(j1 - t - m1 + 1)) + lgammal((ld)(j2 - t + m2 + 1));
    *logabs = lg;
    *sign = (((j1 - j2 - m3 + t) % 2) != 0) ? -1 : 1;
    return 1;
}

/* f[i] = (l1 l2 jmin+i; m -m 0) for i = 0 .. n_out-1 (n_out <= row length). */
static void sg_row_forward(int l1, int l2, int m, long n_out, ld *f)
{
    const long jmin = labs((long)l1 - l2);
    const long d = (long)l1 - l2, s = (long)l1 + l2 + 1;
    long i;
    ld logabs = 0.0L, prev = 0.0L, cur, p_j = 0.0L;
    int sign = 1;
    if (n_out <= 0) return;
    if (abs(m) > l1 || abs(m) > l2) {
        for (i = 0; i < n_out; ++i) f[i] = 0.0L;
        return;
    }
    /* the symbol with the l3 = jmin column first: (jmin l1 l2; 0 m -m) */
    if (!racah_single_term(jmin, l1, l2, 0, m, -m, &logabs, &sign)) {
        for (i = 0; i < n_out; ++i) f[i] = 0.0L; /* not reached for valid rows */
        return;
    }
    cur = (ld)sign * expl(logabs);
    f[0] = cur;
    for (i = 0; i + 1 < n_out; ++i) {
        const long j = jmin + i;
        const ld p_j1 = sg_p(j + 1, d, s);
        const ld nxt = -(-2.0L * (ld)m * (ld)(2 * j + 1) * cur + p_j * prev) / p_j1;
        f[i + 1] = nxt;
        prev = cur;
        cur = nxt;
        p_j = p_j1;
    }
}

/* (l1 l2 l3; m -m 0) for l3 = |l1-l2| .. min(l1+l2, l3_hi) by the forward
 * recursion from the exact lower end; returns the number written. */
int oracle_threej_row_forward(int l1, int l2, int m, int l3_hi, double *out, int n_out)
{
    long jmin, n, i;
    ld *buf;
    if (l1 < 0 || l2 < 0 || !out) return -1;
    jmin = labs((long)l1 - l2);
    n = ((long)l1 + l2 < l3_hi ? (long)l1 + l2 : l3_hi) - jmin + 1;
    if (n <= 0) return 0;
    if (n_out < n) return -1;
    buf = (ld *)malloc(sizeof(ld) * (size_t)n);
    if (!buf) return -2;
    sg_row_forward(l1, l2, m, n, buf);
    for (i = 0; i < n; ++i) out[i] = (double)buf[i];
    free(buf);
    return (int)n;
}

/* ------------------------------------------------------------------------
 * Rows of (l1 l2 l3; m1 m2 m3) with any magnetic numbers, m3 = -m1 - m2 (the
 * families of the Conclusion, e.g. (1 1 -2) and (2 2 -4), among others).
 *
 * The same Schulten--Gordon recursion, now with m3 != 0 in the first
 * column: f(j) = (j l1 l2; m3 m1 m2), an even cyclic permutation of the
 * symbol, and
 *   j A(j+1) f(j+1) + B(j) f(j) + (j+1) A(j) f(j-1) = 0,
 *   A(j) = sqrt[(j^2 - (l1-l2)^2)((l1+l2+1)^2 - j^2)(j^2 - m3^2)],
 *   B(j) = -(2j+1)[(l1(l1+1) - l2(l2+1)) m3 - j(j+1)(m2 - m1)],
 * over j = max(|l1-l2|, |m3|) .. l1+l2, where A vanishes at the lower end.
 * It is run forward and backward and joined in the middle as in sg_row,
 * normalised by sum_j (2j+1) f^2 = 1 (orthogonality at fixed m1, m2), and
 * given the sign of the single-term Racah sum at the stretched end.  With
 * m3 = 0 the rows of sg_row are used ((l1 l2 l3; m -m 0) with m = m1).
 */
static ld sg_a(long j, long d, long s, long m)
{
    ld a = (ld)j * (ld)j - (ld)d * (ld)d;
    ld b = (ld)s * (ld)s - (ld)j * (ld)j;
    ld c = (ld)j * (ld)j - (ld)m * (ld)m;
    if (a <= 0 || b <= 0 || c <= 0) return 0.0L;
    return sqrtl(a * b * c);
}

/* f[i] = (l1 l2 jlo+i; m1 m2 m3), i < n = l1+l2-jlo+1; fw, bw scratch of n. */
static void sg_row_m(int l1, int l2, int m1, int m2, long jlo, long n, ld *f, ld *fw, ld *bw)
{
    const long m3 = -(long)m1 - m2;
    const long d = (long)l1 - l2, s = (long)l1 + l2 + 1, jmax = (long)l1 + l2;
    const ld kab = (ld)((long)l1 * (l1 + 1) - (long)l2 * (l2 + 1)) * (ld)m3;
    const long im = (n - 1) / 2;
    const long lo = im - 2 < 0 ? 0 : im - 2;
    const long hi = im + 2 > n - 1 ? n - 1 : im + 2;
    long i;
    ld logabs = 0.0L;
    int sign = 1;
    for (i = 0; i < n; ++i) fw[i] = bw[i] = 0.0L;
    /* forward from jlo: A(jlo) = 0 */
    fw[0] = 1.0L;
    for (i = 0; i < hi; ++i) {
        const long j = jlo + i;
        const ld b = -(ld)(2 * j + 1) * (kab - (ld)j * (ld)(j + 1) * (ld)(m2 - m1));
        const ld back = i > 0 ? (ld)(j + 1) * sg_a(j, d, s, m3) * fw[i - 1] : 0.0L;
        fw[i + 1] = -(b * fw[i] + back) / ((ld)j * sg_a(j + 1, d, s, m3));
    }
    /* backward from jmax: A(jmax + 1) = 0 */
    bw[n - 1] = 1.0L;
    for (i = n - 1; i > lo; --i) {
        const long j = jlo + i;
        const ld b = -(ld)(2 * j + 1) * (kab - (ld)j * (ld)(j + 1) * (ld)(m2 - m1));
        const ld fwd = i + 1 < n ? (ld)j * sg_a(j + 1, d, s, m3) * bw[i + 1] : 0.0L;
        bw[i - 1] = -(b * bw[i] + fwd) / ((ld)(j + 1) * sg_a(j, d, s, m3));
    }
    /* join: least-squares scale of bw onto fw over lo..hi */
    {
        ld num = 0.0L, den = 0.0L, scale;
        for (i = lo; i <= hi; ++i) {
            num += fw[i] * bw[i];
            den += bw[i] * bw[i];
        }
        scale = num / den;
        for (i = 0; i <= im; ++i) f[i] = fw[i];
        for (i = im + 1; i < n; ++i) f[i] = scale * bw[i];
    }
    /* normalise and take the sign of the stretched end l3 = l1 + l2 */
    {
        ld norm = 0.0L;
        for (i = 0; i < n; ++i) norm += (ld)(2 * (jlo + i) + 1) * f[i] * f[i];
        norm = 1.0L / sqrtl(norm);
        racah_single_term(l1, l2, jmax, m1, m2, m3, &logabs, &sign);
        if ((ld)sign * f[n - 1] < 0) norm = -norm;
        for (i = 0; i < n; ++i) f[i] *= norm;
    }
}

/* (l1 l2 l3; m1 m2 -m1-m2) for l3 = |l1-l2| .. l1+l2 into out[0 .. n_out-1]
 * (float64); entries with l3 < |m1 + m2| are 0, as is the whole row when
 * |m1| > l1 or |m2| > l2.  Returns the row length. */
int oracle_threej_row_m(int l1, int l2, int m1, int m2, double *out, int n_out)
{
    const long m3 = -(long)m1 - m2;
    long n, jlo, i;
    ld *buf;
    if (l1 < 0 || l2 < 0 || !out) return -1;
    n = (long)l1 + l2 - labs((long)l1 - l2) + 1;
    if (n_out < n) return -1;
    for (i = 0; i < n; ++i) out[i] = 0.0;
    if (abs(m1) > l1 || abs(m2) > l2) return (int)n;
    if (m3 == 0) return oracle_threej_row(l1, l2, m1, out, n_out);
    jlo = labs((long)l1 - l2) > labs(m3) ? labs((long)l1 - l2) : labs(m3);
    if (jlo > (long)l1 + l2) return (int)n;
    buf = (ld *)malloc(sizeof(ld) * 3 * (size_t)(l1 + l2 - jlo + 1));
    if (!buf) return -2;
    {
        const long nr = (long)l1 + l2 - jlo + 1;
        const long off = jlo - labs((long)l1 - l2);
        sg_row_m(l1, l2, m1, m2, jlo, nr, buf, buf + nr, buf + 2 * nr);
        for (i = 0; i < nr; ++i) out[off + i] = (double)buf[i];
    }
    free(buf);
    return (int)n;
}

/*
 * Band-limited K rows: as oracle_coupling_rows with the l3 sum restricted to
 * [l3_lo, l3_hi], but only the l2 with |l1 - l2| <= l3_hi are evaluated (the
 * others have no l3 in the band: their K is exactly 0) and every row is built
 * by the forward recursion up to l3_hi.
 */
int oracle_band_rows(int lmax, const double *W_TT, const double *W_TP, const double *W_PP, int w_len,
                     int l3_lo, int l3_hi, const int *rows, int n_rows, unsigned spectra,
                     double *K_out, double *A_out, int n_threads)
{
    const int n_sel = popcount5(spectra & 31u);
    const long ncol = (long)lmax + 1;
    const int need_pol = (spectra & (ORACLE_TE | ORACLE_EE | ORACLE_BB | ORACLE_EB)) != 0;
    int r, err = 0;
    if (lmax < 0 || n_rows < 0 || !rows || !K_out || n_sel == 0 || l3_lo < 0 || l3_hi < l3_lo) return -1;
    if (w_len < (l3_hi < 2 * lmax ? l3_hi : 2 * lmax) + 1) return -1;
    if ((spectra & ORACLE_TT) && !W_TT) return -1;
    if ((spectra & ORACLE_TE) && !W_TP) return -1;
    if ((spectra & (ORACLE_EE | ORACLE_BB | ORACLE_EB)) && !W_PP) return -1;
    for (r = 0; r < n_rows; ++r)
        if (rows[r] < 0 || rows[r] > lmax) return -1;
    if (n_threads > 0) omp_set_num_threads(n_threads);
    memset(K_out, 0, sizeof(double) * (size_t)n_sel * n_rows * ncol);
    if (A_out) memset(A_out, 0, sizeof(double) * (size_t)n_sel * n_rows * ncol);

#pragma omp parallel reduction(| : err)
    {
        const long len = (long)l3_hi + 2;
        ld *x = (ld *)malloc(sizeof(ld) * (size_t)len);
        ld *z = (ld *)malloc(sizeof(ld) * (size_t)len);
        long task;
        if (!x || !z) err |= 1;
#pragma omp for schedule(dynamic, 4)
        for (task = 0; task < (long)n_rows * ncol; ++task) {
            const int l1 = rows[task / ncol];
            const int l2 = (int)(task % ncol);
            const long ri = task / ncol;
            const long jmin = labs((long)l1 - l2);
            const long jtop = ((long)l1 + l2 < l3_hi) ? (long)l1 + l2 : l3_hi;
            const long n = jtop - jmin + 1;
            long i;
            ld acc[5] = {0, 0, 0, 0, 0}, aab[5] = {0, 0, 0, 0, 0};
            ld pref;
            int k, o;
            if (err || n <= 0) continue;
            sg_row_forward(l1, l2, 0, n, x);
            if (need_pol) sg_row_forward(l1, l2, -2, n, z);
            for (i = 0; i < n; ++i) {
                const long l3 = jmin + i;
                const ld w3 = (ld)(2 * l3 + 1);
                const int even = ((l1 + l2 + l3) & 1L) == 0;
                ld t;
                if (l3 < l3_lo) continue;
                if (spectra & ORACLE_TT) {
                    t = w3 * (ld)W_TT[l3] * x[i] * x[i];
                    acc[0] += t; aab[0] += fabsl(t);
                }
                if ((spectra & ORACLE_TE) && even) {
                    t = w3 * (ld)W_TP[l3] * x[i] * z[i];
                    acc[1] += t; aab[1] += fabsl(t);
                }
                if ((spectra & ORACLE_EE) && even) {
                    t = w3 * (ld)W_PP[l3] * z[i] * z[i];
                    acc[2] += t; aab[2] += fabsl(t);
                }
                if ((spectra & ORACLE_BB) && even) {
                    t = w3 * (ld)W_PP[l3] * z[i] * z[i];
                    acc[3] += t; aab[3] += fabsl(t);
                }
                if ((spectra & ORACLE_EB) && !even) {
                    t = w3 * (ld)W_PP[l3] * z[i] * z[i];
                    acc[4] += t; aab[4] += fabsl(t);
                }
            }
            pref = (ld)(2 * l2 + 1) / (4.0L * PI_L);
            for (k = 0, o = 0; k < 5; ++k) {
                if (!(spectra & (1u << k))) continue;
                K_out[((long)o * n_rows + ri) * ncol + l2] = (double)(pref * acc[k]);
                if (A_out) A_out[((long)o * n_rows + ri) * ncol + l2] = (double)(pref * aab[k]);
                ++o;
            }
        }
        free(x);
        free(z);
    }
    return err ? -2 : 0;
}
