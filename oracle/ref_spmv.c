/*
 * CPU oracle for y = A x with A in CSR.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code with the GPU library.
 *
 * What is computed (paper Section 2.1 and Section 3: every storage format the
 * auto-tuner may pick re-encodes the same stored entries, so the result of
 * the method is the plain CSR product):
 *
 *     y_i = sum_{p = row_ptr[i]}^{row_ptr[i+1]-1} val[p] * x[col[p]]
 *
 * Every stored entry counts, explicit zeros included; an empty row gives 0.
 * All arithmetic is IEEE binary64; float32 inputs are widened exactly by the
 * caller before the call.
 *
 * Modes:
 *   accurate  error-free products (TwoProduct via fma) and Neumaier
 *             compensated summation in storage order, plus (|A||x|)_i; this
 *             is the value every parity test compares against.
 *   plain     a naive sequential sum per row, rows split over OpenMP threads
 *             so that each thread holds about the same number of nonzeros,
 *             rounded to whole rows (the paper's multithreaded scheme,
 *             Section 6).  It exists to time a straightforward CPU SpMV;
 *             plain_f32 is the same on float32 storage (binary64 sums,
 *             each row rounded once).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fused
 * multiply-add is introduced behind the code's back; fma() below is
 * explicit and correctly rounded).
 */
#include <math.h>
#include <stdint.h>
#include <omp.h>

/* Accurate mode.  y and absax are written for every row. */
void ref_spmv_accurate(int64_t m, const int64_t *row_ptr, const int32_t *col,
                       const double *val, const double *x, double *y,
                       double *absax)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < m; ++i) {
        double s = 0.0, c = 0.0, a = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            double av = val[p], xv = x[col[p]];
            double prod = av * xv;
            double perr = fma(av, xv, -prod); /* exact: av*xv = prod + perr */
            double t = s + prod;
            if (fabs(s) >= fabs(prod))
                c += (s - t) + prod;
            else
                c += (prod - t) + s;
            s = t;
            c += perr;
            a += fabs(av) * fabs(xv);
        }
        y[i] = s + c;
        absax[i] = a;
    }
}

/* Accurate mode on a subset of rows (rows[k] for k < count). */
void ref_spmv_rows(int64_t count, const int64_t *rows, const int64_t *row_ptr,
                   const int32_t *col, const double *val, const double *x,
                   double *y, double *absax)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < count; ++k) {
        int64_t i = rows[k];
        double s = 0.0, c = 0.0, a = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            double av = val[p], xv = x[col[p]];
            double prod = av * xv;
            double perr = fma(av, xv, -prod);
            double t = s + prod;
            if (fabs(s) >= fabs(prod))
                c += (s - t) + prod;
            else
                c += (prod - t) + s;
            s = t;
            c += perr;
            a += fabs(av) * fabs(xv);
        }
        y[k] = s + c;
        absax[k] = a;
    }
}

/* First row r with row_ptr[r+1] > target, i.e. the row holding nonzero
 * number `target` (or m if target >= nnz). */
static int64_t row_of(int64_t m, const int64_t *row_ptr, int64_t target)
{
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (row_ptr[mid + 1] > target)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

/* Plain mode: naive sum, nnz-balanced contiguous row blocks per thread. */
void ref_spmv_plain(int64_t m, const int64_t *row_ptr, const int32_t *col,
                    const double *val, const double *x, double *y,
                    int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    int64_t nnz = row_ptr[m];
#pragma omp parallel num_threads(nthreads)
    {
        int t = omp_get_thread_num(), T = omp_get_num_threads();
        int64_t r0 = t == 0 ? 0 : row_of(m, row_ptr, (nnz * t) / T);
        int64_t r1 = t == T - 1 ? m : row_of(m, row_ptr, (nnz * (t + 1)) / T);
        for (int64_t i = r0; i < r1; ++i) {
            double s = 0.0;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                s += val[p] * x[col[p]];
            y[i] = s;
        }
    }
}

/* Plain mode on float32 storage (values and x in binary32, as the float32
 * matrices the benchmark times): each product and the running sum in
 * binary64, the row result rounded once to binary32.  For timing. */
void ref_spmv_plain_f32(int64_t m, const int64_t *row_ptr, const int32_t *col,
                        const float *val, const float *x, float *y, int nthreads)
{
    if (nthreads < 1)
        nthreads = 1;
    int64_t nnz = row_ptr[m];
#pragma omp parallel num_threads(nthreads)
    {
        int t = omp_get_thread_num(), T = omp_get_num_threads();
        int64_t r0 = t == 0 ? 0 : row_of(m, row_ptr, (nnz * t) / T);
        int64_t r1 = t == T - 1 ? m : row_of(m, row_ptr, (nnz * (t + 1)) / T);
        for (int64_t i = r0; i < r1; ++i) {
            double s = 0.0;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                s += (double)val[p] * (double)x[col[p]];
            y[i] = (float)s;
        }
    }
}

int ref_max_threads(void) { return omp_get_max_threads(); }
