/*
 * ref.c -- CPU oracle loops for y = A x (test infrastructure only).
 *
 * This file is part of the oracle: a plain, sequential, obviously correct statement of what the
 * GPU library computes.  Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * it; the library never links, loads or calls it, and it shares no code with the GPU path.
 *
 * Build with -ffp-contract=off so that every multiply and add below rounds separately, as
 * written.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>

/*
 * Sum runs of repeated coordinates (the paper leaves repeats unspecified; they are summed).
 * Run r covers sorted positions [run_start[r], run_start[r+1]); the values taken are
 * val[perm[k]] in increasing k, which is increasing original triplet index because the sort that
 * produced perm is stable.  The sum starts from the run's first value: ((v0 + v1) + v2) + ...
 */
void ref_sum_runs(int64_t nruns, const int64_t* run_start, const int64_t* perm,
                  const double* val, double* out) {
    for (int64_t r = 0; r < nruns; ++r) {
        int64_t k = run_start[r];
        double acc = val[perm[k]];
        for (++k; k < run_start[r + 1]; ++k) acc = acc + val[perm[k]];
        out[r] = acc;
    }
}

/*
 * Algorithm 1 (SpMV for the CRS format, Section 2): y = 0, then for every row i and every k in
 * [row_ptr[i], row_ptr[i+1]): y[i] = y[i] + data[k] * x[col_ind[k]].
 */
void ref_alg1(int64_t m, const int64_t* row_ptr, const int32_t* col_ind, const double* data,
              const double* x, double* y) {
    for (int64_t i = 0; i < m; ++i) y[i] = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int32_t j = col_ind[k];
            y[i] = y[i] + data[k] * x[j];
        }
    }
}

/*
 * ParCRS (Section 5.1): the rows of Algorithm 1 shared among OpenMP threads in dynamic chunks of
 * `chunk` rows.  Each row is still summed by one thread in increasing k, so y equals Algorithm 1
 * bit for bit; only the wall time changes.  Returns the number of threads used.
 */
int ref_parcrs(int64_t m, const int64_t* row_ptr, const int32_t* col_ind, const double* data,
               const double* x, double* y, int64_t chunk) {
    int used = 1;
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, chunk)
        for (int64_t i = 0; i < m; ++i) {
            double acc = 0.0;
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) acc = acc + data[k] * x[col_ind[k]];
            y[i] = acc;
        }
    }
    return used;
}

/*
 * Algorithm 1 with an accurate reference beside it.  For each row, in the same k order:
 *   y_plain[i] : Algorithm 1 exactly as above;
 *   y_ref[i]   : the same dot product summed accurately -- each product is split into its
 *                rounded value p and exact rounding error e = fma(a, x, -p) (Dekker's
 *                TwoProduct), and p and e are accumulated with Neumaier's compensated sum
 *                (Neumaier 1974, an improved Kahan-Babuska summation);
 *   scale[i]   : sum over k of |data[k]| * |x[col_ind[k]]|, the row's magnitude.
 * Rows with no entries give +0 in all three.
 */
void ref_alg1_accurate(int64_t m, const int64_t* row_ptr, const int32_t* col_ind,
                       const double* data, const double* x, double* y_plain, double* y_ref,
                       double* scale) {
    for (int64_t i = 0; i < m; ++i) {
        double plain = 0.0, s = 0.0, c = 0.0, mag = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            double a = data[k], b = x[col_ind[k]];
            double p = a * b;
            double e = fma(a, b, -p);
            plain = plain + p;
            /* Neumaier step for p */
            double t = s + p;
            if (fabs(s) >= fabs(p)) c += (s - t) + p; else c += (p - t) + s;
            s = t;
            /* the product's rounding error joins the compensation term */
            c += e;
            mag = mag + fabs(a) * fabs(b);
        }
        y_plain[i] = plain;
        y_ref[i] = s + c;
        scale[i] = mag;
    }
}

/*
 * Triplet SpMV (equation in Section 2): y = 0, then y[row_ind[i]] += data[i] * x[col_ind[i]] for
 * i = 0 .. nnz-1 in the given order.  An independent path from coordinates to y.
 */
void ref_triplet_spmv(int64_t nnz, const int32_t* row_ind, const int32_t* col_ind,
                      const double* data, const double* x, int64_t m, double* y) {
    for (int64_t i = 0; i < m; ++i) y[i] = 0.0;
    for (int64_t i = 0; i < nnz; ++i) y[row_ind[i]] = y[row_ind[i]] + data[i] * x[col_ind[i]];
}
