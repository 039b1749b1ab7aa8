/* Oracle (test infrastructure only): ILU(0) of a CSR matrix in its given row
 * order, and the two triangular solves that apply it.
 *
 * The paper's smoother is ILU(0) (Sec. 3.2, Table 1 step 7, citing Saad's
 * "Iterative methods for sparse linear systems").  ILU(0) keeps exactly the
 * sparsity pattern of A: L (unit lower) and U (upper) overwrite A's stored
 * entries.  The factorisation below is the IKJ variant: rows are processed in
 * ascending order; for each k < i stored in row i (ascending), a_ik /= a_kk and
 * every stored a_ij with j > k and (k, j) stored is reduced by a_ik * a_kj.
 *
 * CSR convention: row_ptr int64 [n+1], col int32 sorted within each row with
 * the diagonal present, val float64.
 */
#include <stdint.h>

/* Returns 0 on success, -(i+1) if the pivot of row i is not positive. */
int64_t oracle_ilu0_factor(int64_t n, const int64_t* rp, const int32_t* ci,
                           double* val, int64_t* diag) {
    for (int64_t i = 0; i < n; ++i) {
        diag[i] = -1;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p)
            if (ci[p] == i) { diag[i] = p; break; }
        if (diag[i] < 0) return -(i + 1);
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t p = rp[i]; p < diag[i]; ++p) {
            int64_t k = ci[p];
            val[p] /= val[diag[k]];
            double lik = val[p];
            int64_t a = p + 1, b = diag[k] + 1;
            while (a < rp[i + 1] && b < rp[k + 1]) {
                if (ci[a] == ci[b]) { val[a] -= lik * val[b]; ++a; ++b; }
                else if (ci[a] < ci[b]) ++a;
                else ++b;
            }
        }
        if (!(val[diag[i]] > 0.0)) return -(i + 1);
    }
    return 0;
}

/* x = U^{-1} L^{-1} b (x may alias b). */
void oracle_ilu0_solve(int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                       const int64_t* diag, const double* b, double* x) {
    for (int64_t i = 0; i < n; ++i) {
        double s = b[i];
        for (int64_t p = rp[i]; p < diag[i]; ++p) s -= val[p] * x[ci[p]];
        x[i] = s;
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int64_t p = diag[i] + 1; p < rp[i + 1]; ++p) s -= val[p] * x[ci[p]];
        x[i] = s / val[diag[i]];
    }
}
