/*
 * FP64 reference implementation of iALS++ (Rendle, Krichene, Zhang, Koren,
 * "iALS++: Speeding up Matrix Factorization with Subspace Optimization").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or helper
 * with the GPU library, and the library never calls it.
 *
 * Everything is plain double-precision C, written for readability: one OpenMP
 * "parallel for" over independent rows per pass (sec. 3.2: with the other side
 * fixed, the per-row problems are independent), no blocking and no fusion.
 *
 * Notation follows the paper: W (U x d) user embeddings, H (I x d) item
 * embeddings, S the observations (u, i, y, alpha), alpha0 the weight of the
 * all-pairs term, lambda the L2 weight, pi a block of coordinates, yhat the cached
 * prediction per observation.
 *
 * Readings taken where the paper leaves room (each also listed in the design notes):
 *  - the "+ lambda" added to a matrix is lambda times the identity (sec. 4, eq. 9);
 *  - the partial Gramian G^{I,pi} = sum_i h_i (x) h_{i,pi} is d x |pi| (eq. 7);
 *  - alpha0 * w_u G^{I,pi} is the full row w_u (1 x d) times G^{I,pi} (d x |pi|);
 *  - the partition P is contiguous blocks of b coordinates in ascending order,
 *    the last one shorter when b does not divide d;
 *  - the |pi| x |pi| system is solved by Cholesky (the matrix is SPD for lambda > 0);
 *  - yhat is recomputed at the start of every epoch and patched in between;
 *  - the loss uses the identity sum_u sum_i <w_u,h_i>^2 = <W^T W, H^T H>_F, which
 *    follows from eq. 2 and eq. 4 (pinned in the tests against the all-pairs sum).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_OK 0
#define ORA_E_INVALID (-1)
#define ORA_E_NOMEM (-2)
#define ORA_E_NOT_SPD (-4)

/* ------------------------------------------------------------------ */
/* Observation index: sort by (row, col).                               */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t key;
    int64_t idx;
} ora_pair;

static int ora_cmp_pair(const void* a, const void* b) {
    const ora_pair* x = (const ora_pair*)a;
    const ora_pair* y = (const ora_pair*)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return 0;
}

/*
 * Build a CSR view of the observations with rows `row` and columns `col`:
 * rows ascending, columns ascending inside a row.  ptr[nrows+1] gets the row
 * offsets, col_out[nnz] the column of each slot and src[nnz] the index of the
 * observation (in the input arrays) that the slot holds.
 * Returns ORA_E_INVALID on an id out of range or a repeated (row, col) pair.
 */
int ora_build_csr(int64_t nnz, int32_t nrows, int32_t ncols, const int32_t* row,
                  const int32_t* col, int64_t* ptr, int32_t* col_out, int64_t* src) {
    if (nnz < 0 || nrows < 0 || ncols < 0) return ORA_E_INVALID;
    ora_pair* p = (ora_pair*)malloc(sizeof(ora_pair) * (size_t)(nnz > 0 ? nnz : 1));
    if (!p) return ORA_E_NOMEM;
    for (int64_t k = 0; k < nnz; ++k) {
        if (row[k] < 0 || row[k] >= nrows || col[k] < 0 || col[k] >= ncols) {
            free(p);
            return ORA_E_INVALID;
        }
        p[k].key = (int64_t)row[k] * (int64_t)ncols + (int64_t)col[k];
        p[k].idx = k;
    }
    qsort(p, (size_t)nnz, sizeof(ora_pair), ora_cmp_pair);
    for (int64_t k = 1; k < nnz; ++k) {
        if (p[k].key == p[k - 1].key) {
            free(p);
            return ORA_E_INVALID;
        }
    }
    for (int32_t r = 0; r <= nrows; ++r) ptr[r] = 0;
    for (int64_t k = 0; k < nnz; ++k) {
        int64_t r = p[k].key / ncols;
        ptr[r + 1] += 1;
        col_out[k] = (int32_t)(p[k].key % ncols);
        src[k] = p[k].idx;
    }
    for (int32_t r = 0; r < nrows; ++r) ptr[r + 1] += ptr[r];
    free(p);
    return ORA_OK;
}

/* ------------------------------------------------------------------ */
/* Model, Gramian, loss                                                 */
/* ------------------------------------------------------------------ */

/* yhat[k] = <w_u, h_i> for every slot k of the user-side CSR (eq. 1). */
void ora_predict(int32_t num_users, int32_t d, const int64_t* uptr, const int32_t* ucol,
                 const double* W, const double* H, double* yhat) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int32_t u = 0; u < num_users; ++u) {
        const double* w = W + (size_t)u * d;
        for (int64_t k = uptr[u]; k < uptr[u + 1]; ++k) {
            const double* h = H + (size_t)ucol[k] * d;
            double s = 0.0;
            for (int32_t f = 0; f < d; ++f) s += w[f] * h[f];
            yhat[k] = s;
        }
    }
}

/* G (d x bw, row-major) = sum_r x_r (x) x_{r, p0:p0+bw}: the partial Gramian of eq. 7.
 * With p0 = 0 and bw = d this is the full Gramian of eq. 4.  Every entry is summed
 * over r in ascending order; the rows r are walked in the outer loop so that X is
 * read row by row (each thread owns a range of output rows f). */
void ora_gramian(int32_t n, int32_t d, const double* X, int32_t p0, int32_t bw, double* G) {
#pragma omp parallel
    {
#pragma omp for schedule(static)
        for (int32_t f = 0; f < d; ++f)
            for (int32_t q = 0; q < bw; ++q) G[(size_t)f * bw + q] = 0.0;
        /* the same static split of f as above: a thread only touches its own rows of G */
#pragma omp for schedule(static)
        for (int32_t f0 = 0; f0 < d; f0 += 16) {
            const int32_t f1 = f0 + 16 < d ? f0 + 16 : d;
            for (int32_t r = 0; r < n; ++r) {
                const double* x = X + (size_t)r * d;
                for (int32_t f = f0; f < f1; ++f)
                    for (int32_t q = 0; q < bw; ++q) G[(size_t)f * bw + q] += x[f] * x[p0 + q];
            }
        }
    }
}

/* Loss of eq. 2 with a freshly computed prediction for every observation.
 * y and a are per user-CSR slot; NULL means all ones.
 * parts[0] = observed term, parts[1] = alpha0 * all-pairs term, parts[2] = lambda * norms. */
double ora_loss(int32_t num_users, int32_t num_items, int32_t d, const int64_t* uptr,
                const int32_t* ucol, const double* y, const double* a, const double* W,
                const double* H, double alpha0, double lambda, double* parts) {
    double obs = 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : obs)
    for (int32_t u = 0; u < num_users; ++u) {
        const double* w = W + (size_t)u * d;
        for (int64_t k = uptr[u]; k < uptr[u + 1]; ++k) {
            const double* h = H + (size_t)ucol[k] * d;
            double s = 0.0;
            for (int32_t f = 0; f < d; ++f) s += w[f] * h[f];
            double yk = y ? y[k] : 1.0;
            double ak = a ? a[k] : 1.0;
            obs += ak * (s - yk) * (s - yk);
        }
    }
    double* GW = (double*)malloc(sizeof(double) * (size_t)d * d);
    double* GH = (double*)malloc(sizeof(double) * (size_t)d * d);
    if (!GW || !GH) {
        free(GW);
        free(GH);
        return NAN;
    }
    ora_gramian(num_users, d, W, 0, d, GW);
    ora_gramian(num_items, d, H, 0, d, GH);
    double allp = 0.0, reg = 0.0;
    for (int64_t k = 0; k < (int64_t)d * d; ++k) allp += GW[k] * GH[k];
    for (int32_t f = 0; f < d; ++f) reg += GW[(size_t)f * d + f] + GH[(size_t)f * d + f];
    free(GW);
    free(GH);
    if (parts) {
        parts[0] = obs;
        parts[1] = alpha0 * allp;
        parts[2] = lambda * reg;
    }
    return obs + alpha0 * allp + lambda * reg;
}

/* ------------------------------------------------------------------ */
/* Block step (sec. 4, eq. 8-9, Algorithm 3)                            */
/* ------------------------------------------------------------------ */

/* In-place Cholesky A = L L^T of an n x n SPD matrix (lower triangle used and
 * overwritten).  Returns 0, or -1 if a pivot is not positive. */
static int ora_cholesky(int32_t n, double* A) {
    for (int32_t j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int32_t k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(s > 0.0)) return -1;
        double ljj = sqrt(s);
        A[(size_t)j * n + j] = ljj;
        for (int32_t i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int32_t k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = t / ljj;
        }
    }
    return 0;
}

/* Solve L L^T x = b in place (b becomes x). */
static void ora_cholesky_solve(int32_t n, const double* L, double* b) {
    for (int32_t i = 0; i < n; ++i) {
        double t = b[i];
        for (int32_t k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * b[k];
        b[i] = t / L[(size_t)i * n + i];
    }
    for (int32_t i = n - 1; i >= 0; --i) {
        double t = b[i];
        for (int32_t k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * b[k];
        b[i] = t / L[(size_t)i * n + i];
    }
}

/*
 * One row of a block pass: the Newton step on x_{r,pi} of sec. 4 for the row x_r
 * of the side being updated (w_u for users, h_i for items), with the other side
 * X_o fixed.  Slots [lo, hi) of the CSR hold the row's observations; col[k] is the
 * partner, slot[k] (or k when slot is NULL) its position in yhat / y / a.
 *   grad = alpha0 * x_r G + lambda * x_{r,pi} + sum_k a_k (yhat_k - y_k) x_{o,pi}
 *   hess = alpha0 * G_{pi,pi} + lambda I + sum_k a_k x_{o,pi} (x) x_{o,pi}
 *   delta = hess^{-1} grad;  x_{r,pi} -= delta;  yhat_k -= <delta, x_{o,pi}>
 * A, g are caller scratch of bw*bw and bw doubles.  Returns 0 or -1 (not SPD).
 */
static int ora_row_step(int32_t d, int32_t p0, int32_t bw, double alpha0, double lambda,
                        int64_t lo, int64_t hi, const int32_t* col, const int32_t* slot,
                        const double* y, const double* a, double* x, const double* Xo,
                        const double* G, double* yhat, double* A, double* g) {
    for (int32_t q = 0; q < bw; ++q) {
        double s = 0.0;
        for (int32_t f = 0; f < d; ++f) s += x[f] * G[(size_t)f * bw + q];
        g[q] = alpha0 * s + lambda * x[p0 + q];
    }
    for (int32_t p = 0; p < bw; ++p)
        for (int32_t q = 0; q < bw; ++q)
            A[(size_t)p * bw + q] = alpha0 * G[(size_t)(p0 + p) * bw + q] + (p == q ? lambda : 0.0);
    for (int64_t k = lo; k < hi; ++k) {
        int64_t s = slot ? (int64_t)slot[k] : k;
        const double* h = Xo + (size_t)col[k] * d + p0;
        double ak = a ? a[s] : 1.0;
        double yk = y ? y[s] : 1.0;
        double res = ak * (yhat[s] - yk);
        for (int32_t q = 0; q < bw; ++q) g[q] += res * h[q];
        for (int32_t p = 0; p < bw; ++p)
            for (int32_t q = 0; q < bw; ++q) A[(size_t)p * bw + q] += ak * h[p] * h[q];
    }
    if (ora_cholesky(bw, A) != 0) return -1;
    ora_cholesky_solve(bw, A, g); /* g now holds delta */
    for (int32_t q = 0; q < bw; ++q) x[p0 + q] -= g[q];
    for (int64_t k = lo; k < hi; ++k) {
        int64_t s = slot ? (int64_t)slot[k] : k;
        const double* h = Xo + (size_t)col[k] * d + p0;
        double dot = 0.0;
        for (int32_t q = 0; q < bw; ++q) dot += g[q] * h[q];
        yhat[s] -= dot;
    }
    return 0;
}

/*
 * One (block, side) pass of Algorithm 3 given the partial Gramian G (d x bw) of
 * the other side: every row of Xt gets its block step.  ptr/col/slot describe
 * the side's CSR (slot NULL: the CSR order is the yhat order).  y and a are
 * indexed by yhat position.  Returns the number of rows whose Hessian was not
 * positive definite (0 expected); those rows are left unchanged.
 */
int64_t ora_pass(int32_t nrows, int32_t d, int32_t p0, int32_t bw, double alpha0, double lambda,
                 const int64_t* ptr, const int32_t* col, const int32_t* slot, const double* y,
                 const double* a, double* Xt, const double* Xo, const double* G, double* yhat) {
    int64_t bad = 0;
#pragma omp parallel reduction(+ : bad)
    {
        double* A = (double*)malloc(sizeof(double) * (size_t)bw * bw);
        double* g = (double*)malloc(sizeof(double) * (size_t)bw);
        if (!A || !g) {
            bad += nrows;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int32_t r = 0; r < nrows; ++r) {
                if (ora_row_step(d, p0, bw, alpha0, lambda, ptr[r], ptr[r + 1], col, slot, y, a,
                                 Xt + (size_t)r * d, Xo, G, yhat, A, g) != 0)
                    bad += 1;
            }
        }
        free(A);
        free(g);
    }
    return bad;
}

/*
 * The same pass restricted to the rows listed in rows[0..nsel): rows are
 * independent within a pass (sec. 3.2), so each listed row gets exactly the
 * block step the full pass would give it.  Used to check single rows of
 * workloads too large for a full float64 pass.
 */
int64_t ora_pass_rows(int32_t nsel, const int32_t* rows, int32_t d, int32_t p0, int32_t bw, double alpha0,
                      double lambda, const int64_t* ptr, const int32_t* col, const int32_t* slot,
                      const double* y, const double* a, double* Xt, const double* Xo, const double* G,
                      double* yhat) {
    int64_t bad = 0;
#pragma omp parallel reduction(+ : bad)
    {
        double* A = (double*)malloc(sizeof(double) * (size_t)bw * bw);
        double* g = (double*)malloc(sizeof(double) * (size_t)bw);
        if (!A || !g) {
            bad += nsel;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int32_t s = 0; s < nsel; ++s) {
                const int32_t r = rows[s];
                if (ora_row_step(d, p0, bw, alpha0, lambda, ptr[r], ptr[r + 1], col, slot, y, a,
                                 Xt + (size_t)r * d, Xo, G, yhat, A, g) != 0)
                    bad += 1;
            }
        }
        free(A);
        free(g);
    }
    return bad;
}

/*
 * Full epochs of Algorithm 3.  uptr/ucol: user CSR (yhat order); iptr/icol: item
 * CSR with iperm[k] = user-CSR slot of item slot k.  y, a per user-CSR slot
 * (NULL = ones).  W, H updated in place; yhat (nnz) is scratch and holds the
 * final cached predictions.  loss_out (n_epochs, nullable) gets eq. 2 after each
 * epoch.  Returns 0, ORA_E_NOT_SPD or ORA_E_NOMEM.
 */
int ora_epochs(int32_t num_users, int32_t num_items, int32_t d, int32_t b, double alpha0,
               double lambda, const int64_t* uptr, const int32_t* ucol, const int64_t* iptr,
               const int32_t* icol, const int32_t* iperm, const double* y, const double* a,
               double* W, double* H, double* yhat, int32_t n_epochs, double* loss_out) {
    if (b <= 0 || d <= 0) return ORA_E_INVALID;
    double* G = (double*)malloc(sizeof(double) * (size_t)d * b);
    if (!G) return ORA_E_NOMEM;
    int status = ORA_OK;
    for (int32_t t = 0; t < n_epochs && status == ORA_OK; ++t) {
        ora_predict(num_users, d, uptr, ucol, W, H, yhat);
        for (int32_t p0 = 0; p0 < d; p0 += b) {
            int32_t bw = (p0 + b <= d) ? b : d - p0;
            ora_gramian(num_items, d, H, p0, bw, G);
            if (ora_pass(num_users, d, p0, bw, alpha0, lambda, uptr, ucol, NULL, y, a, W, H, G,
                         yhat) != 0) {
                status = ORA_E_NOT_SPD;
                break;
            }
            ora_gramian(num_users, d, W, p0, bw, G);
            if (ora_pass(num_items, d, p0, bw, alpha0, lambda, iptr, icol, iperm, y, a, H, W, G,
                         yhat) != 0) {
                status = ORA_E_NOT_SPD;
                break;
            }
        }
        if (loss_out)
            loss_out[t] = ora_loss(num_users, num_items, d, uptr, ucol, y, a, W, H, alpha0, lambda,
                                   NULL);
    }
    free(G);
    return status;
}

/*
 * Fold-in of new users against a fixed item table H (num_items x d) and its
 * full Gramian GH (d x d): w starts at 0 (so yhat starts at 0) and gets `passes`
 * sweeps of block steps over the blocks in ascending order, each the user-side
 * step of Algorithm 3 for this one row with H fixed.  Request r holds the items
 * items[req_ptr[r] .. req_ptr[r+1]) with labels y (NULL = ones) and weights 1.
 * w_out is n_req x d.  Returns 0, ORA_E_INVALID or ORA_E_NOT_SPD.
 */
int ora_foldin(int32_t num_items, int32_t d, int32_t b, double alpha0, double lambda,
               const double* H, const double* GH, int32_t n_req, const int64_t* req_ptr,
               const int32_t* items, const double* y, int32_t passes, double* w_out) {
    if (b <= 0 || d <= 0 || passes < 0) return ORA_E_INVALID;
    for (int32_t r = 0; r < n_req; ++r)
        for (int64_t k = req_ptr[r]; k < req_ptr[r + 1]; ++k)
            if (items[k] < 0 || items[k] >= num_items) return ORA_E_INVALID;
    int status = ORA_OK;
#pragma omp parallel
    {
        double* A = (double*)malloc(sizeof(double) * (size_t)b * b);
        double* g = (double*)malloc(sizeof(double) * (size_t)b);
        double* G = (double*)malloc(sizeof(double) * (size_t)d * b);
#pragma omp for schedule(dynamic, 4)
        for (int32_t r = 0; r < n_req; ++r) {
            int64_t lo = req_ptr[r], hi = req_ptr[r + 1];
            double* w = w_out + (size_t)r * d;
            double* yh = (double*)calloc((size_t)(hi - lo > 0 ? hi - lo : 1), sizeof(double));
            for (int32_t f = 0; f < d; ++f) w[f] = 0.0;
            for (int32_t it = 0; it < passes; ++it) {
                for (int32_t p0 = 0; p0 < d; p0 += b) {
                    int32_t bw = (p0 + b <= d) ? b : d - p0;
                    for (int32_t f = 0; f < d; ++f)
                        for (int32_t q = 0; q < bw; ++q)
                            G[(size_t)f * bw + q] = GH[(size_t)f * d + p0 + q];
                    /* the row's own slots are 0..n-1 of yh; y is offset to this request */
                    if (ora_row_step(d, p0, bw, alpha0, lambda, 0, hi - lo, items + lo, NULL,
                                     y ? y + lo : NULL, NULL, w, H, G, yh, A, g) != 0) {
#pragma omp atomic write
                        status = ORA_E_NOT_SPD;
                    }
                }
            }
            free(yh);
        }
        free(A);
        free(g);
        free(G);
    }
    return status;
}
