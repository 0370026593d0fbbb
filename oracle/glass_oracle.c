/*
 * glass_oracle.c -- plain FP64 CPU oracle for the batched small dense linear
 * algebra path (GEMM, GEMV, Cholesky factor / solve, triangular solve, SE(3)
 * compose / inverse), following the GLASS paper (Sec. III-B lists the
 * operation families: BLAS L2/L3, triangular solves, factorizations, linear
 * solves, SE(3) maps; Sec. III-C says each is checked against an independent
 * reference).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU path.
 *
 * Conventions (the paper fixes no layout; one reading is used everywhere):
 *   - every matrix is row-major, batch-contiguous: X[b][row][col];
 *   - double precision throughout, plain loops, ascending summation,
 *     no blocking, no BLAS/LAPACK calls;
 *   - Cholesky is lower: A = L L^T; the strict upper part of the output is
 *     written as +0.0; a failing pivot (s <= 0 or NaN) stops the problem and
 *     sets info = j+1 (LAPACK convention, 1-based), columns >= j unspecified.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC
 * (-ffp-contract=off keeps every product and sum a separately rounded
 * double operation, so the summation order written here is the one executed).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OIDX(b, sz) ((size_t)(b) * (size_t)(sz))

/* Number of OpenMP threads the oracle will use (1 when built without it). */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ---------------------------------------------------------------- GEMM --
 * Sec. III-B (BLAS L3).  C = alpha * A B + beta * C with A m x k, B k x n,
 * C m x n.  beta == 0 means C is not read (BLAS convention).             */
void oracle_gemm(int m, int n, int k, int batch, double alpha,
                 const double* A, const double* B, double beta, double* C) {
    long long bb;
#pragma omp parallel for schedule(static)
    for (bb = 0; bb < batch; ++bb) {
        const double* a = A + OIDX(bb, m * k);
        const double* b = B + OIDX(bb, k * n);
        double* c = C + OIDX(bb, m * n);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int p = 0; p < k; ++p) s += a[i * k + p] * b[p * n + j];
                double out = alpha * s;
                if (beta != 0.0) out += beta * c[i * n + j];
                c[i * n + j] = out;
            }
    }
}

/* ---------------------------------------------------------------- GEMV --
 * Sec. III-B (BLAS L2).  y = alpha * A x + beta * y, A m x n.           */
void oracle_gemv(int m, int n, int batch, double alpha, const double* A,
                 const double* x, double beta, double* y) {
    long long bb;
#pragma omp parallel for schedule(static)
    for (bb = 0; bb < batch; ++bb) {
        const double* a = A + OIDX(bb, m * n);
        const double* xv = x + OIDX(bb, n);
        double* yv = y + OIDX(bb, m);
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = 0; j < n; ++j) s += a[i * n + j] * xv[j];
            double out = alpha * s;
            if (beta != 0.0) out += beta * yv[i];
            yv[i] = out;
        }
    }
}

/* One Cholesky factorisation (Cholesky-Crout, column by column).
 * Reads only the lower triangle of a (n x n, row-major), overwrites it with
 * L and zeroes the strict upper triangle.  Returns info (0 or j+1).       */
static int chol_one(int n, double* a) {
    for (int j = 0; j < n; ++j) {
        double s = a[j * n + j];
        for (int p = 0; p < j; ++p) s -= a[j * n + p] * a[j * n + p];
        if (!(s > 0.0)) return j + 1;
        double ljj = sqrt(s);
        a[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = a[i * n + j];
            for (int p = 0; p < j; ++p) t -= a[i * n + p] * a[j * n + p];
            a[i * n + j] = t / ljj;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) a[i * n + j] = 0.0;
    return 0;
}

/* Forward then backward substitution with L (lower, non-unit) for every
 * column of b (n x r, row-major): b <- (L L^T)^{-1} b.                    */
static void chol_solve_one(int n, int r, const double* l, double* b) {
    for (int c = 0; c < r; ++c) {
        for (int i = 0; i < n; ++i) {          /* L y = b */
            double t = b[i * r + c];
            for (int p = 0; p < i; ++p) t -= l[i * n + p] * b[p * r + c];
            b[i * r + c] = t / l[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {     /* L^T x = y */
            double t = b[i * r + c];
            for (int p = i + 1; p < n; ++p) t -= l[p * n + i] * b[p * r + c];
            b[i * r + c] = t / l[i * n + i];
        }
    }
}

/* --------------------------------------------------------------- POTRF --
 * Sec. III-B (factorizations).  info may be NULL.                       */
void oracle_potrf(int n, int batch, double* A, int32_t* info) {
    long long bb;
#pragma omp parallel for schedule(static)
    for (bb = 0; bb < batch; ++bb) {
        int inf = chol_one(n, A + OIDX(bb, n * n));
        if (info) info[bb] = inf;
    }
}

/* --------------------------------------------------------------- POTRS --
 * Sec. III-B (linear solves).  B[b] is n x nrhs, overwritten by X.      */
void oracle_potrs(int n, int nrhs, int batch, const double* L, double* B) {
    long long bb;
#pragma omp parallel for schedule(static)
    for (bb = 0; bb < batch; ++bb)
        chol_solve_one(n, nrhs, L + OIDX(bb, n * n), B + OIDX(bb, n * nrhs));
}

/* ---------------------------------------------------------------- POSV --
 * Sec. III-B and the POSV call of Sec. III-A: factor then solve.  When a
 * problem's factorisation fails its solution is left unspecified (here:
 * B untouched).                                                          */
void oracle_posv(int n, int nrhs, int batch, double* A, double* B, int32_t* info) {
    long long bb;
#pragma omp parallel for schedule(static)
    for (bb = 0; bb < batch; ++bb) {
        double* a = A + OIDX(bb, n * n);
        int inf = chol_one(n, a);
        if (info) info[bb] = inf;
        if (inf == 0) chol_solve_one(n, nrhs, a, B + OIDX(bb, n * nrhs));
    }
}

/* ---------------------------------------------------------------- TRSV --
 * Sec. III-B (triangular solves).  L lower, non-unit diagonal, only the
 * lower triangle is read.  trans = 0: L x = b (forward substitution);
 * trans = 1: L^T x = b (backward substitution).  x holds b on entry.     */
void oracle_trsv(int n, int batch, int trans, const double* L, double* x) {
    long long bb;
#pragma omp parallel for schedule(static)
    for (bb = 0; bb < batch; ++bb) {
        const double* l = L + OIDX(bb, n * n);
        double* v = x + OIDX(bb, n);
        if (trans == 0) {
            for (int i = 0; i < n; ++i) {
                double t = v[i];
                for (int p = 0; p < i; ++p) t -= l[i * n + p] * v[p];
                v[i] = t / l[i * n + i];
            }
        } else {
            for (int i = n - 1; i >= 0; --i) {
                double t = v[i];
                for (int p = i + 1; p < n; ++p) t -= l[p * n + i] * v[p];
                v[i] = t / l[i * n + i];
            }
        }
    }
}

/* ---------------------------------------------------------------- SE(3) --
 * Sec. III-B (SE(3) maps).  A homogeneous transform is the 4x4 row-major
 * matrix [R t; 0 0 0 1].  Compose: T = Ta Tb, i.e. R = Ra Rb,
 * t = Ra tb + ta.  Inverse (closed form for a rigid motion): R' = Ra^T,
 * t' = -Ra^T ta.  Row 3 of the output is written as exactly (0,0,0,1);
 * row 3 of the inputs is never read.                                    */
void oracle_se3_compose(int batch, const double* Ta, const double* Tb, double* T) {
    long long bb;
#pragma omp parallel for schedule(static)
    for (bb = 0; bb < batch; ++bb) {
        const double* a = Ta + OIDX(bb, 16);
        const double* b = Tb + OIDX(bb, 16);
        double o[16];
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int p = 0; p < 3; ++p) s += a[i * 4 + p] * b[p * 4 + j];
                o[i * 4 + j] = s;
            }
            double s = 0.0;
            for (int p = 0; p < 3; ++p) s += a[i * 4 + p] * b[p * 4 + 3];
            o[i * 4 + 3] = s + a[i * 4 + 3];
        }
        o[12] = 0.0; o[13] = 0.0; o[14] = 0.0; o[15] = 1.0;
        memcpy(T + OIDX(bb, 16), o, sizeof o);
    }
}

void oracle_se3_inverse(int batch, const double* Ta, double* T) {
    long long bb;
#pragma omp parallel for schedule(static)
    for (bb = 0; bb < batch; ++bb) {
        const double* a = Ta + OIDX(bb, 16);
        double o[16];
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) o[i * 4 + j] = a[j * 4 + i];
            double s = 0.0;
            for (int p = 0; p < 3; ++p) s += a[p * 4 + i] * a[p * 4 + 3];
            o[i * 4 + 3] = -s;
        }
        o[12] = 0.0; o[13] = 0.0; o[14] = 0.0; o[15] = 1.0;
        memcpy(T + OIDX(bb, 16), o, sizeof o);
    }
}

/* ------------------------------------------------------- POSV adjoint --
 * Reverse mode of the Cholesky solve X = A^{-1} B (A symmetric positive
 * definite, B n x r), for a scalar loss with upstream gradient G = dl/dX:
 *   dB = A^{-1} G               (a second solve with the same factor)
 *   dA = -(1/2) (dB X^T + X dB^T)
 * The symmetric form is the gradient restricted to symmetric perturbations
 * of A (A enters only through its lower triangle, and the factorization
 * treats it as symmetric).  L is A's Cholesky factor, X the solution.      */
void oracle_posv_adjoint(int n, int nrhs, int batch, const double* L, const double* X,
                         const double* G, double* dB, double* dA) {
    long long bb;
#pragma omp parallel for schedule(static)
    for (bb = 0; bb < batch; ++bb) {
        const double* l = L + OIDX(bb, n * n);
        const double* x = X + OIDX(bb, n * nrhs);
        double* db = dB + OIDX(bb, n * nrhs);
        double* da = dA + OIDX(bb, n * n);
        memcpy(db, G + OIDX(bb, n * nrhs), sizeof(double) * (size_t)n * nrhs);
        chol_solve_one(n, nrhs, l, db);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int c = 0; c < nrhs; ++c) s += db[i * nrhs + c] * x[j * nrhs + c] + x[i * nrhs + c] * db[j * nrhs + c];
                da[i * n + j] = -0.5 * s;
            }
    }
}

/* ------------------------------------------------------- GEMM, transposed --
 * C = alpha op(A) op(B) + beta C with op(X) = X or X^T (BLAS convention).
 * op(A) is m x k, op(B) is k x n; A is stored m x k (transa = 0) or k x m
 * (transa = 1), B k x n or n x k.  beta == 0: C is not read.             */
void oracle_gemm_t(int transa, int transb, int m, int n, int k, int batch, double alpha,
                   const double* A, const double* B, double beta, double* C) {
    long long bb;
#pragma omp parallel for schedule(static)
    for (bb = 0; bb < batch; ++bb) {
        const double* a = A + OIDX(bb, m * k);
        const double* b = B + OIDX(bb, k * n);
        double* c = C + OIDX(bb, m * n);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) {
                double s = 0.0;
                for (int p = 0; p < k; ++p) {
                    const double av = transa ? a[p * m + i] : a[i * k + p];
                    const double bv = transb ? b[j * k + p] : b[p * n + j];
                    s += av * bv;
                }
                c[i * n + j] = beta == 0.0 ? alpha * s : alpha * s + beta * c[i * n + j];
            }
    }
}

/* ------------------------------------------------------------- LQR gain --
 * Sec. III-B / Sec. IV-E: the feedback gain K = (R + B^T P B)^{-1} B^T P A
 * of one Riccati step, A nx x nx, B nx x nu, P nx x nx, R nu x nu,
 * K nu x nx.  Written out as its definition: S = R + B^T (P B) and
 * T = B^T (P A) by plain sums, then K = S^{-1} T by Cholesky of S (S is
 * symmetric positive definite when R is and P is semidefinite) and
 * forward / backward substitution for every column of T.  info is the
 * Cholesky info of S (K unspecified where it is nonzero).                 */
void oracle_riccati_gain(int nx, int nu, int batch, const double* A, const double* B,
                         const double* P, const double* R, double* K, int32_t* info) {
    long long bb;
#pragma omp parallel for schedule(static)
    for (bb = 0; bb < batch; ++bb) {
        const double* a = A + OIDX(bb, nx * nx);
        const double* b = B + OIDX(bb, nx * nu);
        const double* p = P + OIDX(bb, nx * nx);
        const double* r = R + OIDX(bb, nu * nu);
        double* kk = K + OIDX(bb, nu * nx);
        double* pb = (double*)malloc(sizeof(double) * (size_t)nx * nu);
        double* pa = (double*)malloc(sizeof(double) * (size_t)nx * nx);
        double* s = (double*)malloc(sizeof(double) * (size_t)nu * nu);
        for (int i = 0; i < nx; ++i) {
            for (int j = 0; j < nu; ++j) {
                double t = 0.0;
                for (int q = 0; q < nx; ++q) t += p[i * nx + q] * b[q * nu + j];
                pb[i * nu + j] = t;
            }
            for (int j = 0; j < nx; ++j) {
                double t = 0.0;
                for (int q = 0; q < nx; ++q) t += p[i * nx + q] * a[q * nx + j];
                pa[i * nx + j] = t;
            }
        }
        for (int i = 0; i < nu; ++i) {
            for (int j = 0; j < nu; ++j) {
                double t = 0.0;
                for (int q = 0; q < nx; ++q) t += b[q * nu + i] * pb[q * nu + j];
                s[i * nu + j] = r[i * nu + j] + t;
            }
            for (int j = 0; j < nx; ++j) {
                double t = 0.0;
                for (int q = 0; q < nx; ++q) t += b[q * nu + i] * pa[q * nx + j];
                kk[i * nx + j] = t;
            }
        }
        const int inf = chol_one(nu, s);
        if (info) info[bb] = inf;
        if (inf == 0) chol_solve_one(nu, nx, s, kk);
        free(pb);
        free(pa);
        free(s);
    }
}
