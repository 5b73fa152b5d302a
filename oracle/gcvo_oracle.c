/*
 * FP64 CPU oracle for Generalized-CVO registration.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference that the
 * GPU library is judged against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Everything here is the plain definition, written for a reader to check against
 * the paper by eye:
 *   - per-point covariance from the n nearest points (Sec. "Anisotropic
 *     covariance", eq. (kernel)/(covariance)) with the eigenvalue bound of
 *     Remark 1, found by brute-force distance ranking;
 *   - the objective f(T) = sum_ij c_ij k(x_i, T^{-1} z_j) (eq. (rkhs_loss)) as a
 *     literal double loop over all (i, j), restricted to pairs within the cutoff,
 *     with c_ij = <l^X_i, l^Z_j> from per-point label vectors (1 without labels);
 *   - the Riemannian gradient of Lemma 1 (eq. (gradient));
 *   - the Gauss-Newton Hessian -sum f J^T Sigma^{-1} J (eq. (hessian_gn)) plus
 *     the connection term of eq. (connection_se3);
 *   - the exact frozen-covariance derivative of the gradient (the first, second
 *     and fourth terms of eq. (direction_derivative_gradf)) for derivative tests
 *     and for the exact-Hessian (Newton) variant;
 *   - the update T <- T exp(xi^) of eq. (gn_update) and Algorithm 1's loop;
 *   - the first-order method: the quartic line-search polynomial along the
 *     gradient (App. "Line search", coefficients re-derived) and its step.
 *
 * Readings of points the paper leaves open (length scale, eigenvalue floor,
 * cutoff, damping, annealing schedule) are the ones stated in the project's
 * design notes; each is marked "reading:" below.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared.  Contraction is off
 * so that every product and sum rounds exactly as written.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_INVALID (-1)
#define ORC_ERR_TOO_FEW_POINTS (-2)
#define ORC_ERR_NO_PAIRS (-3)
#define ORC_ERR_SINGULAR (-4)

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra, row-major.                                   */
/* ------------------------------------------------------------------------ */

/* a^ : the 3x3 skew matrix with (a^) b = a x b. */
static void hat3(const double a[3], double A[9]) {
    A[0] = 0.0;   A[1] = -a[2]; A[2] = a[1];
    A[3] = a[2];  A[4] = 0.0;   A[5] = -a[0];
    A[6] = -a[1]; A[7] = a[0];  A[8] = 0.0;
}

/* C[n x m] = A[n x k] * B[k x m] */
static void matmul(const double *A, const double *B, double *C, int n, int k, int m) {
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < m; ++c) {
            double s = 0.0;
            for (int q = 0; q < k; ++q) s += A[r * k + q] * B[q * m + c];
            C[r * m + c] = s;
        }
}

static void transpose(const double *A, double *At, int n, int m) {
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < m; ++c) At[c * n + r] = A[r * m + c];
}

/* Inverse of a 3x3 matrix by Gauss-Jordan elimination with partial pivoting.
 * Returns 0 when a pivot is exactly zero. */
static int inv3(const double A[9], double Ainv[9]) {
    double M[3][6];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 6; ++c) M[r][c] = (c < 3) ? A[r * 3 + c] : (c - 3 == r ? 1.0 : 0.0);
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (M[piv][col] == 0.0) return 0;
        if (piv != col)
            for (int c = 0; c < 6; ++c) { double t = M[col][c]; M[col][c] = M[piv][c]; M[piv][c] = t; }
        double p = M[col][col];
        for (int c = 0; c < 6; ++c) M[col][c] /= p;
        for (int r = 0; r < 3; ++r) {
            if (r == col) continue;
            double fct = M[r][col];
            for (int c = 0; c < 6; ++c) M[r][c] -= fct * M[col][c];
        }
    }
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Ainv[r * 3 + c] = M[r][c + 3];
    return 1;
}

/* Solve A x = b for a general n x n system (n <= 6) by Gaussian elimination with
 * partial pivoting.  Fails (returns 0) when a pivot falls below tiny * max|A|. */
static int solve_lu(const double *A, const double *b, double *x, int n, double tiny) {
    double M[6][7];
    double amax = 0.0;
    for (int r = 0; r < n; ++r) {
        for (int c = 0; c < n; ++c) {
            M[r][c] = A[r * n + c];
            if (fabs(M[r][c]) > amax) amax = fabs(M[r][c]);
        }
        M[r][n] = b[r];
    }
    if (!(amax > 0.0) || !isfinite(amax)) return 0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (!(fabs(M[piv][col]) >= tiny * amax)) return 0;
        if (piv != col)
            for (int c = 0; c <= n; ++c) { double t = M[col][c]; M[col][c] = M[piv][c]; M[piv][c] = t; }
        for (int r = col + 1; r < n; ++r) {
            double fct = M[r][col] / M[col][col];
            for (int c = col; c <= n; ++c) M[r][c] -= fct * M[col][c];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = M[r][n];
        for (int c = r + 1; c < n; ++c) s -= M[r][c] * x[c];
        x[r] = s / M[r][r];
    }
    return 1;
}

/* Classical Jacobi eigen-decomposition of a symmetric 3x3 matrix: repeatedly
 * annihilate the largest off-diagonal entry with a plane rotation.  Eigenvalues
 * are returned in descending order, eigenvectors as the matching columns of V. */
static void jacobi_eig3(const double Ain[9], double lam[3], double V[9]) {
    double A[9];
    memcpy(A, Ain, sizeof A);
    for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        int p = 0, q = 1;
        double big = fabs(A[1]);
        if (fabs(A[2]) > big) { big = fabs(A[2]); p = 0; q = 2; }
        if (fabs(A[5]) > big) { big = fabs(A[5]); p = 1; q = 2; }
        double scale = fabs(A[0]) + fabs(A[4]) + fabs(A[8]);
        if (big == 0.0 || big <= 1e-300 || big < 1e-18 * scale) break;
        double app = A[p * 3 + p], aqq = A[q * 3 + q], apq = A[p * 3 + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        /* A <- J^T A J with J the rotation in the (p, q) plane. */
        for (int k = 0; k < 3; ++k) {
            double akp = A[k * 3 + p], akq = A[k * 3 + q];
            A[k * 3 + p] = c * akp - s * akq;
            A[k * 3 + q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
            double apk = A[p * 3 + k], aqk = A[q * 3 + k];
            A[p * 3 + k] = c * apk - s * aqk;
            A[q * 3 + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {
            double vkp = V[k * 3 + p], vkq = V[k * 3 + q];
            V[k * 3 + p] = c * vkp - s * vkq;
            V[k * 3 + q] = s * vkp + c * vkq;
        }
    }
    double d[3] = {A[0], A[4], A[8]};
    int order[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (d[order[b]] > d[order[a]]) { int t = order[a]; order[a] = order[b]; order[b] = t; }
    double Vs[9];
    for (int k = 0; k < 3; ++k) {
        lam[k] = d[order[k]];
        for (int r = 0; r < 3; ++r) Vs[r * 3 + k] = V[r * 3 + order[k]];
    }
    memcpy(V, Vs, sizeof Vs);
}

/* ------------------------------------------------------------------------ */
/* Per-point covariance shapes (eq. (covariance), Remark 1).                */
/* ------------------------------------------------------------------------ */

/* Indices of the k nearest points of P to P[p] (P[p] itself included), ranked
 * by squared Euclidean distance, ties broken by the smaller index. */
static void knn_one(const double *P, long n, long p, int k, long *out, double *dist) {
    int have = 0;
    const double px = P[3 * p], py = P[3 * p + 1], pz = P[3 * p + 2];
    for (long q = 0; q < n; ++q) {
        double dx = P[3 * q] - px, dy = P[3 * q + 1] - py, dz = P[3 * q + 2] - pz;
        double d = dx * dx + dy * dy + dz * dz;
        /* Is (d, q) lexicographically smaller than the current k-th entry? */
        if (have == k && !(d < dist[k - 1] || (d == dist[k - 1] && q < out[k - 1]))) continue;
        int pos = (have < k) ? have++ : k - 1;
        while (pos > 0 && (d < dist[pos - 1] || (d == dist[pos - 1] && q < out[pos - 1]))) {
            dist[pos] = dist[pos - 1];
            out[pos] = out[pos - 1];
            --pos;
        }
        dist[pos] = d;
        out[pos] = q;
    }
}

int orc_knn(const double *P, long n, int k, long *out) {
    if (!P || !out || n < 0 || k < 1 || k > 64) return ORC_ERR_INVALID;
    if (n < k) return ORC_ERR_TOO_FEW_POINTS;
#pragma omp parallel for schedule(dynamic, 64)
    for (long p = 0; p < n; ++p) {
        double dist[64];
        knn_one(P, n, p, k, out + p * k, dist);
    }
    return ORC_OK;
}

/* Shape of one point from its neighbour list: M = 1/(k-1) sum (q-p)(q-p)^T
 * centred at p (eq. (covariance)); eigenvalues l1 >= l2 >= l3;
 * reading: S = U diag(1, max(l2/l1, rho), max(l3/l1, rho)) U^T (Remark 1's
 * bound, applied per point with the largest mode normalised to one), and
 * S = I when l1 <= 1e-300 (all neighbours coincide).  Output order
 * (xx, xy, xz, yy, yz, zz). */
static void shape_from_neighbours(const double *P, long p, const long *nb, int k, double rho,
                                  double S6[6]) {
    double M[9] = {0};
    for (int a = 0; a < k; ++a) {
        const double *q = P + 3 * nb[a];
        double d[3] = {q[0] - P[3 * p], q[1] - P[3 * p + 1], q[2] - P[3 * p + 2]};
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) M[r * 3 + c] += d[r] * d[c];
    }
    for (int i = 0; i < 9; ++i) M[i] /= (double)(k - 1);
    double lam[3], U[9];
    jacobi_eig3(M, lam, U);
    double S[9];
    if (!(lam[0] > 1e-300)) {
        for (int i = 0; i < 9; ++i) S[i] = (i % 4 == 0) ? 1.0 : 0.0;
    } else {
        double w[3] = {1.0, lam[1] / lam[0], lam[2] / lam[0]};
        for (int m = 1; m < 3; ++m) if (w[m] < rho) w[m] = rho;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int m = 0; m < 3; ++m) s += U[r * 3 + m] * w[m] * U[c * 3 + m];
                S[r * 3 + c] = s;
            }
    }
    S6[0] = S[0]; S6[1] = S[1]; S6[2] = S[2]; S6[3] = S[4]; S6[4] = S[5]; S6[5] = S[8];
}

int orc_point_shapes(const double *P, long n, int k, double rho, double *S6) {
    if (!P || !S6 || n < 0 || k < 2 || k > 64 || !(rho > 0.0) || rho > 1.0) return ORC_ERR_INVALID;
    if (n < k) return ORC_ERR_TOO_FEW_POINTS;
#pragma omp parallel for schedule(dynamic, 64)
    for (long p = 0; p < n; ++p) {
        long nb[64];
        double dist[64];
        knn_one(P, n, p, k, nb, dist);
        shape_from_neighbours(P, p, nb, k, rho, S6 + 6 * p);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Pair search: which target points are within the cutoff of a source point. */
/* ------------------------------------------------------------------------ */

/*
 * The sums below visit, for each transformed source point y, every target
 * point i with ||x_i - y||^2 <= cutoff^2, in increasing i.  Two ways of finding
 * them give the same index lists:
 *   - brute force: test every i (the definition);
 *   - grid: a uniform grid over X with cells of edge >= cutoff, so every point
 *     within the cutoff of y lies in one of the 27 cells around y's cell; the
 *     same distance test is applied to their points and the accepted indices
 *     are sorted ascending.
 * The grid is used when nx * nz reaches orc_set_grid_threshold's value
 * (default 25e6, i.e. above two 5000-point clouds) and there is a cutoff.
 */
static long long g_grid_min_pairs = 25000000LL;

void orc_set_grid_threshold(long long min_pairs) { g_grid_min_pairs = min_pairs; }

typedef struct {
    int on;
    double lo[3], inv_h;
    long n[3];
    long *start; /* [ncells + 1]: cell c holds idx[start[c] .. start[c + 1]) */
    long *idx;   /* point indices grouped by cell, ascending within a cell     */
} pair_search;

static long clampl(long v, long lo, long hi) { return v < lo ? lo : (v > hi ? hi : v); }

static long grid_cell(const pair_search *S, const double p[3], int d) {
    return (long)floor((p[d] - S->lo[d]) * S->inv_h);
}

static void search_free(pair_search *S);

/* Sets up the grid when it is to be used; without memory for it the search
 * stays brute force (the same index lists). */
static void search_init(pair_search *S, const double *X, long nx, long nz, double cutoff) {
    memset(S, 0, sizeof *S);
    if (!(cutoff > 0.0) || nx == 0 || (long long)nx * (long long)nz < g_grid_min_pairs) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (long i = 0; i < nx; ++i)
        for (int d = 0; d < 3; ++d) {
            if (X[3 * i + d] < lo[d]) lo[d] = X[3 * i + d];
            if (X[3 * i + d] > hi[d]) hi[d] = X[3 * i + d];
        }
    /* Edge slightly above the cutoff (so rounding of the cell coordinates
     * cannot put a point within the cutoff two cells away), doubled until the
     * grid has at most 8 cells per point. */
    double h = cutoff * (1.0 + 1e-9);
    long n[3];
    for (;;) {
        double cells = 1.0;
        for (int d = 0; d < 3; ++d) {
            n[d] = (long)floor((hi[d] - lo[d]) / h) + 1;
            cells *= (double)n[d];
        }
        if (cells <= 8.0 * (double)nx + 1024.0) break;
        h *= 2.0;
    }
    S->on = 1;
    for (int d = 0; d < 3; ++d) {
        S->lo[d] = lo[d];
        S->n[d] = n[d];
    }
    S->inv_h = 1.0 / h;
    const long ncells = n[0] * n[1] * n[2];
    S->start = (long *)calloc((size_t)ncells + 1, sizeof(long));
    S->idx = (long *)malloc(sizeof(long) * (size_t)nx);
    long *cell = (long *)malloc(sizeof(long) * (size_t)nx);
    if (!S->start || !S->idx || !cell) {
        free(cell);
        search_free(S);
        return;
    }
    for (long i = 0; i < nx; ++i) {
        long c[3];
        for (int d = 0; d < 3; ++d) c[d] = clampl(grid_cell(S, X + 3 * i, d), 0, n[d] - 1);
        cell[i] = c[0] + n[0] * (c[1] + n[1] * c[2]);
        S->start[cell[i] + 1] += 1;
    }
    for (long c = 0; c < ncells; ++c) S->start[c + 1] += S->start[c];
    long *fill = (long *)malloc(sizeof(long) * (size_t)ncells);
    if (!fill) {
        free(cell);
        search_free(S);
        return;
    }
    memcpy(fill, S->start, sizeof(long) * (size_t)ncells);
    for (long i = 0; i < nx; ++i) S->idx[fill[cell[i]]++] = i;   /* ascending i within each cell */
    free(fill);
    free(cell);
}

static void search_free(pair_search *S) {
    free(S->start);
    free(S->idx);
    memset(S, 0, sizeof *S);
}

static int cmp_long(const void *a, const void *b) {
    const long x = *(const long *)a, y = *(const long *)b;
    return (x > y) - (x < y);
}

/* Indices i with ||x_i - y||^2 <= rc2, ascending, into *buf (grown as needed;
 * the caller frees it).  Returns the count, or -1 on allocation failure. */
static long pairs_of(const pair_search *S, const double *X, long nx, const double y[3], double rc2, long **buf,
                     long *cap) {
    long m = 0;
#define ORC_PUSH(ii)                                                              \
    do {                                                                          \
        if (m == *cap) {                                                          \
            long nc = *cap ? 2 * *cap : 256;                                      \
            long *nb = (long *)realloc(*buf, sizeof(long) * (size_t)nc);          \
            if (!nb) return -1;                                                   \
            *buf = nb;                                                            \
            *cap = nc;                                                            \
        }                                                                         \
        (*buf)[m++] = (ii);                                                       \
    } while (0)
    if (!S->on) {
        for (long i = 0; i < nx; ++i) {
            double r3[3] = {X[3 * i] - y[0], X[3 * i + 1] - y[1], X[3 * i + 2] - y[2]};
            double d2 = r3[0] * r3[0] + r3[1] * r3[1] + r3[2] * r3[2];
            if (d2 <= rc2) ORC_PUSH(i);
        }
        return m;
    }
    long c[3], lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        const double u = (y[d] - S->lo[d]) * S->inv_h;
        if (!(u > -2.0 && u < (double)S->n[d] + 1.0)) return 0;   /* no cell within reach (or NaN) */
        c[d] = (long)floor(u);
        lo[d] = clampl(c[d] - 1, 0, S->n[d] - 1);
        hi[d] = clampl(c[d] + 1, 0, S->n[d] - 1);
        if (c[d] + 1 < 0 || c[d] - 1 > S->n[d] - 1) return 0;
    }
    for (long cz = lo[2]; cz <= hi[2]; ++cz)
        for (long cy = lo[1]; cy <= hi[1]; ++cy)
            for (long cx = lo[0]; cx <= hi[0]; ++cx) {
                const long cell = cx + S->n[0] * (cy + S->n[1] * cz);
                for (long a = S->start[cell]; a < S->start[cell + 1]; ++a) {
                    const long i = S->idx[a];
                    double r3[3] = {X[3 * i] - y[0], X[3 * i + 1] - y[1], X[3 * i + 2] - y[2]};
                    double d2 = r3[0] * r3[0] + r3[1] * r3[1] + r3[2] * r3[2];
                    if (d2 <= rc2) ORC_PUSH(i);
                }
            }
#undef ORC_PUSH
    if (m > 1) qsort(*buf, (size_t)m, sizeof(long), cmp_long);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Objective, gradient and Hessians at a pose (literal double sum).         */
/* ------------------------------------------------------------------------ */

static void shape6_to_mat(const double s[6], double S[9]) {
    S[0] = s[0]; S[1] = s[1]; S[2] = s[2];
    S[3] = s[1]; S[4] = s[3]; S[5] = s[4];
    S[6] = s[2]; S[7] = s[4]; S[8] = s[5];
}

/*
 * Sums over every pair (i, j) with ||x_i - y_j||^2 <= cutoff^2, y_j = R^T (z_j - t):
 *   Sigma_ij = (ell^2 / 2) * (S_i + Rs^T S_j Rs)      reading of eq. (covariance)
 *            with the length scale folded in and Rs the rotation the covariances
 *            are frozen at (Rs = R unless R_shape is given; Remark 2);
 *   f_ij     = sigma2 * exp(-1/2 r^T Sigma_ij^{-1} r), r = x_i - y_j   (eq. (kernel))
 *   J_j      = [ -y_j^ , I ]                                        (eq. (f_ij_J_j))
 *   f       += f_ij
 *   g       += -f_ij J_j^T Sigma^{-1} r                              (Lemma 1)
 *   Hmain   += -f_ij J_j^T Sigma^{-1} J_j                            (eq. (hessian_gn))
 *   T1      += f_ij (J^T u)(J^T u)^T, u = Sigma^{-1} r    (product rule on f_ij)
 *   T2      += -f_ij [ u^ J_j ; 0 ]                       (derivative of J_j)
 * cutoff <= 0 means no cutoff.  T1/T2 may be NULL.  The loop runs j-outer; each
 * source point's slice is summed into its own slot and the slots are added in
 * j order, so the result does not depend on the thread count.
 */
/* Label weight c_ij = <l^X_i, l^Z_j> of eq. (rkhs_loss) (pose-invariant
 * per-point features, row-major [n][dim]); 1 without labels. */
static double label_weight(const double *LX, const double *LZ, int dim, long i, long j) {
    if (!LX || !LZ || dim <= 0) return 1.0;
    double c = 0.0;
    for (int d = 0; d < dim; ++d) c += LX[(size_t)i * dim + d] * LZ[(size_t)j * dim + d];
    return c;
}

int orc_eval_l(const double *X, const double *SX, const double *LX, long nx, const double *Z, const double *SZ,
               const double *LZ, long nz, int label_dim, const double T[16], const double *R_shape, double ell,
               double cutoff, double sigma2, double *f_out, double g_out[6], double Hmain_out[36],
               double *T1_out, double *T2_out, long long *npairs_out);

int orc_eval(const double *X, const double *SX, long nx, const double *Z, const double *SZ, long nz,
             const double T[16], const double *R_shape, double ell, double cutoff, double sigma2,
             double *f_out, double g_out[6], double Hmain_out[36], double *T1_out, double *T2_out,
             long long *npairs_out) {
    return orc_eval_l(X, SX, NULL, nx, Z, SZ, NULL, nz, 0, T, R_shape, ell, cutoff, sigma2, f_out, g_out, Hmain_out,
                      T1_out, T2_out, npairs_out);
}

/* The same sums with every pair weighted by its label weight c_ij. */
int orc_eval_l(const double *X, const double *SX, const double *LX, long nx, const double *Z, const double *SZ,
               const double *LZ, long nz, int label_dim, const double T[16], const double *R_shape, double ell,
               double cutoff, double sigma2, double *f_out, double g_out[6], double Hmain_out[36],
               double *T1_out, double *T2_out, long long *npairs_out) {
    if (!X || !SX || !Z || !SZ || !T || nx < 0 || nz < 0 || !(ell > 0.0) || !f_out || !g_out ||
        !Hmain_out)
        return ORC_ERR_INVALID;
    const int want_t = (T1_out != NULL) || (T2_out != NULL);
    const int stride = 1 + 6 + 36 + (want_t ? 72 : 0);
    double *slot = (double *)calloc((size_t)(nz > 0 ? nz : 1) * stride, sizeof(double));
    long long *pcount = (long long *)calloc((size_t)(nz > 0 ? nz : 1), sizeof(long long));
    if (!slot || !pcount) { free(slot); free(pcount); return ORC_ERR_INVALID; }
    double R[9], t[3], Rs[9];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R[r * 3 + c] = T[r * 4 + c];
        t[r] = T[r * 4 + 3];
    }
    memcpy(Rs, R_shape ? R_shape : R, sizeof Rs);
    double Rst[9];
    transpose(Rs, Rst, 3, 3);
    const double half_l2 = 0.5 * ell * ell;
    const double rc2 = (cutoff > 0.0) ? cutoff * cutoff : INFINITY;
    pair_search search;
    search_init(&search, X, nx, nz, cutoff);
    int failed = 0;

#pragma omp parallel
    {
    long *pairs = NULL, cap = 0;
#pragma omp for schedule(dynamic, 16)
    for (long j = 0; j < nz; ++j) {
        double *acc = slot + (size_t)j * stride;
        double zt[3] = {Z[3 * j] - t[0], Z[3 * j + 1] - t[1], Z[3 * j + 2] - t[2]};
        double y[3];
        for (int r = 0; r < 3; ++r) y[r] = R[0 * 3 + r] * zt[0] + R[1 * 3 + r] * zt[1] + R[2 * 3 + r] * zt[2];
        double Sj[9], tmp[9], SjR[9];
        shape6_to_mat(SZ + 6 * j, Sj);
        matmul(Rst, Sj, tmp, 3, 3, 3);
        matmul(tmp, Rs, SjR, 3, 3, 3);
        double J[18], Jt[18], yh[9];
        hat3(y, yh);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                J[r * 6 + c] = -yh[r * 3 + c];
                J[r * 6 + 3 + c] = (r == c) ? 1.0 : 0.0;
            }
        transpose(J, Jt, 3, 6);
        const long m = pairs_of(&search, X, nx, y, rc2, &pairs, &cap);
        if (m < 0) {
#pragma omp atomic write
            failed = 1;
            continue;
        }
        for (long a = 0; a < m; ++a) {
            const long i = pairs[a];
            double r3[3] = {X[3 * i] - y[0], X[3 * i + 1] - y[1], X[3 * i + 2] - y[2]};
            double Si[9], Sig[9], Sinv[9];
            shape6_to_mat(SX + 6 * i, Si);
            for (int a = 0; a < 9; ++a) Sig[a] = half_l2 * (Si[a] + SjR[a]);
            if (!inv3(Sig, Sinv)) continue;
            double u[3];
            matmul(Sinv, r3, u, 3, 3, 1);
            double quad = r3[0] * u[0] + r3[1] * u[1] + r3[2] * u[2];
            double fij = label_weight(LX, LZ, label_dim, i, j) * sigma2 * exp(-0.5 * quad);
            double Jtu[6], SinvJ[18], JtSJ[36];
            matmul(Jt, u, Jtu, 6, 3, 1);
            matmul(Sinv, J, SinvJ, 3, 3, 6);
            matmul(Jt, SinvJ, JtSJ, 6, 3, 6);
            acc[0] += fij;
            for (int a = 0; a < 6; ++a) acc[1 + a] += -fij * Jtu[a];
            for (int a = 0; a < 36; ++a) acc[7 + a] += -fij * JtSJ[a];
            if (want_t) {
                double *t1 = acc + 43, *t2 = acc + 79;
                for (int a = 0; a < 6; ++a)
                    for (int b = 0; b < 6; ++b) t1[a * 6 + b] += fij * Jtu[a] * Jtu[b];
                double uh[9], uhJ[18];
                hat3(u, uh);
                matmul(uh, J, uhJ, 3, 3, 6);
                for (int a = 0; a < 18; ++a) t2[a] += -fij * uhJ[a];
            }
            pcount[j] += 1;
        }
    }
    free(pairs);
    }
    search_free(&search);
    if (failed) { free(slot); free(pcount); return ORC_ERR_INVALID; }

    double f = 0.0, g[6] = {0}, H[36] = {0}, T1[36] = {0}, T2[36] = {0};
    long long np = 0;
    for (long j = 0; j < nz; ++j) {
        const double *acc = slot + (size_t)j * stride;
        f += acc[0];
        for (int a = 0; a < 6; ++a) g[a] += acc[1 + a];
        for (int a = 0; a < 36; ++a) H[a] += acc[7 + a];
        if (want_t) {
            for (int a = 0; a < 36; ++a) T1[a] += acc[43 + a];
            for (int a = 0; a < 18; ++a) T2[a] += acc[79 + a];
        }
        np += pcount[j];
    }
    free(slot);
    free(pcount);
    *f_out = f;
    memcpy(g_out, g, sizeof g);
    memcpy(Hmain_out, H, sizeof H);
    if (T1_out) memcpy(T1_out, T1, sizeof T1);
    if (T2_out) memcpy(T2_out, T2, sizeof T2);
    if (npairs_out) *npairs_out = np;
    return ORC_OK;
}

/* Connection term of eq. (connection_se3): Gamma^v(xi, grad f) = C(g) xi with
 * C(g) = [[ -1/2 g_w^, 0 ], [ -g_v^, 0 ]]. */
void orc_connection(const double g[6], double C[36]) {
    double gw[9], gv[9];
    hat3(g, gw);
    hat3(g + 3, gv);
    memset(C, 0, 36 * sizeof(double));
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            C[r * 6 + c] = -0.5 * gw[r * 3 + c];
            C[(r + 3) * 6 + c] = -gv[r * 3 + c];
        }
}

/* exp(xi^) for xi = (w, v): closed form R = I + A W + B W^2, t = (I + B W + C W^2) v
 * with A = sin(th)/th, B = (1-cos th)/th^2, C = (th - sin th)/th^3.  B is
 * evaluated as (1/2) (sin(th/2)/(th/2))^2, which has no cancellation; A and B
 * use their Taylor series below th = 1e-5 and C below th = 1e-2, where the
 * closed form of C cancels. */
void orc_se3_exp(const double xi[6], double T[16]) {
    double th2 = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
    double th = sqrt(th2);
    double A, B, Cc;
    if (th < 1e-5) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
    } else {
        double h = sin(0.5 * th) / (0.5 * th);
        A = sin(th) / th;
        B = 0.5 * h * h;
    }
    if (th < 1e-2)
        Cc = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0 - th2 * th2 * th2 / 362880.0;
    else
        Cc = (th - sin(th)) / (th2 * th);
    double W[9], W2[9];
    hat3(xi, W);
    matmul(W, W, W2, 3, 3, 3);
    double R[9], V[9];
    for (int a = 0; a < 9; ++a) {
        double I = (a % 4 == 0) ? 1.0 : 0.0;
        R[a] = I + A * W[a] + B * W2[a];
        V[a] = I + B * W[a] + Cc * W2[a];
    }
    double tv[3];
    matmul(V, xi + 3, tv, 3, 3, 1);
    memset(T, 0, 16 * sizeof(double));
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) T[r * 4 + c] = R[r * 3 + c];
        T[r * 4 + 3] = tv[r];
    }
    T[15] = 1.0;
}

/*
 * Line-search polynomial of the first-order method (Sec. "A first-order
 * method", App. "Line search"), re-derived because the printed coefficients
 * are partly garbled (reading): along T(t) = T exp(t xi^) with the covariances
 * frozen at T,
 *   y_j(t) = exp(-t xi^) y_j = y - t e1 + t^2/2 e2 - t^3/6 e3 + t^4/24 e4 + O(t^5),
 *   e1 = w x y_j + v,  e_{k+1} = w x e_k,
 * so with P = Sigma_ij^{-1} and r = x_i - y_j the exponent of k_ij is
 *   -1/2 r^T P r + beta t + gamma t^2 + delta t^3 + eps t^4 + O(t^5),
 *   beta  = -e1.P r
 *   gamma = -1/2 e1.P e1 + 1/2 e2.P r
 *   delta =  1/2 e1.P e2 - 1/6 e3.P r
 *   eps   = -1/8 e2.P e2 - 1/6 e1.P e3 + 1/24 e4.P r
 * and exp() of that series is 1 + g1 t + g2 t^2 + g3 t^3 + g4 t^4 with the
 * paper's combination g1 = beta, g2 = gamma + beta^2/2, g3 = delta + beta gamma
 * + beta^3/6, g4 = eps + beta delta + beta^2 gamma/2 + gamma^2/2 + beta^4/24.
 * c[0] = sum f_ij, c[k] = sum f_ij g^k_ij (k = 1..4): G(t) ~ sum_k c[k] t^k.
 * Same pair set and loop order as orc_eval.
 */
int orc_line_coeffs_l(const double *X, const double *SX, const double *LX, long nx, const double *Z,
                      const double *SZ, const double *LZ, long nz, int label_dim, const double T[16], double ell,
                      double cutoff, double sigma2, const double xi[6], double c_out[5], long long *npairs_out);

int orc_line_coeffs(const double *X, const double *SX, long nx, const double *Z, const double *SZ, long nz,
                    const double T[16], double ell, double cutoff, double sigma2, const double xi[6],
                    double c_out[5], long long *npairs_out) {
    return orc_line_coeffs_l(X, SX, NULL, nx, Z, SZ, NULL, nz, 0, T, ell, cutoff, sigma2, xi, c_out, npairs_out);
}

int orc_line_coeffs_l(const double *X, const double *SX, const double *LX, long nx, const double *Z,
                      const double *SZ, const double *LZ, long nz, int label_dim, const double T[16], double ell,
                      double cutoff, double sigma2, const double xi[6], double c_out[5], long long *npairs_out) {
    if (!X || !SX || !Z || !SZ || !T || !xi || !c_out || nx < 0 || nz < 0 || !(ell > 0.0))
        return ORC_ERR_INVALID;
    double *slot = (double *)calloc((size_t)(nz > 0 ? nz : 1) * 5, sizeof(double));
    long long *pcount = (long long *)calloc((size_t)(nz > 0 ? nz : 1), sizeof(long long));
    if (!slot || !pcount) { free(slot); free(pcount); return ORC_ERR_INVALID; }
    double R[9], t[3], Rt[9];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R[r * 3 + c] = T[r * 4 + c];
        t[r] = T[r * 4 + 3];
    }
    transpose(R, Rt, 3, 3);
    const double half_l2 = 0.5 * ell * ell;
    const double rc2 = (cutoff > 0.0) ? cutoff * cutoff : INFINITY;
    double W[9];
    hat3(xi, W);
    pair_search search;
    search_init(&search, X, nx, nz, cutoff);
    int failed = 0;

#pragma omp parallel
    {
    long *pairs = NULL, cap = 0;
#pragma omp for schedule(dynamic, 16)
    for (long j = 0; j < nz; ++j) {
        double *acc = slot + (size_t)j * 5;
        double zt[3] = {Z[3 * j] - t[0], Z[3 * j + 1] - t[1], Z[3 * j + 2] - t[2]};
        double y[3];
        matmul(Rt, zt, y, 3, 3, 1);
        double Sj[9], tmp[9], SjR[9];
        shape6_to_mat(SZ + 6 * j, Sj);
        matmul(Rt, Sj, tmp, 3, 3, 3);
        matmul(tmp, R, SjR, 3, 3, 3);
        double e[5][3];                        /* e[1..4] */
        matmul(W, y, e[1], 3, 3, 1);
        for (int a = 0; a < 3; ++a) e[1][a] += xi[3 + a];
        for (int k = 2; k <= 4; ++k) matmul(W, e[k - 1], e[k], 3, 3, 1);
        const long m = pairs_of(&search, X, nx, y, rc2, &pairs, &cap);
        if (m < 0) {
#pragma omp atomic write
            failed = 1;
            continue;
        }
        for (long a = 0; a < m; ++a) {
            const long i = pairs[a];
            double r3[3] = {X[3 * i] - y[0], X[3 * i + 1] - y[1], X[3 * i + 2] - y[2]};
            double Si[9], Sig[9], P[9];
            shape6_to_mat(SX + 6 * i, Si);
            for (int a = 0; a < 9; ++a) Sig[a] = half_l2 * (Si[a] + SjR[a]);
            if (!inv3(Sig, P)) continue;
            double Pr[3], Pe1[3], Pe2[3];
            matmul(P, r3, Pr, 3, 3, 1);
            matmul(P, e[1], Pe1, 3, 3, 1);
            matmul(P, e[2], Pe2, 3, 3, 1);
            double quad = r3[0] * Pr[0] + r3[1] * Pr[1] + r3[2] * Pr[2];
            double fij = label_weight(LX, LZ, label_dim, i, j) * sigma2 * exp(-0.5 * quad);
            double e1Pr = 0, e2Pr = 0, e3Pr = 0, e4Pr = 0, e1Pe1 = 0, e2Pe2 = 0, e1Pe2 = 0, e3Pe1 = 0;
            for (int a = 0; a < 3; ++a) {
                e1Pr += e[1][a] * Pr[a];
                e2Pr += e[2][a] * Pr[a];
                e3Pr += e[3][a] * Pr[a];
                e4Pr += e[4][a] * Pr[a];
                e1Pe1 += e[1][a] * Pe1[a];
                e2Pe2 += e[2][a] * Pe2[a];
                e1Pe2 += e[1][a] * Pe2[a];
                e3Pe1 += e[3][a] * Pe1[a];
            }
            double beta = -e1Pr;
            double gamma = -0.5 * e1Pe1 + 0.5 * e2Pr;
            double delta = 0.5 * e1Pe2 - e3Pr / 6.0;
            double eps = -0.125 * e2Pe2 - e3Pe1 / 6.0 + e4Pr / 24.0;
            double g1 = beta;
            double g2 = gamma + 0.5 * beta * beta;
            double g3 = delta + beta * gamma + beta * beta * beta / 6.0;
            double g4 = eps + beta * delta + 0.5 * beta * beta * gamma + 0.5 * gamma * gamma +
                        beta * beta * beta * beta / 24.0;
            acc[0] += fij;
            acc[1] += fij * g1;
            acc[2] += fij * g2;
            acc[3] += fij * g3;
            acc[4] += fij * g4;
            pcount[j] += 1;
        }
    }
    free(pairs);
    }
    search_free(&search);
    if (failed) { free(slot); free(pcount); return ORC_ERR_INVALID; }
    double c[5] = {0};
    long long np = 0;
    for (long j = 0; j < nz; ++j) {
        for (int k = 0; k < 5; ++k) c[k] += slot[(size_t)j * 5 + k];
        np += pcount[j];
    }
    free(slot);
    free(pcount);
    memcpy(c_out, c, sizeof c);
    if (npairs_out) *npairs_out = np;
    return ORC_OK;
}

static double dpoly(const double c[5], double t) {
    return c[1] + t * (2.0 * c[2] + t * (3.0 * c[3] + t * 4.0 * c[4]));
}

/* Bisection of G' on [lo, hi] with G'(lo) > 0 >= G'(hi). */
static double bisect_root(const double c[5], double lo, double hi) {
    for (int it = 0; it < 400 && hi - lo > 1e-17 * hi; ++it) {
        double mid = 0.5 * (lo + hi);
        if (dpoly(c, mid) > 0.0) lo = mid;
        else hi = mid;
    }
    return hi;
}

/*
 * Step size of eq. (linesearch): the smallest positive real root t* of
 * G'(t) = c1 + 2 c2 t + 3 c3 t^2 + 4 c4 t^3 and mu = max(mu0, t*).  The
 * critical points of G' (roots of G'', closed form) split t > 0 into intervals
 * where G' is monotone; the first interval whose right end has G' <= 0 holds
 * t*, found by bisection.  Reading where the quartic's derivative has no
 * positive root (a positive quartic term far outside the expansion's range,
 * common once the iterate is near a maximum): the paper falls back to a fixed
 * minimum step mu0, whose size depends on the objective's units; here the
 * fallback is the maximiser of the quadratic part, -c1 / (2 c2), when c2 < 0,
 * and mu0 only when even that does not exist.  Returns 1 (quartic root),
 * 2 (quadratic step) or 0 (mu0).
 */
int orc_first_order_step(const double c[5], double mu0, double *mu) {
    *mu = mu0;
    if (!(c[1] > 0.0)) return 0;
    const double tq = (c[2] < 0.0) ? c[1] / (-2.0 * c[2]) : 0.0;
    double cp[2];
    int ncp = 0;
    /* G'' = 2 c2 + 6 c3 t + 12 c4 t^2 */
    if (c[4] != 0.0) {
        double a = 12.0 * c[4], b = 6.0 * c[3], cc = 2.0 * c[2];
        double disc = b * b - 4.0 * a * cc;
        if (disc >= 0.0) {
            double sq = sqrt(disc);
            double r1 = (-b - sq) / (2.0 * a), r2 = (-b + sq) / (2.0 * a);
            if (r1 > r2) { double tt = r1; r1 = r2; r2 = tt; }
            if (r1 > 0.0) cp[ncp++] = r1;
            if (r2 > 0.0 && r2 != r1) cp[ncp++] = r2;
        }
    } else if (c[3] != 0.0) {
        double r = -2.0 * c[2] / (6.0 * c[3]);
        if (r > 0.0) cp[ncp++] = r;
    }
    double lo = 0.0;
    for (int k = 0; k < ncp; ++k) {
        if (dpoly(c, cp[k]) <= 0.0) {
            double t = bisect_root(c, lo, cp[k]);
            *mu = t > mu0 ? t : mu0;
            return 1;
        }
        lo = cp[k];
    }
    /* last interval (lo, inf): a root exists only if G' tends to -inf */
    double lead = (c[4] != 0.0) ? c[4] : (c[3] != 0.0) ? c[3] : c[2];
    double hi = (lo > 0.0) ? 2.0 * lo : 1e-30;
    if (lead < 0.0)
        for (int it = 0; it < 4000 && dpoly(c, hi) > 0.0; ++it) hi *= 2.0;
    if (!(lead < 0.0) || dpoly(c, hi) > 0.0) {
        if (tq > 0.0) {
            *mu = tq > mu0 ? tq : mu0;
            return 2;
        }
        return 0;
    }
    double t = bisect_root(c, lo, hi);
    *mu = t > mu0 ? t : mu0;
    return 1;
}

/*
 * Step of eq. (gn_update): xi = -H^{-1} g with H = Hmain + C(g) (or, for the
 * exact-Hessian variant, H = T1 + T2 + Hmain + C(g), passed in as H).
 * Reading of the damping the paper leaves open:
 *   1. g == 0 => xi = 0.
 *   2. Solve H xi = -g by partial-pivoting elimination; accept when no pivot is
 *      below 1e-12 * max|H| and g . xi > 0 (an ascent direction).
 *   3. Otherwise drop C(g) and solve (Hmain - lambda * ||diag Hmain||_2 * I) xi = -g
 *      for lambda = 1e-6 * 10^m, m = 0..6, accepting the first that passes the
 *      same test.  Hmain is negative semi-definite, so this succeeds unless
 *      Hmain vanishes.
 *   4. Otherwise ORC_ERR_SINGULAR.
 * *damped receives 0 (plain), m + 1 (damped at attempt m).
 */
int orc_solve_step(const double H[36], const double Hmain[36], const double g[6], double xi[6],
                   int *damped) {
    double mg[6];
    int zero = 1;
    for (int a = 0; a < 6; ++a) {
        mg[a] = -g[a];
        if (g[a] != 0.0) zero = 0;
    }
    if (damped) *damped = 0;
    if (zero) {
        memset(xi, 0, 6 * sizeof(double));
        return ORC_OK;
    }
    double x[6];
    if (solve_lu(H, mg, x, 6, 1e-12)) {
        double gx = 0.0;
        for (int a = 0; a < 6; ++a) gx += g[a] * x[a];
        if (gx > 0.0) {
            memcpy(xi, x, sizeof x);
            return ORC_OK;
        }
    }
    double dn = 0.0;
    for (int a = 0; a < 6; ++a) dn += Hmain[a * 7] * Hmain[a * 7];
    dn = sqrt(dn);
    double lam = 1e-6;
    for (int m = 0; m <= 6; ++m, lam *= 10.0) {
        double Hd[36];
        memcpy(Hd, Hmain, sizeof Hd);
        for (int a = 0; a < 6; ++a) Hd[a * 7] -= lam * dn;
        if (solve_lu(Hd, mg, x, 6, 1e-12)) {
            double gx = 0.0;
            for (int a = 0; a < 6; ++a) gx += g[a] * x[a];
            if (gx > 0.0) {
                memcpy(xi, x, sizeof x);
                if (damped) *damped = m + 1;
                return ORC_OK;
            }
        }
    }
    return ORC_ERR_SINGULAR;
}

/* 1 when the symmetric part of H is negative definite: Cholesky of
 * -(H + H^T)/2 with every pivot above 1e-12 * max|H|. */
static int sym_negative_definite(const double H[36]) {
    double A[36], amax = 0.0;
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            A[r * 6 + c] = -0.5 * (H[r * 6 + c] + H[c * 6 + r]);
            if (fabs(H[r * 6 + c]) > amax) amax = fabs(H[r * 6 + c]);
        }
    if (!(amax > 0.0)) return 0;
    for (int k = 0; k < 6; ++k) {
        double d = A[k * 6 + k];
        for (int m = 0; m < k; ++m) d -= A[k * 6 + m] * A[k * 6 + m];
        if (!(d > 1e-12 * amax)) return 0;
        d = sqrt(d);
        A[k * 6 + k] = d;
        for (int r = k + 1; r < 6; ++r) {
            double v = A[r * 6 + k];
            for (int m = 0; m < k; ++m) v -= A[r * 6 + m] * A[k * 6 + m];
            A[r * 6 + k] = v / d;
        }
    }
    return 1;
}

static int pose_is_rigid(const double T[16]) {
    for (int a = 0; a < 16; ++a) if (!isfinite(T[a])) return 0;
    if (fabs(T[12]) > 1e-6 || fabs(T[13]) > 1e-6 || fabs(T[14]) > 1e-6 || fabs(T[15] - 1.0) > 1e-6)
        return 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += T[k * 4 + a] * T[k * 4 + b];
            if (fabs(s - (a == b ? 1.0 : 0.0)) > 1e-6) return 0;
        }
    double det = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
                 T[2] * (T[4] * T[9] - T[5] * T[8]);
    return fabs(det - 1.0) <= 1e-6;
}

/*
 * Algorithm 1 with the Gauss-Newton update (solver 0), the exact
 * frozen-covariance Hessian (solver 1, the exact-Hessian variant, whose step
 * replaces the Gauss-Newton step where the exact model is concave and the step
 * stays within twice the Gauss-Newton step's length) or the
 * first-order ascent with the quartic line search and minimum step min_step
 * (solver 2), from T_init, with the length-scale annealing the
 * paper sketches for Sigma (reading):
 *   stage s uses ell_s; ell_0 = ell, ell_{s+1} = max(alpha * ell_s, ell_min);
 *   a non-final stage ends when ||xi||_1 < stage_tol or after
 *   max_iters_per_stage iterations; the final stage (ell_s == ell_min) runs
 *   until ||xi||_1 < tol; every stage counts toward max_iters in total.
 * Each iteration: transform Z by T^{-1}, freeze Sigma_ij at the current R
 * (Remark 2), evaluate f, g and the Hessian, step, retract T <- T exp(xi^).
 * SX/SZ may be NULL, in which case the shapes are computed with (knn, rho).
 * info[] receives: 0 status, 1 converged, 2 iterations, 3 stages used, 4 f,
 * 5..10 g, 11 ||xi||_1 of the last step, 12 pairs at the last iteration,
 * 13 damped steps (Newton: also steps taken with the Gauss-Newton system;
 * first-order: steps not taken at a quartic root), 14..29
 * iterations per stage (up to 16 stages).
 * On error T_out is left untouched.
 */
int orc_register_l(const double *X, const double *SXin, const double *LX, long nx, const double *Z,
                   const double *SZin, const double *LZ, long nz, int label_dim, const double T_init[16],
                   double ell, double ell_min, double alpha, double cutoff_scale, int knn, double rho,
                   double sigma2, int max_iters, int max_iters_per_stage, double tol, double stage_tol, int solver,
                   double min_step, double T_out[16], double info[32]);

int orc_register(const double *X, const double *SXin, long nx, const double *Z, const double *SZin,
                 long nz, const double T_init[16], double ell, double ell_min, double alpha,
                 double cutoff_scale, int knn, double rho, double sigma2, int max_iters,
                 int max_iters_per_stage, double tol, double stage_tol, int solver, double min_step,
                 double T_out[16], double info[32]) {
    return orc_register_l(X, SXin, NULL, nx, Z, SZin, NULL, nz, 0, T_init, ell, ell_min, alpha, cutoff_scale, knn,
                          rho, sigma2, max_iters, max_iters_per_stage, tol, stage_tol, solver, min_step, T_out,
                          info);
}

/* The registration with label weights c_ij (eq. (rkhs_loss)); labels may be NULL. */
int orc_register_l(const double *X, const double *SXin, const double *LX, long nx, const double *Z,
                   const double *SZin, const double *LZ, long nz, int label_dim, const double T_init[16],
                   double ell, double ell_min, double alpha, double cutoff_scale, int knn, double rho,
                   double sigma2, int max_iters, int max_iters_per_stage, double tol, double stage_tol, int solver,
                   double min_step, double T_out[16], double info[32]) {
    const int newton = (solver == 1), first_order = (solver == 2);
    for (int a = 0; a < 32; ++a) info[a] = 0.0;
    if (!X || !Z || !T_init || !T_out || nx < 0 || nz < 0 || !(ell > 0.0) || !(ell_min > 0.0) ||
        ell_min > ell || !(alpha > 0.0) || alpha > 1.0 || !(cutoff_scale > 0.0) || max_iters < 1 ||
        max_iters_per_stage < 1 || !(tol > 0.0) || !pose_is_rigid(T_init) || solver < 0 || solver > 2 ||
        (first_order && !(min_step > 0.0))) {
        info[0] = ORC_ERR_INVALID;
        return ORC_ERR_INVALID;
    }
    if (alpha == 1.0 && ell_min < ell) {
        info[0] = ORC_ERR_INVALID;
        return ORC_ERR_INVALID;
    }
    double *SX = NULL, *SZ = NULL;
    int st = ORC_OK;
    if (!SXin || !SZin) {
        if (nx < knn || nz < knn) { info[0] = ORC_ERR_TOO_FEW_POINTS; return ORC_ERR_TOO_FEW_POINTS; }
        SX = (double *)malloc(sizeof(double) * 6 * (size_t)(nx > 0 ? nx : 1));
        SZ = (double *)malloc(sizeof(double) * 6 * (size_t)(nz > 0 ? nz : 1));
        if (!SX || !SZ) { free(SX); free(SZ); info[0] = ORC_ERR_INVALID; return ORC_ERR_INVALID; }
        st = orc_point_shapes(X, nx, knn, rho, SX);
        if (st == ORC_OK) st = orc_point_shapes(Z, nz, knn, rho, SZ);
        if (st != ORC_OK) { free(SX); free(SZ); info[0] = st; return st; }
    }
    const double *sx = SXin ? SXin : SX, *sz = SZin ? SZin : SZ;

    double T[16];
    memcpy(T, T_init, sizeof T);
    double cur_ell = ell;
    int stage = 0, stage_it = 0, it = 0, converged = 0, damped_steps = 0;
    double f = 0.0, g[6] = {0}, xi_l1 = INFINITY;
    long long np = 0;
    while (it < max_iters) {
        double Hm[36], T1[36], T2[36], C[36], H[36];
        st = orc_eval_l(X, sx, LX, nx, Z, sz, LZ, nz, label_dim, T, NULL, cur_ell, cutoff_scale * cur_ell, sigma2,
                        &f, g, Hm, newton ? T1 : NULL, newton ? T2 : NULL, &np);
        if (st != ORC_OK) break;
        if (np == 0) { st = ORC_ERR_NO_PAIRS; break; }
        double xi[6];
        if (first_order) {
            /* gradient ascent along g with the line-search step (eq. (fo_update)) */
            double cl[5], mu;
            st = orc_line_coeffs_l(X, sx, LX, nx, Z, sz, LZ, nz, label_dim, T, cur_ell, cutoff_scale * cur_ell,
                                   sigma2, g, cl, NULL);
            if (st != ORC_OK) break;
            if (orc_first_order_step(cl, min_step, &mu) != 1) ++damped_steps;
            for (int a = 0; a < 6; ++a) xi[a] = mu * g[a];
        } else {
            orc_connection(g, C);
            for (int a = 0; a < 36; ++a) H[a] = Hm[a] + C[a];
            int dmp = 0;
            st = orc_solve_step(H, Hm, g, xi, &dmp);
            if (st != ORC_OK) break;
            int use_exact = 0;
            if (newton) {
                /* Newton (reading): the exact step replaces the Gauss-Newton
                 * step where the exact system's symmetric part is negative
                 * definite (a concave model), the step is an ascent direction,
                 * and it is at most twice as long as the Gauss-Newton step (a
                 * trust region borrowed from it).  Far from a maximum, pure
                 * Newton steps leave the basin. */
                double HE[36], mg[6], xn[6];
                for (int a = 0; a < 36; ++a) HE[a] = H[a] + T1[a] + T2[a];
                for (int a = 0; a < 6; ++a) mg[a] = -g[a];
                if (sym_negative_definite(HE) && solve_lu(HE, mg, xn, 6, 1e-12)) {
                    double gx = 0.0, nn = 0.0, ng = 0.0;
                    for (int a = 0; a < 6; ++a) {
                        gx += g[a] * xn[a];
                        nn += xn[a] * xn[a];
                        ng += xi[a] * xi[a];
                    }
                    if (gx > 0.0 && nn <= 4.0 * ng) {
                        memcpy(xi, xn, sizeof xn);
                        use_exact = 1;
                    }
                }
            }
            if (dmp || (newton && !use_exact)) ++damped_steps;
        }
        double E[16], Tn[16];
        orc_se3_exp(xi, E);
        matmul(T, E, Tn, 4, 4, 4);
        memcpy(T, Tn, sizeof T);
        xi_l1 = 0.0;
        for (int a = 0; a < 6; ++a) xi_l1 += fabs(xi[a]);
        ++it;
        ++stage_it;
        if (stage < 16) info[14 + stage] = stage_it;
        const int final_stage = !(cur_ell > ell_min);
        if (final_stage) {
            if (xi_l1 < tol) { converged = 1; break; }
        } else if (xi_l1 < stage_tol || stage_it >= max_iters_per_stage) {
            cur_ell = alpha * cur_ell;
            if (cur_ell < ell_min) cur_ell = ell_min;
            ++stage;
            stage_it = 0;
        }
    }
    free(SX);
    free(SZ);
    info[0] = st;
    if (st != ORC_OK) return st;
    memcpy(T_out, T, sizeof T);
    info[1] = converged;
    info[2] = it;
    info[3] = stage + 1;
    info[4] = f;
    for (int a = 0; a < 6; ++a) info[5 + a] = g[a];
    info[11] = xi_l1;
    info[12] = (double)np;
    info[13] = damped_steps;
    return ORC_OK;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
