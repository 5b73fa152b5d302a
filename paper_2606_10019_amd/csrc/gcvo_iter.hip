// One Gauss-Newton iteration of Algorithm 1 as a single kernel launch.
//
// Every block owns 256 source points of one pair (sorted by their own grid, so
// a block's points are spatially close).  Per point j:
//   y_j = R'^T (z_j - t'),  S'_j = R'^T S_j R'         (Alg. 1 transform; Remark 4)
// where T' = C^{-1} T C is the current pose in the frame recentred on the target
// centroid c.  The point scans the 3 x 3 x 3 neighbouring cells of the stage's
// target grid (9 contiguous x-rows), and for every target within the cutoff
//   S  = S_i + S'_j              (pair covariance = ell^2/2 * S, eq. (covariance))
//   C  = adj(S), det = det(S)    (so Sigma^{-1} = (2/ell^2) C / det)
//   q  = r^T C r,  f = exp(-q / (ell^2 det))              (eq. (kernel), sigma2 later)
//   F += f,  A += (f/det) C r,  B += (f/det) C
// Because J_j = [-y_j^, I] depends only on j (eq. (f_ij_J_j)), the pair sums
// finish per source point:
//   a = (2/ell^2) A, Bm = (2/ell^2) B
//   g_v -= a, g_w -= y x a                                     (Lemma 1)
//   H_main -= J^T Bm J = [[y^ Bm y^, -y^ Bm], [Bm y^, -Bm]]    (eq. (hessian_gn))
// The 28 sums are reduced per wave and per block in the pair-term precision
// (FP32 in the default path) and written as one block partial.  The last block
// of the pair to finish sums the partials with compensated per-lane sums and an
// FP64 tree, maps them back to the caller's frame, adds the connection term
// (eq. (connection_se3)), solves the damped 6x6 system in FP64, retracts
// T <- T exp(xi^) (eq. (gn_update)) and advances the stage/stop logic.
#include <math.h>

#include "gcvo_dev.h"

namespace gcvo {

template <typename R>
struct Fast;
template <>
struct Fast<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
};
template <>
struct Fast<double> {
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double exp2(double x) { return ::exp2(x); }
};

// ------------------------------------------------------------------ FP64 step

// Solve A x = b (6x6) by elimination with partial pivoting; false when a pivot
// is below tiny * max|A|.
__device__ __noinline__ bool lu_solve6(const double Ain[36], const double b[6], double x[6], double tiny) {
    double A[6][6], y[6];
    int perm[6];
    double amax = 0.0;
    for (int r = 0; r < 6; ++r) {
        perm[r] = r;
        for (int c = 0; c < 6; ++c) {
            A[r][c] = Ain[r * 6 + c];
            amax = fmax(amax, fabs(A[r][c]));
        }
    }
    if (!(amax > 0.0) || !isfinite(amax)) return false;
    for (int k = 0; k < 6; ++k) {
        int p = k;
        for (int r = k + 1; r < 6; ++r)
            if (fabs(A[r][k]) > fabs(A[p][k])) p = r;
        if (!(fabs(A[p][k]) >= tiny * amax)) return false;
        if (p != k) {
            for (int c = 0; c < 6; ++c) {
                double t = A[k][c]; A[k][c] = A[p][c]; A[p][c] = t;
            }
            int t = perm[k]; perm[k] = perm[p]; perm[p] = t;
        }
        for (int r = k + 1; r < 6; ++r) {
            A[r][k] /= A[k][k];
            for (int c = k + 1; c < 6; ++c) A[r][c] -= A[r][k] * A[k][c];
        }
    }
    for (int r = 0; r < 6; ++r) {   // forward substitution with the unit-lower factor
        double s = b[perm[r]];
        for (int c = 0; c < r; ++c) s -= A[r][c] * y[c];
        y[r] = s;
    }
    for (int r = 5; r >= 0; --r) {
        double s = y[r];
        for (int c = r + 1; c < 6; ++c) s -= A[r][c] * x[c];
        x[r] = s / A[r][r];
    }
    return true;
}

// Damped Gauss-Newton step (reading of the damping the paper leaves open):
// plain H first; if singular or not an ascent direction, H_main shifted by
// -lambda * ||diag H_main||_2 with lambda = 1e-6 * 10^m, m = 0..6.
// Returns 0 (plain), m + 1 (damped) or -1 (failed).
__device__ __noinline__ int damped_step(const double H[36], const double Hm[36], const double g[6], double xi[6]) {
    bool zero = true;
    double mg[6];
    for (int a = 0; a < 6; ++a) {
        mg[a] = -g[a];
        zero = zero && (g[a] == 0.0);
    }
    if (zero) {
        for (int a = 0; a < 6; ++a) xi[a] = 0.0;
        return 0;
    }
    double x[6];
    if (lu_solve6(H, mg, x, 1e-12)) {
        double gx = 0.0;
        for (int a = 0; a < 6; ++a) gx += g[a] * x[a];
        if (gx > 0.0) {
            for (int a = 0; a < 6; ++a) xi[a] = x[a];
            return 0;
        }
    }
    double dn = 0.0;
    for (int a = 0; a < 6; ++a) dn += Hm[7 * a] * Hm[7 * a];
    dn = sqrt(dn);
    double lam = 1e-6;
    for (int m = 0; m <= 6; ++m, lam *= 10.0) {
        double Hd[36];
        for (int e = 0; e < 36; ++e) Hd[e] = Hm[e];
        for (int a = 0; a < 6; ++a) Hd[7 * a] -= lam * dn;
        if (lu_solve6(Hd, mg, x, 1e-12)) {
            double gx = 0.0;
            for (int a = 0; a < 6; ++a) gx += g[a] * x[a];
            if (gx > 0.0) {
                for (int a = 0; a < 6; ++a) xi[a] = x[a];
                return m + 1;
            }
        }
    }
    return -1;
}

// exp of the twist (w, v): Rodrigues for the rotation, the left Jacobian V for
// the translation; half-angle form for (1 - cos)/th^2, series for small angles.
__device__ __noinline__ void twist_exp(const double xi[6], double E[16]) {
    const double wx = xi[0], wy = xi[1], wz = xi[2];
    const double th2 = wx * wx + wy * wy + wz * wz, th = sqrt(th2);
    double a, b, c;
    if (th < 1e-5) {
        a = 1.0 - th2 / 6.0;
        b = 0.5 - th2 / 24.0;
    } else {
        const double sh = sin(0.5 * th) / (0.5 * th);
        a = sin(th) / th;
        b = 0.5 * sh * sh;
    }
    if (th < 1e-2)
        c = (1.0 / 6.0) - th2 * (1.0 / 120.0) + th2 * th2 * (1.0 / 5040.0);
    else
        c = (th - sin(th)) / (th2 * th);
    // W = w^, W^2 = w w^T - th2 I
    const double W[3][3] = {{0.0, -wz, wy}, {wz, 0.0, -wx}, {-wy, wx, 0.0}};
    const double w[3] = {wx, wy, wz};
    double Rm[3][3], V[3][3];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
            const double W2 = w[r] * w[q] - (r == q ? th2 : 0.0);
            const double I = (r == q) ? 1.0 : 0.0;
            Rm[r][q] = I + a * W[r][q] + b * W2;
            V[r][q] = I + b * W[r][q] + c * W2;
        }
    for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) E[4 * r + q] = Rm[r][q];
        E[4 * r + 3] = V[r][0] * xi[3] + V[r][1] * xi[4] + V[r][2] * xi[5];
    }
    E[12] = E[13] = E[14] = 0.0;
    E[15] = 1.0;
}

// ------------------------------------------------------------------ pair kernel

template <typename Real>
struct PairSums {
    Real F, A0, A1, A2, B00, B01, B02, B11, B12, B22;
};

template <typename Real>
__device__ __forceinline__ void pair_term(PairSums<Real> &s, unsigned &cnt, Real rx, Real ry, Real rz,
                                          Real s00, Real s01, Real s02, Real s11, Real s12, Real s22,
                                          Real rc2, Real kexp) {
    const Real d2 = rx * rx + ry * ry + rz * rz;
    if (d2 <= rc2) {
        const Real c00 = s11 * s22 - s12 * s12;
        const Real c01 = s02 * s12 - s01 * s22;
        const Real c02 = s01 * s12 - s02 * s11;
        const Real c11 = s00 * s22 - s02 * s02;
        const Real c12 = s01 * s02 - s00 * s12;
        const Real c22 = s00 * s11 - s01 * s01;
        const Real det = s00 * c00 + s01 * c01 + s02 * c02;
        const Real inv = Fast<Real>::rcp(det);
        const Real ux = c00 * rx + c01 * ry + c02 * rz;
        const Real uy = c01 * rx + c11 * ry + c12 * rz;
        const Real uz = c02 * rx + c12 * ry + c22 * rz;
        const Real q = rx * ux + ry * uy + rz * uz;
        const Real f = Fast<Real>::exp2(q * (inv * kexp));
        const Real w = f * inv;
        s.F += f;
        s.A0 += w * ux; s.A1 += w * uy; s.A2 += w * uz;
        s.B00 += w * c00; s.B01 += w * c01; s.B02 += w * c02;
        s.B11 += w * c11; s.B12 += w * c12; s.B22 += w * c22;
        ++cnt;
    }
}

// Upper-triangle index of (r, c), r <= c, in row-major order of a 6x6 matrix.
__host__ __device__ constexpr int ut(int r, int c) { return r * 6 - (r * (r - 1)) / 2 + (c - r); }

// Single-thread FP64 tail of an iteration: frame change of the summed terms,
// connection term, damped solve, retraction, stage and stop logic.  Kept out of
// line so that its registers do not limit the occupancy of the pair loop.
__device__ __noinline__ void finish_iteration(PairDev &P, State &St, const double *tot,
                                              unsigned long long tot_pairs, int stage) {
    // Back to the caller's frame: with A = [[I, 0], [-c^, I]] (the adjoint of the
    // recentring translation), g = A^T g', H_main = A^T H' A.
    double gp[6], Hp[36];
    for (int a = 0; a < 6; ++a) gp[a] = tot[1 + a];
    for (int r = 0; r < 6; ++r)
        for (int c = r; c < 6; ++c) Hp[6 * r + c] = Hp[6 * c + r] = tot[7 + ut(r, c)];
    const double *cc = P.centre;
    const double Ch[3][3] = {{0.0, -cc[2], cc[1]}, {cc[2], 0.0, -cc[0]}, {-cc[1], cc[0], 0.0}};
    double A[36];
    for (int e = 0; e < 36; ++e) A[e] = 0.0;
    for (int a = 0; a < 6; ++a) A[7 * a] = 1.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) A[6 * (3 + r) + c] = -Ch[r][c];
    double g[6], HA[36], Hm[36];
    for (int a = 0; a < 6; ++a) {
        double acc = 0.0;
        for (int b = 0; b < 6; ++b) acc += A[6 * b + a] * gp[b];
        g[a] = acc;
    }
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            double acc = 0.0;
            for (int b = 0; b < 6; ++b) acc += Hp[6 * r + b] * A[6 * b + c];
            HA[6 * r + c] = acc;
        }
    for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
            double acc = 0.0;
            for (int b = 0; b < 6; ++b) acc += A[6 * b + r] * HA[6 * b + c];
            Hm[6 * r + c] = acc;
        }
    const double sig = P.sigma2;
    const double f = sig * tot[0];
    for (int a = 0; a < 6; ++a) g[a] *= sig;
    for (int e = 0; e < 36; ++e) Hm[e] *= sig;
    // H_GN = H_main + C(g), C(g) = [[-1/2 g_w^, 0], [-g_v^, 0]]
    double H[36];
    for (int e = 0; e < 36; ++e) H[e] = Hm[e];
    {
        const double gw[3] = {g[0], g[1], g[2]}, gv[3] = {g[3], g[4], g[5]};
        const double Gw[3][3] = {{0.0, -gw[2], gw[1]}, {gw[2], 0.0, -gw[0]}, {-gw[1], gw[0], 0.0}};
        const double Gv[3][3] = {{0.0, -gv[2], gv[1]}, {gv[2], 0.0, -gv[0]}, {-gv[1], gv[0], 0.0}};
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                H[6 * r + c] -= 0.5 * Gw[r][c];
                H[6 * (3 + r) + c] -= Gv[r][c];
            }
    }
    St.f = f;
    for (int a = 0; a < 6; ++a) St.g[a] = g[a];
    for (int e = 0; e < 36; ++e) St.H[e] = H[e];
    St.pairs_last = (long long)tot_pairs;
    if (P.iter_pairs && St.iter < P.max_iters) P.iter_pairs[St.iter] = (long long)tot_pairs;
    St.counter = 0;
    if (P.eval_only) {
        St.done = 1;
        return;
    }
    if (tot_pairs == 0) {
        St.status = GCVO_ERR_NO_PAIRS;
        St.done = 1;
        return;
    }
    double xi[6];
    const int dmp = damped_step(H, Hm, g, xi);
    if (dmp < 0) {
        St.status = GCVO_ERR_SINGULAR;
        St.done = 1;
        return;
    }
    if (dmp > 0) ++St.damped;
    double E[16], Tn[16];
    twist_exp(xi, E);
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
            for (int b = 0; b < 4; ++b) acc += St.T[4 * r + b] * E[4 * b + c];
            Tn[4 * r + c] = acc;
        }
    for (int e = 0; e < 16; ++e) St.T[e] = Tn[e];
    double l1 = 0.0;
    for (int a = 0; a < 6; ++a) {
        St.xi[a] = xi[a];
        l1 += fabs(xi[a]);
    }
    St.xi_l1 = l1;
    St.iter += 1;
    St.stage_iter += 1;
    St.stage_iters[stage] = St.stage_iter;
    const bool final_stage = (stage + 1 >= P.n_stages);
    if (final_stage) {
        if (l1 < P.tol) {
            St.converged = 1;
            St.done = 1;
        }
    } else if (l1 < P.stage_tol || St.stage_iter >= P.max_per_stage) {
        St.stage = stage + 1;
        St.stage_iter = 0;
    }
    if (St.iter >= P.max_iters) St.done = 1;
}

template <typename Real>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_iterate(PairDev *pairs, const BlockTask *tasks) {
    const BlockTask task = tasks[blockIdx.x];
    PairDev &P = pairs[task.pair];
    State &St = *P.st;
    if (St.done) return;
    const int tid = threadIdx.x;
    const int stage = St.stage;
    const double ell = P.ell[stage];
    const Grid G = *P.t_grid[stage];
    const int *cells = P.t_cells[stage];
    const int nt = P.n_t, ns = P.n_s;
    constexpr bool kExact = sizeof(Real) == 8;   // FP64: recentre the original coordinates in FP64
    const float *tx = P.t_sorted[stage], *ty = tx + nt, *tz = ty + nt;
    const float *t0 = tz + nt, *t1 = t0 + nt, *t2 = t1 + nt, *t3 = t2 + nt, *t4 = t3 + nt, *t5 = t4 + nt;
    const float *ox = t5 + nt, *oy = ox + nt, *oz = oy + nt;
    const double c0 = P.centre[0], c1 = P.centre[1], c2 = P.centre[2];

    // Recentred pose T' = C^{-1} T C: R' = R, t' = R c + t - c.
    double Rd[9], td[3];
    for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) Rd[3 * r + q] = St.T[4 * r + q];
        td[r] = St.T[4 * r + 3] - P.centre[r];
        for (int q = 0; q < 3; ++q) td[r] += Rd[3 * r + q] * P.centre[q];
    }

    PairSums<Real> s = {};
    unsigned cnt = 0;
    const int j = task.block * kBlock + tid;
    Real yx = 0, yy = 0, yz = 0;
    if (j < ns) {
        const float *src = P.s_sorted;
        double zx, zy, zz;
        if (kExact) {
            zx = ((double)src[9 * ns + j] - c0) - td[0];
            zy = ((double)src[10 * ns + j] - c1) - td[1];
            zz = ((double)src[11 * ns + j] - c2) - td[2];
        } else {
            zx = (double)src[j] - td[0];
            zy = (double)src[ns + j] - td[1];
            zz = (double)src[2 * ns + j] - td[2];
        }
        // y = R^T (z - t)
        const double y0 = Rd[0] * zx + Rd[3] * zy + Rd[6] * zz;
        const double y1 = Rd[1] * zx + Rd[4] * zy + Rd[7] * zz;
        const double y2 = Rd[2] * zx + Rd[5] * zy + Rd[8] * zz;
        yx = (Real)y0; yy = (Real)y1; yz = (Real)y2;
        // S' = R^T S R
        const double S[3][3] = {{src[3 * ns + j], src[4 * ns + j], src[5 * ns + j]},
                                {src[4 * ns + j], src[6 * ns + j], src[7 * ns + j]},
                                {src[5 * ns + j], src[7 * ns + j], src[8 * ns + j]}};
        double SR[3][3], Sp[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) SR[a][b] = S[a][0] * Rd[b] + S[a][1] * Rd[3 + b] + S[a][2] * Rd[6 + b];
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b) Sp[a][b] = Rd[a] * SR[0][b] + Rd[3 + a] * SR[1][b] + Rd[6 + a] * SR[2][b];
        const Real p00 = (Real)Sp[0][0], p01 = (Real)Sp[0][1], p02 = (Real)Sp[0][2];
        const Real p11 = (Real)Sp[1][1], p12 = (Real)Sp[1][2], p22 = (Real)Sp[2][2];

        const double rc = P.cutoff_scale * ell;
        const Real rc2 = (Real)(rc * rc);
        // f = exp(-q / (ell^2 det)) = exp2(q * inv_det * kexp)
        const Real kexp = (Real)(-1.4426950408889634 / (ell * ell));
        const float fyx = (float)y0, fyy = (float)y1, fyz = (float)y2;
        const int cx = (int)floorf((fyx - G.lo[0]) * G.inv_h);
        const int cy = (int)floorf((fyy - G.lo[1]) * G.inv_h);
        const int cz = (int)floorf((fyz - G.lo[2]) * G.inv_h);
        const int x0 = max(cx - 1, 0), x1 = min(cx + 1, G.n[0] - 1);
        if (x0 <= x1) {
            for (int dz = -1; dz <= 1; ++dz) {
                const int zc = cz + dz;
                if (zc < 0 || zc >= G.n[2]) continue;
                for (int dy = -1; dy <= 1; ++dy) {
                    const int yc = cy + dy;
                    if (yc < 0 || yc >= G.n[1]) continue;
                    const int row = G.n[0] * (yc + G.n[1] * zc);
                    const int b = cells[row + x0], e = cells[row + x1 + 1];
                    for (int i = b; i < e; ++i) {
                        const Real xx = kExact ? (Real)((double)ox[i] - c0) : (Real)tx[i];
                        const Real xy = kExact ? (Real)((double)oy[i] - c1) : (Real)ty[i];
                        const Real xz = kExact ? (Real)((double)oz[i] - c2) : (Real)tz[i];
                        pair_term<Real>(s, cnt, xx - yx, xy - yy, xz - yz,
                                        (Real)t0[i] + p00, (Real)t1[i] + p01, (Real)t2[i] + p02,
                                        (Real)t3[i] + p11, (Real)t4[i] + p12, (Real)t5[i] + p22, rc2, kexp);
                    }
                }
            }
        }
    }

    // Finish the source point: the 28 sums in the recentred frame.
    Real v[kNumSums];
    {
        const Real k2 = (Real)(2.0 / (ell * ell));
        const Real a0 = k2 * s.A0, a1 = k2 * s.A1, a2 = k2 * s.A2;
        const Real b00 = k2 * s.B00, b01 = k2 * s.B01, b02 = k2 * s.B02;
        const Real b11 = k2 * s.B11, b12 = k2 * s.B12, b22 = k2 * s.B22;
        v[0] = s.F;
        // g_w = -y x a, g_v = -a
        v[1] = -(yy * a2 - yz * a1);
        v[2] = -(yz * a0 - yx * a2);
        v[3] = -(yx * a1 - yy * a0);
        v[4] = -a0; v[5] = -a1; v[6] = -a2;
        // Y = y^, M = Y B  (B symmetric)
        const Real B[3][3] = {{b00, b01, b02}, {b01, b11, b12}, {b02, b12, b22}};
        const Real Y[3][3] = {{0, -yz, yy}, {yz, 0, -yx}, {-yy, yx, 0}};
        Real M[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) M[r][c] = Y[r][0] * B[0][c] + Y[r][1] * B[1][c] + Y[r][2] * B[2][c];
        // top-left Y B Y, top-right -Y B, bottom-right -B
        for (int r = 0; r < 3; ++r)
            for (int c = r; c < 3; ++c)
                v[7 + ut(r, c)] = M[r][0] * Y[0][c] + M[r][1] * Y[1][c] + M[r][2] * Y[2][c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) v[7 + ut(r, 3 + c)] = -M[r][c];
        for (int r = 0; r < 3; ++r)
            for (int c = r; c < 3; ++c) v[7 + ut(3 + r, 3 + c)] = -B[r][c];
    }

    // Block reduction in Real: wave sums, then the 4 waves in fixed order.
    __shared__ Real sh[4][kNumSums];
    __shared__ unsigned sh_cnt[4];
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) v[k] = wave_sum(v[k]);
    cnt = wave_sum(cnt);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < kNumSums; ++k) sh[wave][k] = v[k];
        sh_cnt[wave] = cnt;
    }
    __syncthreads();
    Real *part = reinterpret_cast<Real *>(P.partials) + (size_t)task.block * kPartialStride;
    if (tid < kNumSums) part[tid] = ((sh[0][tid] + sh[1][tid]) + sh[2][tid]) + sh[3][tid];
    if (tid == kNumSums)
        *reinterpret_cast<unsigned long long *>(part + kNumSums) =
            (unsigned long long)sh_cnt[0] + sh_cnt[1] + sh_cnt[2] + sh_cnt[3];

    // Last block of this pair: reduce, step, advance.
    __shared__ int sh_last;
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const unsigned prev = __hip_atomic_fetch_add(&St.counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        sh_last = (prev == (unsigned)(P.n_blocks - 1));
    }
    __syncthreads();
    if (!sh_last) return;
    __threadfence();

    __shared__ double tot[kNumSums];
    __shared__ unsigned long long tot_pairs;
    const Real *parts = reinterpret_cast<const Real *>(P.partials);
    for (int k = wave; k < kNumSums + 1; k += 4) {
        if (k < kNumSums) {
            // compensated per-lane sum over the lane's blocks, then an FP64 tree
            Real sum = 0, comp = 0;
            for (int b = lane; b < P.n_blocks; b += 64) {
                const Real x = __builtin_nontemporal_load(parts + (size_t)b * kPartialStride + k) - comp;
                const Real t = sum + x;
                comp = (t - sum) - x;
                sum = t;
            }
            double d = (double)sum - (double)comp;
            d = wave_sum(d);
            if (lane == 0) tot[k] = d;
        } else {
            unsigned long long c = 0;
            for (int b = lane; b < P.n_blocks; b += 64)
                c += __builtin_nontemporal_load(
                    reinterpret_cast<const unsigned long long *>(parts + (size_t)b * kPartialStride + kNumSums));
            c = wave_sum(c);
            if (lane == 0) tot_pairs = c;
        }
    }
    __syncthreads();
    if (tid != 0) return;

    finish_iteration(P, St, tot, tot_pairs, stage);
}

__global__ void k_count_active(const PairDev *pairs, int n_pairs, int *active) {
    __shared__ int sh[4];
    int c = 0;
    for (int p = threadIdx.x; p < n_pairs; p += blockDim.x) c += pairs[p].st->done ? 0 : 1;
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) *active = sh[0] + sh[1] + sh[2] + sh[3];
}

hipError_t launch_iterations(PairDev *pairs, BlockTask *tasks, int n_tasks, int n_iters, int precision,
                             hipStream_t s) {
    if (n_tasks <= 0) return hipSuccess;
    for (int it = 0; it < n_iters; ++it) {
        if (precision == GCVO_PRECISION_FP64)
            hipLaunchKernelGGL(k_iterate<double>, dim3(n_tasks), dim3(kBlock), 0, s, pairs, tasks);
        else
            hipLaunchKernelGGL(k_iterate<float>, dim3(n_tasks), dim3(kBlock), 0, s, pairs, tasks);
    }
    return hipGetLastError();
}

hipError_t launch_count_active(PairDev *pairs, int n_pairs, int *active, hipStream_t s) {
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, s, pairs, n_pairs, active);
    return hipGetLastError();
}

}  // namespace gcvo
