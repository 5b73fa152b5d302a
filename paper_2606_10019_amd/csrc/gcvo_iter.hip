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
//
// All 6x6 algebra below is fully unrolled with compile-time indices so that it
// stays in registers (one lane per pair runs it).

// Solve A x = b (6x6) by Gaussian elimination with partial pivoting (rows of A
// and b swapped in place); false when a pivot is below tiny * max|A|.
__device__ __forceinline__ bool solve6(double A[6][6], double b[6], double x[6], double tiny) {
    double amax = 0.0;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) amax = fmax(amax, fabs(A[r][c]));
    if (!(amax > 0.0) || !isfinite(amax)) return false;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        int p = k;
        double best = fabs(A[k][k]);
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            const double v = fabs(A[r][k]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (!(best >= tiny * amax)) return false;
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            if (r == p) {
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    const double t = A[k][c];
                    A[k][c] = A[r][c];
                    A[r][c] = t;
                }
                const double t = b[k];
                b[k] = b[r];
                b[r] = t;
            }
        }
        const double inv = 1.0 / A[k][k];
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            const double f = A[r][k] * inv;
#pragma unroll
            for (int c = k + 1; c < 6; ++c) A[r][c] -= f * A[k][c];
            b[r] -= f * b[k];
        }
    }
#pragma unroll
    for (int r = 5; r >= 0; --r) {
        double acc = b[r];
#pragma unroll
        for (int c = r + 1; c < 6; ++c) acc -= A[r][c] * x[c];
        x[r] = acc / A[r][r];
    }
    return true;
}

// Damped Gauss-Newton step (reading of the damping the paper leaves open):
// plain H first; if singular or not an ascent direction, H_main shifted by
// -lambda * ||diag H_main||_2 with lambda = 1e-6 * 10^m, m = 0..6.
// Returns 0 (plain), m + 1 (damped) or -1 (failed).
__device__ __forceinline__ int damped_step(const double H[6][6], const double Hm[6][6], const double g[6],
                                           double xi[6]) {
    bool zero = true;
#pragma unroll
    for (int a = 0; a < 6; ++a) zero = zero && (g[a] == 0.0);
    if (zero) {
#pragma unroll
        for (int a = 0; a < 6; ++a) xi[a] = 0.0;
        return 0;
    }
    double dn = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) dn += Hm[a][a] * Hm[a][a];
    dn = sqrt(dn);
    for (int m = -1; m <= 6; ++m) {
        double A[6][6], b[6], x[6];
        const double shift = (m < 0) ? 0.0 : 1e-6 * exp10((double)m) * dn;
#pragma unroll
        for (int r = 0; r < 6; ++r) {
#pragma unroll
            for (int c = 0; c < 6; ++c) A[r][c] = (m < 0) ? H[r][c] : Hm[r][c];
            A[r][r] -= shift;
            b[r] = -g[r];
        }
        if (solve6(A, b, x, 1e-12)) {
            double gx = 0.0;
#pragma unroll
            for (int a = 0; a < 6; ++a) gx += g[a] * x[a];
            if (gx > 0.0) {
#pragma unroll
                for (int a = 0; a < 6; ++a) xi[a] = x[a];
                return m + 1;
            }
        }
    }
    return -1;
}

// exp of the twist (w, v): Rodrigues for the rotation, the left Jacobian V for
// the translation; half-angle form for (1 - cos)/th^2, series for small angles.
__device__ __forceinline__ void twist_exp(const double xi[6], double E[4][4]) {
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
    double V[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double W2 = w[r] * w[q] - (r == q ? th2 : 0.0);
            const double I = (r == q) ? 1.0 : 0.0;
            E[r][q] = I + a * W[r][q] + b * W2;
            V[r][q] = I + b * W[r][q] + c * W2;
        }
#pragma unroll
    for (int r = 0; r < 3; ++r) E[r][3] = V[r][0] * xi[3] + V[r][1] * xi[4] + V[r][2] * xi[5];
    E[3][0] = E[3][1] = E[3][2] = 0.0;
    E[3][3] = 1.0;
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

// FP64 tail of an iteration (one lane per pair): frame change of the summed
// terms, connection term, damped solve, retraction, stage and stop logic.
__device__ __forceinline__ void finish_iteration(PairDev &P, State &St, const double tot[kNumSums],
                                                 unsigned long long tot_pairs, int stage) {
    // Back to the caller's frame.  With K = -c^ and A = [[I, 0], [K, I]] (the
    // adjoint of the recentring translation): g = A^T g', H_main = A^T H' A.
    // In 3x3 blocks H' = [[P, Q], [Q^T, S]] this is
    //   [[P + QK + (QK)^T + K^T S K,  Q + (SK)^T], [Q^T + SK,  S]].
    const double cx = P.centre[0], cy = P.centre[1], cz = P.centre[2];
    const double K[3][3] = {{0.0, cz, -cy}, {-cz, 0.0, cx}, {cy, -cx, 0.0}};
    double Pm[3][3], Q[3][3], S[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Pm[r][c] = tot[7 + ut(r < c ? r : c, r < c ? c : r)];
            Q[r][c] = tot[7 + ut(r, 3 + c)];
            S[r][c] = tot[7 + ut(3 + (r < c ? r : c), 3 + (r < c ? c : r))];
        }
    double QK[3][3], SK[3][3], KSK[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            QK[r][c] = Q[r][0] * K[0][c] + Q[r][1] * K[1][c] + Q[r][2] * K[2][c];
            SK[r][c] = S[r][0] * K[0][c] + S[r][1] * K[1][c] + S[r][2] * K[2][c];
        }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) KSK[r][c] = K[0][r] * SK[0][c] + K[1][r] * SK[1][c] + K[2][r] * SK[2][c];
    const double sig = P.sigma2;
    double g[6], Hm[6][6];
    {
        const double gw[3] = {tot[1], tot[2], tot[3]}, gv[3] = {tot[4], tot[5], tot[6]};
        // g_w = g'_w + K^T g'_v, g_v = g'_v
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            g[r] = sig * (gw[r] + K[0][r] * gv[0] + K[1][r] * gv[1] + K[2][r] * gv[2]);
            g[3 + r] = sig * gv[r];
        }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Hm[r][c] = sig * (Pm[r][c] + QK[r][c] + QK[c][r] + KSK[r][c]);
            Hm[r][3 + c] = sig * (Q[r][c] + SK[c][r]);
            Hm[3 + r][c] = sig * (Q[c][r] + SK[r][c]);
            Hm[3 + r][3 + c] = sig * S[r][c];
        }
    const double f = sig * tot[0];
    // H_GN = H_main + C(g), C(g) = [[-1/2 g_w^, 0], [-g_v^, 0]]
    double H[6][6];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) H[r][c] = Hm[r][c];
    {
        const double Gw[3][3] = {{0.0, -g[2], g[1]}, {g[2], 0.0, -g[0]}, {-g[1], g[0], 0.0}};
        const double Gv[3][3] = {{0.0, -g[5], g[4]}, {g[5], 0.0, -g[3]}, {-g[4], g[3], 0.0}};
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                H[r][c] -= 0.5 * Gw[r][c];
                H[3 + r][c] -= Gv[r][c];
            }
    }
    St.f = f;
#pragma unroll
    for (int a = 0; a < 6; ++a) St.g[a] = g[a];
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) St.H[6 * r + c] = H[r][c];
    St.pairs_last = (long long)tot_pairs;
    if (P.iter_pairs && St.iter < P.max_iters) P.iter_pairs[St.iter] = (long long)tot_pairs;
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
    double E[4][4], T[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) T[r][c] = St.T[4 * r + c];
    twist_exp(xi, E);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) acc += T[r][b] * E[b][c];
            St.T[4 * r + c] = acc;
        }
    double l1 = 0.0;
#pragma unroll
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

// Lane layout of the pair kernel: a wave serves kGroupsPerWave neighbouring
// source points (sorted order), kGroupLanes lanes each.  Every point lists the
// contiguous x-rows of target cells that meet its cutoff ball; its lanes walk
// that list with stride kGroupLanes through a (row, offset) cursor, so no lane
// idles at row ends.  The 16 partial sums of a point are combined with xor
// shuffles.
template <typename Real>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_iterate(PairDev *pairs,
                                                                                          const BlockTask *tasks) {
    const BlockTask task = tasks[blockIdx.x];
    PairDev &P = pairs[task.pair];
    State &St = *P.st;
    if (St.done) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = lane / kGroupLanes, q = lane % kGroupLanes;
    const int stage = St.stage;
    const double ell = P.ell[stage];
    const Grid G = *P.t_grid[stage];
    const int *cells = P.t_cells[stage];
    const int nt = P.n_t, ns = P.n_s;
    constexpr bool kExact = sizeof(Real) == 8;   // FP64: recentre the original coordinates in FP64
    const float4 *trec = reinterpret_cast<const float4 *>(P.t_sorted[stage]);
    const double c0 = P.centre[0], c1 = P.centre[1], c2 = P.centre[2];

    // Recentred pose T' = C^{-1} T C: R' = R, t' = R c + t - c.
    double Rd[9], td[3];
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) Rd[3 * r + k] = St.T[4 * r + k];
        td[r] = St.T[4 * r + 3] - P.centre[r];
        for (int k = 0; k < 3; ++k) td[r] += Rd[3 * r + k] * P.centre[k];
    }

    const int j = task.block * kPointsPerBlock + wave * kGroupsPerWave + grp;
    const bool valid = j < ns;
    double y0 = 0.0, y1 = 0.0, y2 = 0.0;
    Real p00 = 0, p01 = 0, p02 = 0, p11 = 0, p12 = 0, p22 = 0;
    if (valid) {
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
        y0 = Rd[0] * zx + Rd[3] * zy + Rd[6] * zz;
        y1 = Rd[1] * zx + Rd[4] * zy + Rd[7] * zz;
        y2 = Rd[2] * zx + Rd[5] * zy + Rd[8] * zz;
        // S' = R^T S R
        const double S[3][3] = {{src[3 * ns + j], src[4 * ns + j], src[5 * ns + j]},
                                {src[4 * ns + j], src[6 * ns + j], src[7 * ns + j]},
                                {src[5 * ns + j], src[7 * ns + j], src[8 * ns + j]}};
        double SR[3][3], Sp[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) SR[a][b] = S[a][0] * Rd[b] + S[a][1] * Rd[3 + b] + S[a][2] * Rd[6 + b];
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b) Sp[a][b] = Rd[a] * SR[0][b] + Rd[3 + a] * SR[1][b] + Rd[6 + a] * SR[2][b];
        p00 = (Real)Sp[0][0]; p01 = (Real)Sp[0][1]; p02 = (Real)Sp[0][2];
        p11 = (Real)Sp[1][1]; p12 = (Real)Sp[1][2]; p22 = (Real)Sp[2][2];
    }
    const Real yx = (Real)y0, yy = (Real)y1, yz = (Real)y2;
    const double rc = P.cutoff_scale * ell;
    const Real rc2 = (Real)(rc * rc);
    const Real kexp = (Real)(-1.4426950408889634 / (ell * ell));   // f = exp2(q * inv_det * kexp)

    // Candidate rows of this point: the x-rows of cells (fixed cy, cz) that meet
    // the ball of radius rcm = 1.001 * cutoff around y, each clipped to the x
    // extent of the ball's section over that row.  A group's 16 lanes fill the
    // group's row table, then walk it with stride 16.
    __shared__ int sh_rs[kBlock / 64][kGroupsPerWave][kMaxRows], sh_rl[kBlock / 64][kGroupsPerWave][kMaxRows];
    PairSums<Real> s = {};
    unsigned cnt = 0;
    {
        const float rcm = (float)(rc * (double)kCellMargin);
        const float fy0 = (float)y0, fy1 = (float)y1, fy2 = (float)y2;
        const float gx = (fy0 - G.lo[0]) * G.inv_h, gy = (fy1 - G.lo[1]) * G.inv_h, gz = (fy2 - G.lo[2]) * G.inv_h;
        // radius in cell units, padded for the FP32 rounding of cell coordinates
        const float rh = rcm * G.inv_h + 4e-7f * fmaxf(fabsf(gx), fmaxf(fabsf(gy), fabsf(gz)));
        const int y_lo = max(0, (int)floorf(gy - rh)), y_hi = min(G.n[1] - 1, (int)floorf(gy + rh));
        const int z_lo = max(0, (int)floorf(gz - rh)), z_hi = min(G.n[2] - 1, (int)floorf(gz + rh));
        const int nyr = (valid && y_lo <= y_hi && z_lo <= z_hi) ? y_hi - y_lo + 1 : 0;
        const int nrows = (nyr > 0) ? nyr * (z_hi - z_lo + 1) : 0;
        int (*rs_t)[kMaxRows] = sh_rs[wave];
        int (*rl_t)[kMaxRows] = sh_rl[wave];
        for (int r0 = 0; r0 < nrows; r0 += kMaxRows) {
            const int nb = min(kMaxRows, nrows - r0);
            for (int r = q; r < nb; r += kGroupLanes) {
                const int cy = y_lo + (r0 + r) % nyr, cz = z_lo + (r0 + r) / nyr;
                // distance (cell units) from the point to the row's y-z square
                const float dy = fmaxf(0.0f, fmaxf((float)cy - gy, gy - (float)(cy + 1)));
                const float dz = fmaxf(0.0f, fmaxf((float)cz - gz, gz - (float)(cz + 1)));
                const float rem = rh * rh - dy * dy - dz * dz;
                int b = 0, len = 0;
                if (rem >= 0.0f) {
                    const float ext = sqrtf(rem);
                    const int x_lo = max(0, (int)floorf(gx - ext)), x_hi = min(G.n[0] - 1, (int)floorf(gx + ext));
                    if (x_lo <= x_hi) {
                        const int row = G.n[0] * (cy + G.n[1] * cz);
                        b = cells[row + x_lo];
                        len = cells[row + x_hi + 1] - b;
                    }
                }
                rs_t[grp][r] = b;
                rl_t[grp][r] = len;
            }
            __builtin_amdgcn_wave_barrier();
            int r = 0, o = q, rs = rs_t[grp][0], rl = rl_t[grp][0];
            while (r < nb && o >= rl) {
                o -= rl;
                if (++r < nb) { rs = rs_t[grp][r]; rl = rl_t[grp][r]; }
            }
            while (r < nb) {
                const float4 *rec = trec + 3 * (size_t)(rs + o);
                const float4 ra = rec[0], rb = rec[1], rcc = rec[2];
                const Real xx = kExact ? (Real)((double)rcc.y - c0) : (Real)ra.x;
                const Real xy = kExact ? (Real)((double)rcc.z - c1) : (Real)ra.y;
                const Real xz = kExact ? (Real)((double)rcc.w - c2) : (Real)ra.z;
                pair_term<Real>(s, cnt, xx - yx, xy - yy, xz - yz, (Real)ra.w + p00, (Real)rb.x + p01,
                                (Real)rb.y + p02, (Real)rb.z + p11, (Real)rb.w + p12, (Real)rcc.x + p22, rc2,
                                kexp);
                o += kGroupLanes;
                while (r < nb && o >= rl) {
                    o -= rl;
                    if (++r < nb) { rs = rs_t[grp][r]; rl = rl_t[grp][r]; }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
    }

    // Combine the 16 lanes of each point.
#pragma unroll
    for (int off = kGroupLanes / 2; off >= 1; off >>= 1) {
        s.F += __shfl_xor(s.F, off, 64);
        s.A0 += __shfl_xor(s.A0, off, 64); s.A1 += __shfl_xor(s.A1, off, 64); s.A2 += __shfl_xor(s.A2, off, 64);
        s.B00 += __shfl_xor(s.B00, off, 64); s.B01 += __shfl_xor(s.B01, off, 64);
        s.B02 += __shfl_xor(s.B02, off, 64); s.B11 += __shfl_xor(s.B11, off, 64);
        s.B12 += __shfl_xor(s.B12, off, 64); s.B22 += __shfl_xor(s.B22, off, 64);
    }

    // Finish the source point (lane 0 of its group): the 28 sums, recentred frame.
    __shared__ Real sh_pts[kPointsPerBlock][kNumSums];
    __shared__ unsigned sh_cnt[kBlock / 64];
    if (q == 0) {
        Real v[kNumSums];
        const Real k2 = valid ? (Real)(2.0 / (ell * ell)) : (Real)0;
        const Real a0 = k2 * s.A0, a1 = k2 * s.A1, a2 = k2 * s.A2;
        const Real b00 = k2 * s.B00, b01 = k2 * s.B01, b02 = k2 * s.B02;
        const Real b11 = k2 * s.B11, b12 = k2 * s.B12, b22 = k2 * s.B22;
        v[0] = valid ? s.F : (Real)0;
        // g_w = -y x a, g_v = -a
        v[1] = -(yy * a2 - yz * a1);
        v[2] = -(yz * a0 - yx * a2);
        v[3] = -(yx * a1 - yy * a0);
        v[4] = -a0; v[5] = -a1; v[6] = -a2;
        // Y = y^, M = Y B; H blocks: top-left Y B Y, top-right -Y B, bottom-right -B
        const Real B[3][3] = {{b00, b01, b02}, {b01, b11, b12}, {b02, b12, b22}};
        const Real Y[3][3] = {{0, -yz, yy}, {yz, 0, -yx}, {-yy, yx, 0}};
        Real M[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) M[r][c] = Y[r][0] * B[0][c] + Y[r][1] * B[1][c] + Y[r][2] * B[2][c];
        for (int r = 0; r < 3; ++r)
            for (int c = r; c < 3; ++c) v[7 + ut(r, c)] = M[r][0] * Y[0][c] + M[r][1] * Y[1][c] + M[r][2] * Y[2][c];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) v[7 + ut(r, 3 + c)] = -M[r][c];
        for (int r = 0; r < 3; ++r)
            for (int c = r; c < 3; ++c) v[7 + ut(3 + r, 3 + c)] = -B[r][c];
        const int slot = wave * kGroupsPerWave + grp;
#pragma unroll
        for (int k = 0; k < kNumSums; ++k) sh_pts[slot][k] = v[k];
    }
    cnt = wave_sum(cnt);
    if (lane == 0) sh_cnt[wave] = cnt;
    __syncthreads();
    Real *part = reinterpret_cast<Real *>(P.partials) + (size_t)task.block * kPartialStride;
    if (tid < kNumSums) {
        Real acc = 0;
        for (int pnt = 0; pnt < kPointsPerBlock; ++pnt) acc += sh_pts[pnt][tid];
        part[tid] = acc;
    }
    if (tid == kNumSums) {
        unsigned long long c = 0;
        for (int w = 0; w < kBlock / 64; ++w) c += sh_cnt[w];
        *reinterpret_cast<unsigned long long *>(part + kNumSums) = c;
    }

}

// Cross-block reduction of one pair's block sums, split over kReduceSplit
// blocks per pair.  Block s takes the pair-kernel blocks b = s (mod
// kReduceSplit); in it, thread t adds component t % 32 (the 28 sums and the
// pair count) over every 32nd of those blocks with a Kahan-compensated sum in
// the pair-term precision, and the 32 slices are added in FP64 in a fixed
// order.  The step kernel adds the kReduceSplit results, again in fixed order.
constexpr int kReduceThreads = 1024;
constexpr int kSlices = kReduceThreads / 32;

template <typename Real>
__global__ __launch_bounds__(kReduceThreads) void k_reduce(PairDev *pairs) {
    PairDev &P = pairs[blockIdx.y];
    State &St = *P.st;
    if (St.done) return;
    const int split = blockIdx.x;
    const int tid = threadIdx.x, ck = tid & 31, slice = tid >> 5;
    const Real *parts = reinterpret_cast<const Real *>(P.partials);
    __shared__ double sh[kSlices][33];
    __shared__ unsigned long long sh_c[kSlices];
    const int nb = P.n_blocks, step = kSlices * kReduceSplit;
    if (ck < kNumSums) {
        Real sm = 0, cp = 0;
        for (int b = split + kReduceSplit * slice; b < nb; b += step) {
            const Real y = parts[(size_t)b * kPartialStride + ck] - cp;
            const Real t = sm + y;
            cp = (t - sm) - y;
            sm = t;
        }
        sh[slice][ck] = (double)sm - (double)cp;
    } else if (ck == kNumSums) {
        unsigned long long c = 0;
        for (int b = split + kReduceSplit * slice; b < nb; b += step)
            c += *reinterpret_cast<const unsigned long long *>(parts + (size_t)b * kPartialStride + kNumSums);
        sh_c[slice] = c;
    }
    __syncthreads();
    if (tid < kNumSums) {
        double acc = 0.0;
        for (int sl = 0; sl < kSlices; ++sl) acc += sh[sl][tid];
        St.sub[split][tid] = acc;
    } else if (tid == kNumSums) {
        unsigned long long c = 0;
        for (int sl = 0; sl < kSlices; ++sl) c += sh_c[sl];
        St.sub_pairs[split] = c;
    }
}

// The FP64 step of one pair, on one lane (its registers are not shared with
// any wide kernel).  A pair that finishes decrements the batch's count of
// active pairs, which the host polls.
__global__ __launch_bounds__(64) void k_step(PairDev *pairs, int *active) {
    PairDev &P = pairs[blockIdx.x];
    State &St = *P.st;
    if (St.done || threadIdx.x != 0) return;
    double tot[kNumSums];
    unsigned long long c = 0;
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int sp = 0; sp < kReduceSplit; ++sp) acc += St.sub[sp][k];
        tot[k] = acc;
    }
#pragma unroll
    for (int sp = 0; sp < kReduceSplit; ++sp) c += St.sub_pairs[sp];
    finish_iteration(P, St, tot, c, St.stage);
    if (St.done) atomicSub(active, 1);
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

hipError_t launch_iterations(PairDev *pairs, int n_pairs, BlockTask *tasks, int n_tasks, int n_iters,
                             int precision, int *active, hipStream_t s) {
    if (n_tasks <= 0) return hipSuccess;
    for (int it = 0; it < n_iters; ++it) {
        if (precision == GCVO_PRECISION_FP64) {
            hipLaunchKernelGGL(k_iterate<double>, dim3(n_tasks), dim3(kBlock), 0, s, pairs, tasks);
            hipLaunchKernelGGL(k_reduce<double>, dim3(kReduceSplit, n_pairs), dim3(kReduceThreads), 0, s, pairs);
        } else {
            hipLaunchKernelGGL(k_iterate<float>, dim3(n_tasks), dim3(kBlock), 0, s, pairs, tasks);
            hipLaunchKernelGGL(k_reduce<float>, dim3(kReduceSplit, n_pairs), dim3(kReduceThreads), 0, s, pairs);
        }
        hipLaunchKernelGGL(k_step, dim3(n_pairs), dim3(64), 0, s, pairs, active);
    }
    return hipGetLastError();
}

hipError_t launch_count_active(PairDev *pairs, int n_pairs, int *active, hipStream_t s) {
    hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, s, pairs, n_pairs, active);
    return hipGetLastError();
}

}  // namespace gcvo
