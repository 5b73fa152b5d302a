// Solver iterations of Algorithm 1: the pair kernel, the cross-block reduction
// and the FP64 step, for the three solvers.
//
// Pair kernel (k_iterate).  A block serves kPointsPerBlock source points of one
// pair (Morton order, so a block's points are close), kGroupLanes lanes per
// point.  Per point j:
//   y_j = R'^T (z_j - t'),  S'_j = R'^T S_j R'         (Alg. 1 transform; Remark 4)
// where T' is the current pose in the frame recentred on the target centroid.
// The point lists the x-rows of target cells that meet its cutoff ball, and
// for every target within the cutoff
//   S  = S_i + S'_j              (pair covariance = ell^2/2 * S, eq. (covariance))
//   C  = adj(S), det = det(S)    (so Sigma^{-1} = (2/ell^2) C / det)
//   q  = r^T C r,  f = exp(-q / (ell^2 det))              (eq. (kernel), sigma2 later)
//   F += f,  A += (f/det) C r,  B += (f/det) C
// Because J_j = [-y_j^, I] depends only on j (eq. (f_ij_J_j)), the pair sums
// finish per source point:
//   a = (2/ell^2) A, Bm = (2/ell^2) B
//   g_v -= a, g_w -= y x a                                     (Lemma 1)
//   H_main -= J^T Bm J = [[y^ Bm y^, -y^ Bm], [Bm y^, -Bm]]    (eq. (hessian_gn))
// Pass modes:
//   kModeGN     the 28 sums above (Gauss-Newton, and the gradient pass of the
//               first-order solver);
//   kModeExact  also Q = sum_i f u u^T (u = Sigma^{-1} r) per point, giving the
//               product-rule term T1 = J^T Q J, and sum_j y_j a_j^T, giving the
//               derivative-of-J term T2 (eq. (direction_derivative_gradf)):
//               the exact frozen-covariance Hessian of the exact-Hessian solver;
//   kModeLine   the quartic line-search coefficients along a unit direction
//               (first-order solver, App. "Line search", re-derived).
// Sums are reduced per point (DPP row permutations over the point's 16 lanes)
// and per block in the pair-term precision and written as one block partial;
// the FP64 transform and the per-point finish run once per block, on wave 0.
//
// Reduction (k_reduce): kReduceSplit blocks per pair sum the block partials
// with compensated per-lane sums and FP64 slices.  Step (k_step): one lane per
// pair adds the splits in FP64, maps the sums back to the caller's frame, adds
// the connection term (eq. (connection_se3)), solves in FP64 (damped Gauss-Newton
// or Newton system, or the line-search root), retracts T <- T exp(xi^)
// (eq. (gn_update)) and advances the stage/stop logic.
#include <hip/hip_ext.h>
#include <math.h>

#include <type_traits>

#include "gcvo_dev.h"

namespace gcvo {

// 1/x from the hardware estimate refined by two Newton-Raphson steps
// (r <- r + r (1 - x r), each squaring the relative error): within an ulp or so
// of the rounded quotient for normal x whose reciprocal is normal, in about a
// third of the instructions of an IEEE division.
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

template <typename R>
struct Fast;
template <>
struct Fast<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
};
template <>
struct Fast<double> {
    static __device__ __forceinline__ double rcp(double x) { return rcp_nr(x); }   // det > 0 for pairs
    static __device__ __forceinline__ double exp2(double x) { return ::exp2(x); }
};

// ------------------------------------------------------------------ FP64 step
//
// All 6x6 algebra below is fully unrolled with compile-time indices so that it
// stays in registers (one lane per pair runs it).

// Solve A x = b (6x6) by Gaussian elimination with partial pivoting on the
// augmented matrix M = [A | b] (rows swapped in place; b in column 6, so that
// the swaps of b stay in registers like those of A); false when a pivot is
// below tiny * max|A|.
__device__ __forceinline__ bool solve6(double M[6][7], double x[6], double tiny) {
    // max |A| as a tree of fmax (exact, so any order gives the same value)
    double rmax[6];
#pragma unroll
    for (int r = 0; r < 6; ++r)
        rmax[r] = fmax(fmax(fmax(fabs(M[r][0]), fabs(M[r][1])), fmax(fabs(M[r][2]), fabs(M[r][3]))),
                       fmax(fabs(M[r][4]), fabs(M[r][5])));
    const double amax = fmax(fmax(0.0, fmax(rmax[0], rmax[1])), fmax(fmax(rmax[2], rmax[3]), fmax(rmax[4], rmax[5])));
    if (!(amax > 0.0) || !isfinite(amax)) return false;
    double invd[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        int p = k;
        double best = fabs(M[k][k]);
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            const double v = fabs(M[r][k]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (!(best >= tiny * amax)) return false;
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            if (r == p) {   // columns left of k are no longer read
#pragma unroll
                for (int c = k; c < 7; ++c) {
                    const double t = M[k][c];
                    M[k][c] = M[r][c];
                    M[r][c] = t;
                }
            }
        }
        const double inv = rcp_nr(M[k][k]);
        invd[k] = inv;
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            const double f = M[r][k] * inv;
#pragma unroll
            for (int c = k + 1; c < 7; ++c) M[r][c] -= f * M[k][c];
        }
    }
#pragma unroll
    for (int r = 5; r >= 0; --r) {
        double acc = M[r][6];
#pragma unroll
        for (int c = r + 1; c < 6; ++c) acc -= M[r][c] * x[c];
        x[r] = acc * invd[r];
    }
    return true;
}

// 3x3 adjugate (adj(M) M = det(M) I); returns det(M).
__device__ __forceinline__ double adj3(const double m[3][3], double a[3][3]) {
    a[0][0] = m[1][1] * m[2][2] - m[1][2] * m[2][1];
    a[0][1] = m[0][2] * m[2][1] - m[0][1] * m[2][2];
    a[0][2] = m[0][1] * m[1][2] - m[0][2] * m[1][1];
    a[1][0] = m[1][2] * m[2][0] - m[1][0] * m[2][2];
    a[1][1] = m[0][0] * m[2][2] - m[0][2] * m[2][0];
    a[1][2] = m[0][2] * m[1][0] - m[0][0] * m[1][2];
    a[2][0] = m[1][0] * m[2][1] - m[1][1] * m[2][0];
    a[2][1] = m[0][1] * m[2][0] - m[0][0] * m[2][1];
    a[2][2] = m[0][0] * m[1][1] - m[0][1] * m[1][0];
    return m[0][0] * a[0][0] + m[0][1] * a[1][0] + m[0][2] * a[2][0];
}

// Maximum absolute row sum of a 3x3 matrix.
__device__ __forceinline__ double norm_inf3(const double m[3][3]) {
    return fmax(fmax(fabs(m[0][0]) + fabs(m[0][1]) + fabs(m[0][2]), fabs(m[1][0]) + fabs(m[1][1]) + fabs(m[1][2])),
                fabs(m[2][0]) + fabs(m[2][1]) + fabs(m[2][2]));
}

// Solve H x = -g through the Schur complement of the lower-right 3x3 block, for
// a well-conditioned H only.  With H = [[A, B], [C, D]] in 3x3 blocks, Di = D^-1,
// E = B Di and S = A - E C:  x1 = S^-1 (r1 - E r2), x2 = Di (r2 - C x1), r = -g.
// From the block form of H^-1,
//   ||H^-1||_inf <= (1 + ||Di|| ||C||) (1 + ||E||) ||S^-1|| + ||Di||,
// and every pivot of the partial-pivoting elimination of H (H = P L U with
// |l_ij| <= 1) has |u_kk| >= 1 / (6 ||H^-1||_inf).  So when that bound times
// max|H| is at most kBlockCond, every pivot of solve6 exceeds its threshold
// 1e-12 max|H| by a factor of 16 or more: both methods take the same branch and
// their solutions differ by rounding only.  Returns false (x untouched) unless
// the bound holds (also for singular D or S and non-finite entries).  Some 200
// operations without branches, against ~600 with pivot search and row swaps.
constexpr double kBlockCond = 1e10;
__device__ __forceinline__ bool solve6_blocks(const double H[6][6], const double g[6], double x[6]) {
    double A[3][3], B[3][3], C[3][3], D[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            A[r][c] = H[r][c];
            B[r][c] = H[r][3 + c];
            C[r][c] = H[3 + r][c];
            D[r][c] = H[3 + r][3 + c];
        }
    double rmax[6];
#pragma unroll
    for (int r = 0; r < 6; ++r)
        rmax[r] = fmax(fmax(fmax(fabs(H[r][0]), fabs(H[r][1])), fmax(fabs(H[r][2]), fabs(H[r][3]))),
                       fmax(fabs(H[r][4]), fabs(H[r][5])));
    const double amax = fmax(fmax(rmax[0], rmax[1]), fmax(fmax(rmax[2], rmax[3]), fmax(rmax[4], rmax[5])));
    double Da[3][3], Di[3][3], E[3][3], S[3][3], Sa[3][3];
    const double iD = rcp_nr(adj3(D, Da));
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Di[r][c] = Da[r][c] * iD;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) E[r][c] = B[r][0] * Di[0][c] + B[r][1] * Di[1][c] + B[r][2] * Di[2][c];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) S[r][c] = A[r][c] - (E[r][0] * C[0][c] + E[r][1] * C[1][c] + E[r][2] * C[2][c]);
    const double iS = rcp_nr(adj3(S, Sa));
    const double nDi = norm_inf3(Di);
    const double bound = ((1.0 + nDi * norm_inf3(C)) * (1.0 + norm_inf3(E)) * (norm_inf3(Sa) * fabs(iS)) + nDi) * amax;
    if (!(bound <= kBlockCond)) return false;
    const double r1[3] = {-g[0], -g[1], -g[2]}, r2[3] = {-g[3], -g[4], -g[5]};
    double t[3], x1[3], u[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) t[r] = r1[r] - (E[r][0] * r2[0] + E[r][1] * r2[1] + E[r][2] * r2[2]);
#pragma unroll
    for (int r = 0; r < 3; ++r) x1[r] = (Sa[r][0] * t[0] + Sa[r][1] * t[1] + Sa[r][2] * t[2]) * iS;
#pragma unroll
    for (int r = 0; r < 3; ++r) u[r] = r2[r] - (C[r][0] * x1[0] + C[r][1] * x1[1] + C[r][2] * x1[2]);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        x[r] = x1[r];
        x[3 + r] = Di[r][0] * u[0] + Di[r][1] * u[1] + Di[r][2] * u[2];
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
    {   // plain H: the block solve where it is well conditioned, else the
        // pivoting elimination (its own copy of the solve, so that H's registers
        // serve as the working matrix without a select between H and H_main)
        double x[6];
        bool solved = solve6_blocks(H, g, x);
        if (!solved) {
            double A[6][7];
#pragma unroll
            for (int r = 0; r < 6; ++r) {
#pragma unroll
                for (int c = 0; c < 6; ++c) A[r][c] = H[r][c];
                A[r][6] = -g[r];
            }
            solved = solve6(A, x, 1e-12);
        }
        if (solved) {
            double gx = 0.0;
#pragma unroll
            for (int a = 0; a < 6; ++a) gx += g[a] * x[a];
            if (gx > 0.0) {
#pragma unroll
                for (int a = 0; a < 6; ++a) xi[a] = x[a];
                return 0;
            }
        }
    }
    double dn = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) dn += Hm[a][a] * Hm[a][a];
    for (int m = 0; m <= 6; ++m) {
        double A[6][7], x[6];
        const double shift = 1e-6 * exp10((double)m) * sqrt(dn);
#pragma unroll
        for (int r = 0; r < 6; ++r) {
#pragma unroll
            for (int c = 0; c < 6; ++c) A[r][c] = Hm[r][c];
            A[r][r] -= shift;
            A[r][6] = -g[r];
        }
        if (solve6(A, x, 1e-12)) {
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
    }
    double sn = 0.0, ch = 1.0, ith = 0.0;
    if (th >= 1e-5) {
        const double h = 0.5 * th;
        if (h <= 0.25) {
            // Taylor series of sin h and cos h, truncated where the next term is
            // below 1e-19 of the sum for h <= 1/4 (coefficients 1/n!)
            const double h2 = h * h;
            sn = h * (1.0 + h2 * (-1.0 / 6 + h2 * (1.0 / 120 + h2 * (-1.0 / 5040 + h2 * (1.0 / 362880 +
                 h2 * (-1.0 / 39916800 + h2 * (1.0 / 6227020800.0)))))));
            ch = 1.0 + h2 * (-1.0 / 2 + h2 * (1.0 / 24 + h2 * (-1.0 / 720 + h2 * (1.0 / 40320 +
                 h2 * (-1.0 / 3628800 + h2 * (1.0 / 479001600.0))))));
        } else {
            sincos(h, &sn, &ch);
        }
        ith = rcp_nr(th);
        const double sh = 2.0 * sn * ith;   // sin(th/2) / (th/2)
        a = 2.0 * sn * ch * ith;
        b = 0.5 * sh * sh;
    }
    if (th < 1e-2)
        c = (1.0 / 6.0) - th2 * (1.0 / 120.0) + th2 * th2 * (1.0 / 5040.0);
    else
        c = (th - 2.0 * sn * ch) * (ith * ith * ith);
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

constexpr int kModeGN = 0, kModeExact = 1, kModeLine = 2, kModeIso = 3;

template <int Mode>
struct ModeInfo {
    static constexpr int sums = (Mode == kModeGN || Mode == kModeIso) ? kNumSums
                                : Mode == kModeExact                  ? kSumsExact
                                                                      : kSumsLine;
};

typedef const vf4 __attribute__((address_space(1))) *GRec4;

template <typename Real>
struct PairSums {
    Real F, A0, A1, A2, B00, B01, B02, B11, B12, B22;   // Gauss-Newton terms
    Real Q00, Q01, Q02, Q11, Q12, Q22;                  // exact mode: sum (f/det^2) u' u'^T
    Real L1, L2, L3, L4;                                // line mode: sum f g^k
};

// Per-point direction data of the line mode: e1 = w x y + v, e_{k+1} = w x e_k.
template <typename Real>
struct LineDir {
    Real e[4][3];
};

// One pair already known to lie within the cutoff; cw is its label weight c_ij
// (1 without labels).  Isotropic pairs (all shapes the identity, Remark 3):
// S_ij = 2I, adj = 4I, det = 8, so (f/det) C r = f r / 2 and (f/det) C = f/2 I
// with f = exp(-|r|^2 / (2 ell^2)): the same sums from a handful of operations.
template <typename Real, int Mode>
__device__ __forceinline__ void pair_heavy(PairSums<Real> &s, Real rx, Real ry, Real rz, Real s00, Real s01,
                                           Real s02, Real s11, Real s12, Real s22, Real kexp, Real k2,
                                           const LineDir<Real> &ld, Real cw) {
    if constexpr (Mode == kModeIso) {
        const Real f = cw * Fast<Real>::exp2((rx * rx + ry * ry + rz * rz) * (kexp * (Real)0.5));
        const Real hf = (Real)0.5 * f;
        s.F += f;
        s.A0 += hf * rx; s.A1 += hf * ry; s.A2 += hf * rz;
        s.B00 += hf;
        return;
    }
    {
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
        const Real f = cw * Fast<Real>::exp2(q * (inv * kexp));
        s.F += f;
        if constexpr (Mode == kModeLine) {
            // P = Sigma^{-1} = sc * C
            const Real sc = k2 * inv;
            const Real pr0 = sc * ux, pr1 = sc * uy, pr2 = sc * uz;
            const Real *e1 = ld.e[0], *e2 = ld.e[1], *e3 = ld.e[2], *e4 = ld.e[3];
            const Real p10 = sc * (c00 * e1[0] + c01 * e1[1] + c02 * e1[2]);
            const Real p11 = sc * (c01 * e1[0] + c11 * e1[1] + c12 * e1[2]);
            const Real p12 = sc * (c02 * e1[0] + c12 * e1[1] + c22 * e1[2]);
            const Real p20 = sc * (c00 * e2[0] + c01 * e2[1] + c02 * e2[2]);
            const Real p21 = sc * (c01 * e2[0] + c11 * e2[1] + c12 * e2[2]);
            const Real p22 = sc * (c02 * e2[0] + c12 * e2[1] + c22 * e2[2]);
            const Real e1Pr = e1[0] * pr0 + e1[1] * pr1 + e1[2] * pr2;
            const Real e2Pr = e2[0] * pr0 + e2[1] * pr1 + e2[2] * pr2;
            const Real e3Pr = e3[0] * pr0 + e3[1] * pr1 + e3[2] * pr2;
            const Real e4Pr = e4[0] * pr0 + e4[1] * pr1 + e4[2] * pr2;
            const Real e1Pe1 = e1[0] * p10 + e1[1] * p11 + e1[2] * p12;
            const Real e2Pe2 = e2[0] * p20 + e2[1] * p21 + e2[2] * p22;
            const Real e1Pe2 = e1[0] * p20 + e1[1] * p21 + e1[2] * p22;
            const Real e3Pe1 = e3[0] * p10 + e3[1] * p11 + e3[2] * p12;
            const Real be = -e1Pr;
            const Real ga = (Real)0.5 * (e2Pr - e1Pe1);
            const Real de = (Real)0.5 * e1Pe2 - e3Pr * (Real)(1.0 / 6.0);
            const Real ep = (Real)-0.125 * e2Pe2 - e3Pe1 * (Real)(1.0 / 6.0) + e4Pr * (Real)(1.0 / 24.0);
            const Real b2 = be * be;
            s.L1 += f * be;
            s.L2 += f * (ga + (Real)0.5 * b2);
            s.L3 += f * (de + be * ga + b2 * be * (Real)(1.0 / 6.0));
            s.L4 += f * (ep + be * de + (Real)0.5 * b2 * ga + (Real)0.5 * ga * ga + b2 * b2 * (Real)(1.0 / 24.0));
        } else {
            const Real w = f * inv;
            s.A0 += w * ux; s.A1 += w * uy; s.A2 += w * uz;
            s.B00 += w * c00; s.B01 += w * c01; s.B02 += w * c02;
            s.B11 += w * c11; s.B12 += w * c12; s.B22 += w * c22;
            if constexpr (Mode == kModeExact) {
                const Real wq = w * inv;
                const Real qx = wq * ux, qy = wq * uy, qz = wq * uz;
                s.Q00 += qx * ux; s.Q01 += qx * uy; s.Q02 += qx * uz;
                s.Q11 += qy * uy; s.Q12 += qy * uz; s.Q22 += qz * uz;
            }
        }
    }
}

// Upper-triangle index of (r, c), r <= c, in row-major order of a 6x6 matrix.
__host__ __device__ constexpr int ut(int r, int c) { return r * 6 - (r * (r - 1)) / 2 + (c - r); }

// ------------------------------------------------------------------ FP64 step

// Caller-frame g and a symmetric 6x6 term from recentred-frame sums (f at
// tot[0], g' at tot[1..6], the symmetric term's upper triangle at tot[off..]).
// With K = -c^ and A = [[I, 0], [K, I]] (the adjoint of the recentring
// translation): g = A^T g', X = A^T X' A; in 3x3 blocks X' = [[P, Q], [Q^T, S]]
//   X = [[P + QK + (QK)^T + K^T S K,  Q + (SK)^T], [Q^T + SK,  S]].
__device__ __forceinline__ void frame_sym(const double c[3], const double *upper, double sig, double X[6][6]) {
    const double K[3][3] = {{0.0, c[2], -c[1]}, {-c[2], 0.0, c[0]}, {c[1], -c[0], 0.0}};
    double Pm[3][3], Q[3][3], S[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            Pm[r][q] = upper[ut(r < q ? r : q, r < q ? q : r)];
            Q[r][q] = upper[ut(r, 3 + q)];
            S[r][q] = upper[ut(3 + (r < q ? r : q), 3 + (r < q ? q : r))];
        }
    double QK[3][3], SK[3][3], KSK[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            QK[r][q] = Q[r][0] * K[0][q] + Q[r][1] * K[1][q] + Q[r][2] * K[2][q];
            SK[r][q] = S[r][0] * K[0][q] + S[r][1] * K[1][q] + S[r][2] * K[2][q];
        }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) KSK[r][q] = K[0][r] * SK[0][q] + K[1][r] * SK[1][q] + K[2][r] * SK[2][q];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            X[r][q] = sig * (Pm[r][q] + QK[r][q] + QK[q][r] + KSK[r][q]);
            X[r][3 + q] = sig * (Q[r][q] + SK[q][r]);
            X[3 + r][q] = sig * (Q[q][r] + SK[r][q]);
            X[3 + r][3 + q] = sig * S[r][q];
        }
}

__device__ __forceinline__ void frame_grad(const double c[3], const double *tot, double sig, double g[6]) {
    const double K[3][3] = {{0.0, c[2], -c[1]}, {-c[2], 0.0, c[0]}, {c[1], -c[0], 0.0}};
    const double gw[3] = {tot[1], tot[2], tot[3]}, gv[3] = {tot[4], tot[5], tot[6]};
    // g_w = g'_w + K^T g'_v, g_v = g'_v
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        g[r] = sig * (gw[r] + K[0][r] * gv[0] + K[1][r] * gv[1] + K[2][r] * gv[2]);
        g[3 + r] = sig * gv[r];
    }
}

// Empty asm statements that hold a loaded value at a point of the program, so
// that the compiler can neither sink its load past a following branch nor
// issue it late: they put a kernel's dependent-free loads into one memory
// round trip ahead of its early-exit test.  pin_s / pin_v are volatile, and
// the compiler then gives later loads of the kernel their per-lane form (for
// kernels with none, or with per-lane loads only); tie_s instead makes `key`,
// a value the early-exit test reads, depend on x without changing either, so
// that later uniform loads stay scalar.
template <typename T>
__device__ __forceinline__ void pin_s(T x) {
    asm volatile("" ::"s"(x));
}
template <typename T>
__device__ __forceinline__ void pin_v(T x) {
    asm volatile("" ::"v"(x));
}
template <typename T>
__device__ __forceinline__ void tie_s(int &key, T x) {
    asm("" : "+s"(key) : "s"(x));
}

// What the step reads from the descriptor and the state, loaded once at the
// step kernel's start, in the same memory round trip as the reduction splits;
// after that the step reads registers only and writes the state back.
struct StepIn {
    double T[16];
    double centre[3];
    double dir[6];
    double sigma2, tol, stage_tol, min_step, gnorm;
    long long *iter_pairs;
    int iter, stage, stage_iter, damped, n_stages, max_iters, max_per_stage, eval_only;
};

__device__ __forceinline__ StepIn load_step_in(const PairDev &P) {
    const State &St = P.st;
    StepIn R;
#pragma unroll
    for (int i = 0; i < 16; ++i) R.T[i] = St.T[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) R.centre[a] = P.centre[a];
#pragma unroll
    for (int a = 0; a < 6; ++a) R.dir[a] = St.dir[a];
    R.sigma2 = P.sigma2;
    R.tol = P.tol;
    R.stage_tol = P.stage_tol;
    R.min_step = P.min_step;
    R.gnorm = St.gnorm;
    R.iter_pairs = P.iter_pairs;
    R.iter = St.iter;
    R.stage = St.stage;
    R.stage_iter = St.stage_iter;
    R.damped = St.damped;
    R.n_stages = P.n_stages;
    R.max_iters = P.max_iters;
    R.max_per_stage = P.max_per_stage;
    R.eval_only = P.eval_only;
    return R;
}

__device__ __forceinline__ void pin_step_in(const StepIn &R) {
#pragma unroll
    for (int i = 0; i < 16; ++i) pin_s(R.T[i]);
#pragma unroll
    for (int a = 0; a < 3; ++a) pin_s(R.centre[a]);
#pragma unroll
    for (int a = 0; a < 6; ++a) pin_s(R.dir[a]);
    pin_s(R.sigma2);
    pin_s(R.tol);
    pin_s(R.stage_tol);
    pin_s(R.min_step);
    pin_s(R.gnorm);
    pin_s(R.iter_pairs);
    pin_s(R.iter);
    pin_s(R.stage);
    pin_s(R.stage_iter);
    pin_s(R.damped);
    pin_s(R.n_stages);
    pin_s(R.max_iters);
    pin_s(R.max_per_stage);
    pin_s(R.eval_only);
}

// Record the evaluation (f, g, H) of the current pass; H only for evaluation
// calls, the one reader of it (a registration reports f, g and the pair count).
__device__ __forceinline__ void record_eval(const StepIn &R, State &St, double f, const double g[6],
                                            const double H[6][6], unsigned long long tot_pairs) {
    St.f = f;
#pragma unroll
    for (int a = 0; a < 6; ++a) St.g[a] = g[a];
    if (R.eval_only) {
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = 0; c < 6; ++c) St.H[6 * r + c] = H[r][c];
    }
    St.pairs_last = (long long)tot_pairs;
    if (R.iter_pairs && R.iter < R.max_iters) R.iter_pairs[R.iter] = (long long)tot_pairs;
}

// T <- T exp(xi^), then the stage and stop logic; returns the done flag.
__device__ __forceinline__ int apply_step(const StepIn &R, State &St, const double xi[6]) {
    double E[4][4];
    twist_exp(xi, E);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) acc += R.T[4 * r + b] * E[b][c];
            St.T[4 * r + c] = acc;
        }
    double l1 = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        St.xi[a] = xi[a];
        l1 += fabs(xi[a]);
    }
    St.xi_l1 = l1;
    const int stage = R.stage, iter = R.iter + 1, stage_iter = R.stage_iter + 1;
    St.iter = iter;
    St.stage_iters[stage] = stage_iter;
    const bool final_stage = (stage + 1 >= R.n_stages);
    int done = 0;
    if (final_stage) {
        if (l1 < R.tol) {
            St.converged = 1;
            done = 1;
        }
        St.stage_iter = stage_iter;
    } else if (l1 < R.stage_tol || stage_iter >= R.max_per_stage) {
        St.stage = stage + 1;
        St.stage_iter = 0;
    } else {
        St.stage_iter = stage_iter;
    }
    if (iter >= R.max_iters) done = 1;
    if (done) St.done = 1;
    return done;
}

// Symmetric part of H negative definite: Cholesky of -(H + H^T)/2 with every
// pivot above 1e-12 * max|H|.
__device__ __forceinline__ bool negative_definite(const double H[6][6]) {
    double A[6][6], amax = 0.0;
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            A[r][c] = -0.5 * (H[r][c] + H[c][r]);
            amax = fmax(amax, fabs(H[r][c]));
        }
    if (!(amax > 0.0)) return false;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double d = A[k][k];
#pragma unroll
        for (int m = 0; m < k; ++m) d -= A[k][m] * A[k][m];
        ok = ok && (d > 1e-12 * amax);
        d = sqrt(fmax(d, 1e-300));
        A[k][k] = d;
#pragma unroll
        for (int r = k + 1; r < 6; ++r) {
            double v = A[r][k];
#pragma unroll
            for (int m = 0; m < k; ++m) v -= A[r][m] * A[k][m];
            A[r][k] = v / d;
        }
    }
    return ok;
}

// Gauss-Newton (or Newton) iteration tail.  tot: the pass's sums.  With
// exact != 0, tot also holds T1 (upper triangle at kNumSums) and
// M = sum_j y_j a_j^T (row-major at kNumSums + 21), and the exact system
// matrix is H_main + T1 + T2 + C(g) with T2' = [[M - tr(M) I, (g'_v)^], [0, 0]],
// which maps to the caller's frame as [[P2 + Q2 K, Q2], [0, 0]].  Reading: the
// exact step replaces the (damped) Gauss-Newton step where the exact system's
// symmetric part is negative definite, the step is an ascent direction, and it
// is at most twice as long as the Gauss-Newton step; far from a maximum, pure
// Newton steps leave the basin.  The damped fallback always uses H_main.
__device__ __forceinline__ int finish_iteration(const StepIn &R, State &St, const double *tot,
                                                 unsigned long long tot_pairs, bool exact) {
    const double sig = R.sigma2;
    double g[6], Hm[6][6], H[6][6];
    frame_grad(R.centre, tot, sig, g);
    frame_sym(R.centre, tot + 7, sig, Hm);
    // H_GN = H_main + C(g), C(g) = [[-1/2 g_w^, 0], [-g_v^, 0]]
    {
        const double Gw[3][3] = {{0.0, -g[2], g[1]}, {g[2], 0.0, -g[0]}, {-g[1], g[0], 0.0}};
        const double Gv[3][3] = {{0.0, -g[5], g[4]}, {g[5], 0.0, -g[3]}, {-g[4], g[3], 0.0}};
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = 0; c < 6; ++c) H[r][c] = Hm[r][c];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                H[r][c] -= 0.5 * Gw[r][c];
                H[3 + r][c] -= Gv[r][c];
            }
    }
    record_eval(R, St, sig * tot[0], g, H, tot_pairs);
    if (R.eval_only) {
        St.done = 1;
        return 1;
    }
    if (tot_pairs == 0) {
        St.status = GCVO_ERR_NO_PAIRS;
        St.done = 1;
        return 1;
    }
    double xi[6];
    const int dmp = damped_step(H, Hm, g, xi);
    if (dmp < 0) {
        St.status = GCVO_ERR_SINGULAR;
        St.done = 1;
        return 1;
    }
    bool used_exact = false;
    if (exact) {
        double HE[6][6];
        {
            double T1[6][6];
            frame_sym(R.centre, tot + kNumSums, sig, T1);
            const double *M = tot + kNumSums + 21;
            const double tr = M[0] + M[4] + M[8];
            const double c0 = R.centre[0], c1 = R.centre[1], c2 = R.centre[2];
            const double K[3][3] = {{0.0, c2, -c1}, {-c2, 0.0, c0}, {c1, -c0, 0.0}};
            const double Q2[3][3] = {{0.0, -g[5], g[4]}, {g[5], 0.0, -g[3]}, {-g[4], g[3], 0.0}};   // (g_v)^
#pragma unroll
            for (int r = 0; r < 6; ++r)
#pragma unroll
                for (int c = 0; c < 6; ++c) HE[r][c] = H[r][c] + T1[r][c];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    HE[r][c] += sig * (M[3 * r + c] - (r == c ? tr : 0.0)) + Q2[r][0] * K[0][c] +
                                Q2[r][1] * K[1][c] + Q2[r][2] * K[2][c];
                    HE[r][3 + c] += Q2[r][c];
                }
        }
        if (negative_definite(HE)) {
            double Me[6][7], xn[6];
#pragma unroll
            for (int r = 0; r < 6; ++r) {
#pragma unroll
                for (int c = 0; c < 6; ++c) Me[r][c] = HE[r][c];
                Me[r][6] = -g[r];
            }
            if (solve6(Me, xn, 1e-12)) {
                double gx = 0.0, nn = 0.0, ng = 0.0;
#pragma unroll
                for (int a = 0; a < 6; ++a) {
                    gx += g[a] * xn[a];
                    nn += xn[a] * xn[a];
                    ng += xi[a] * xi[a];
                }
                if (gx > 0.0 && nn <= 4.0 * ng) {
#pragma unroll
                    for (int a = 0; a < 6; ++a) xi[a] = xn[a];
                    used_exact = true;
                }
            }
        }
    }
    if (dmp > 0 || (exact && !used_exact)) St.damped = R.damped + 1;
    return apply_step(R, St, xi);
}

// First-order solver, gradient pass done: store the unit ascent direction and
// hand over to the line pass (a zero gradient is a zero step).
__device__ __forceinline__ int finish_direction(const StepIn &R, State &St, const double *tot,
                                                 unsigned long long tot_pairs) {
    const double sig = R.sigma2;
    double g[6], Hm[6][6];
    frame_grad(R.centre, tot, sig, g);
    frame_sym(R.centre, tot + 7, sig, Hm);
    record_eval(R, St, sig * tot[0], g, Hm, tot_pairs);
    if (tot_pairs == 0) {
        St.status = GCVO_ERR_NO_PAIRS;
        St.done = 1;
        return 1;
    }
    double n2 = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) n2 += g[a] * g[a];
    const double gn = sqrt(n2);
    if (!(gn > 0.0) || !isfinite(gn)) {
        const double zero[6] = {0, 0, 0, 0, 0, 0};
        return apply_step(R, St, zero);
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) St.dir[a] = g[a] / gn;
    St.gnorm = gn;
    St.phase = 1;
    return 0;
}

// G'(s) = c1 + 2 c2 s + 3 c3 s^2 + 4 c4 s^3.
__device__ __forceinline__ double dG(const double c[5], double s) {
    return c[1] + s * (2.0 * c[2] + s * (3.0 * c[3] + s * (4.0 * c[4])));
}

// Root of G' in [a, b] with G'(a) > 0 >= G'(b): Newton steps kept inside the
// shrinking bracket, bisection when a step leaves it.
__device__ __forceinline__ double bracketed_root(const double c[5], double a, double b) {
    double x = 0.5 * (a + b);
    for (int it = 0; it < 200; ++it) {
        const double v = dG(c, x);
        if (v > 0.0) a = x;
        else b = x;
        if (!(b - a > 1e-16 * b)) break;
        const double d = 2.0 * c[2] + x * (6.0 * c[3] + x * 12.0 * c[4]);
        double xn = (d != 0.0) ? x - v / d : 0.5 * (a + b);
        if (!(xn > a && xn < b)) xn = 0.5 * (a + b);
        x = xn;
    }
    return b;
}

// Step length along the unit direction (eq. (linesearch) with the quadratic
// fallback reading): 1 = smallest positive root of G', 2 = maximiser of the
// quadratic part, 0 = none (the caller applies the minimum step).
__device__ __forceinline__ int line_step(const double c[5], double &s) {
    s = 0.0;
    if (!(c[1] > 0.0)) return 0;
    // G''(s) = 2 c2 + 6 c3 s + 12 c4 s^2: its positive roots split s > 0 into
    // intervals where G' is monotone.
    double crit[2];
    int nc = 0;
    const double qa = 12.0 * c[4], qb = 6.0 * c[3], qc = 2.0 * c[2];
    if (qa != 0.0) {
        const double disc = qb * qb - 4.0 * qa * qc;
        if (disc >= 0.0) {
            const double sq = sqrt(disc);
            // numerically stable pair of roots
            const double qq = -0.5 * (qb + (qb >= 0.0 ? sq : -sq));
            double r1 = (qq != 0.0) ? qc / qq : 0.0, r2 = qq / qa;
            if (r1 > r2) { const double t = r1; r1 = r2; r2 = t; }
            if (r1 > 0.0) crit[nc++] = r1;
            if (r2 > 0.0 && r2 != r1) crit[nc++] = r2;
        }
    } else if (qb != 0.0) {
        const double r = -qc / qb;
        if (r > 0.0) crit[nc++] = r;
    }
    double lo = 0.0;
    for (int k = 0; k < nc; ++k) {
        if (dG(c, crit[k]) <= 0.0) {
            s = bracketed_root(c, lo, crit[k]);
            return 1;
        }
        lo = crit[k];
    }
    const double lead = (c[4] != 0.0) ? c[4] : (c[3] != 0.0) ? c[3] : c[2];
    if (lead < 0.0) {
        double hi = (lo > 0.0) ? 2.0 * lo : 1e-30;
        for (int it = 0; it < 4000 && dG(c, hi) > 0.0; ++it) hi *= 2.0;
        if (dG(c, hi) <= 0.0) {
            s = bracketed_root(c, lo, hi);
            return 1;
        }
    }
    if (c[2] < 0.0) {
        s = c[1] / (-2.0 * c[2]);
        return 2;
    }
    return 0;
}

// First-order solver, line pass done: step mu * g with mu = max(min_step, s / |g|).
__device__ __forceinline__ int finish_line(const StepIn &R, State &St, const double *tot) {
    double c[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) c[k] = R.sigma2 * tot[k];
    double s;
    const int kind = line_step(c, s);
    if (kind != 1) St.damped = R.damped + 1;
    const double s_min = R.min_step * R.gnorm;
    if (!(s > s_min)) s = s_min;
    double xi[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) xi[a] = s * R.dir[a];
    St.phase = 0;
    return apply_step(R, St, xi);
}

// Lane layout of the pair kernel: a wave serves kGroupsPerWave neighbouring
// source points (sorted order), kGroupLanes lanes each.  Every point lists the
// contiguous x-rows of target cells that meet its cutoff ball; its lanes walk
// that list with stride kGroupLanes through a (row, offset) cursor, so no lane
// idles at row ends.  A group is one 16-lane DPP row, so its 16 partial sums
// are combined with DPP lane permutations inside the VALU instructions: the
// row mirrored (lane i with lane 15 - i), each half mirrored (i with 7 - i),
// then neighbours and pairs of a quad swapped.  Each step adds two equal-sized
// disjoint sets of lanes, so after four steps every lane holds the row's sum
// (bitwise the same in all 16 lanes: each addition is commutative).
template <typename Real>
__device__ __forceinline__ void group_sum(Real &v) {
    v += dpp_row<kDppRowMirror>(v);
    v += dpp_row<kDppRowHalfMirror>(v);
    v += dpp_row<kDppQuadSwap1>(v);
    v += dpp_row<kDppQuadSwap2>(v);
}

template <typename Real, int Mode, bool kLab>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_iterate(PairDev *pairs,
                                                                                          const BlockTask *tasks) {
    constexpr int NS = ModeInfo<Mode>::sums;
    // A launch over one pair passes no task table: block b serves that pair's
    // block b, and the kernel's first dependent load goes away.
    const BlockTask task = tasks ? tasks[blockIdx.x] : BlockTask{0, (int)blockIdx.x};
    PairDev &P = pairs[task.pair];
    State &St = P.st;
    // Everything that does not depend on the stage goes out in one batch ahead
    // of the done/phase test; the stage's fields and the source point follow
    // in a second: two memory round trips instead of a chain of dependent ones.
    int done = St.done;
    const int phase = St.phase, stage = St.stage;
    double Tm[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) Tm[i] = St.T[i];
    const double c0 = P.centre[0], c1 = P.centre[1], c2 = P.centre[2];
    const int ns = P.n_s;
    typedef const __attribute__((address_space(1))) float *GFloat;
    const GFloat src = (GFloat)P.s_sorted;
    void *const partials = P.partials;
    const float4 *const slab = kLab ? P.s_lab : nullptr;
    double dir[6] = {};
    if constexpr (Mode == kModeLine) {
#pragma unroll
        for (int a = 0; a < 6; ++a) dir[a] = St.dir[a];
    }
    tie_s(done, phase);
    tie_s(done, stage);
#pragma unroll
    for (int i = 0; i < 12; ++i) tie_s(done, Tm[i]);
    tie_s(done, c0);
    tie_s(done, c1);
    tie_s(done, c2);
    tie_s(done, ns);
    tie_s(done, src);
    tie_s(done, partials);
    if constexpr (kLab) tie_s(done, slab);
    if constexpr (Mode == kModeLine) {
#pragma unroll
        for (int a = 0; a < 6; ++a) tie_s(done, dir[a]);
    }
    if ((done != 0) | (phase != (Mode == kModeLine ? 1 : 0))) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = lane / kGroupLanes, q = lane % kGroupLanes;
    const double rc = P.cut[stage], kexp_d = P.kexp[stage], k2_d = P.k2[stage];
    const Grid G = P.t_grid[stage];
    typedef const __attribute__((address_space(1))) int *GInt;
    const GInt cells = (GInt)P.t_cells[stage];
    constexpr bool kExact = sizeof(Real) == 8;   // FP64: recentre the original coordinates in FP64
    // Target records through a global-address-space pointer: global (not
    // flat) loads, which do not wait on LDS traffic.
    const GRec4 trec = (GRec4)(P.t_sorted[stage]);
    typedef const vf4 __attribute__((address_space(1))) *GLab;
    const GLab tlab = kLab ? (GLab)(P.t_lab[stage]) : (GLab)nullptr;
    const double cc[3] = {c0, c1, c2};

    // Recentred pose T' = C^{-1} T C: R' = R, t' = R c + t - c.
    double Rd[9], td[3];
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) Rd[3 * r + k] = Tm[4 * r + k];
        td[r] = Tm[4 * r + 3] - cc[r];
        for (int k = 0; k < 3; ++k) td[r] += Rd[3 * r + k] * cc[k];
    }

    // The block's source points are transformed once, by wave 0 (point l on
    // lanes l, l + 16, l + 32, l + 48), and handed to their groups through LDS:
    // the other waves would repeat the same FP64 work for four points each.
    // Points past the end are read as point 0 (a launched block's pair has at
    // least one) and then given y = 0 and S' = 0; their groups walk no rows.
    __shared__ double sh_y[kPointsPerBlock][3];
    __shared__ Real sh_sp[kPointsPerBlock][6];
    if (wave == 0) {
        __builtin_amdgcn_s_setprio(2);   // the block's other waves wait for this transform
        const int pt = lane & (kPointsPerBlock - 1);
        const int jt = task.block * kPointsPerBlock + pt;
        const int jc = jt < ns ? jt : 0;
        float sv[9];   // coordinates (FP64 path: the original ones), then the 6 shape entries
#pragma unroll
        for (int a = 0; a < 3; ++a) sv[a] = src[(kExact ? 9 + a : a) * ns + jc];
#pragma unroll
        for (int a = 0; a < 6; ++a) sv[3 + a] = src[(3 + a) * ns + jc];
        // The stage's fields are read only after the barrier (the cell table
        // and records inside the row loop); tying them to the source point
        // makes all these loads complete together.
        int vkey = jt < ns;
        asm("" : "+v"(vkey)
            : "v"(sv[0]), "v"(sv[1]), "v"(sv[2]), "v"(sv[3]), "v"(sv[4]), "v"(sv[5]), "v"(sv[6]), "v"(sv[7]),
              "v"(sv[8]), "s"(cells), "s"(trec), "s"(rc), "s"(G.lo[0]), "s"(G.lo[1]), "s"(G.lo[2]), "s"(G.h),
              "s"(G.inv_h), "s"(G.n[0]), "s"(G.n[1]), "s"(G.n[2]), "s"(G.inv_hx), "s"(kexp_d), "s"(k2_d),
              "s"(tlab));
        const bool pv = vkey != 0;
        double zx, zy, zz;
        if (kExact) {
            zx = ((double)sv[0] - c0) - td[0];
            zy = ((double)sv[1] - c1) - td[1];
            zz = ((double)sv[2] - c2) - td[2];
        } else {
            zx = (double)sv[0] - td[0];
            zy = (double)sv[1] - td[1];
            zz = (double)sv[2] - td[2];
        }
        // y = R^T (z - t)
        const double ty0 = Rd[0] * zx + Rd[3] * zy + Rd[6] * zz;
        const double ty1 = Rd[1] * zx + Rd[4] * zy + Rd[7] * zz;
        const double ty2 = Rd[2] * zx + Rd[5] * zy + Rd[8] * zz;
        // S' = R^T S R
        const double S[3][3] = {{sv[3], sv[4], sv[5]}, {sv[4], sv[6], sv[7]}, {sv[5], sv[7], sv[8]}};
        double SR[3][3], Sp[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) SR[a][b] = S[a][0] * Rd[b] + S[a][1] * Rd[3 + b] + S[a][2] * Rd[6 + b];
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b) Sp[a][b] = Rd[a] * SR[0][b] + Rd[3 + a] * SR[1][b] + Rd[6 + a] * SR[2][b];
        if (lane < kPointsPerBlock) {
            sh_y[pt][0] = pv ? ty0 : 0.0;
            sh_y[pt][1] = pv ? ty1 : 0.0;
            sh_y[pt][2] = pv ? ty2 : 0.0;
            sh_sp[pt][0] = pv ? (Real)Sp[0][0] : (Real)0;
            sh_sp[pt][1] = pv ? (Real)Sp[0][1] : (Real)0;
            sh_sp[pt][2] = pv ? (Real)Sp[0][2] : (Real)0;
            sh_sp[pt][3] = pv ? (Real)Sp[1][1] : (Real)0;
            sh_sp[pt][4] = pv ? (Real)Sp[1][2] : (Real)0;
            sh_sp[pt][5] = pv ? (Real)Sp[2][2] : (Real)0;
        }
        __builtin_amdgcn_s_setprio(0);
    } else {
        // the other waves request the stage's fields before they wait
        pin_s(cells); pin_s(trec); pin_s(rc);
        pin_s(G.lo[0]); pin_s(G.lo[1]); pin_s(G.lo[2]); pin_s(G.h); pin_s(G.inv_h);
        pin_s(G.n[0]); pin_s(G.n[1]); pin_s(G.n[2]); pin_s(G.inv_hx);
        pin_s(kexp_d); pin_s(k2_d); pin_s(tlab);
    }
    const int slot = wave * kGroupsPerWave + grp;
    const int j = task.block * kPointsPerBlock + slot;
    const bool lane_valid = j < ns;
    // label vector of the source point (zero-padded to 4), requested before the barrier
    vf4 lz = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (kLab) {
        if (lane_valid) {
            const float4 l = slab[j];
            lz = vf4{l.x, l.y, l.z, l.w};
        }
    }
    __syncthreads();
    const double y0 = sh_y[slot][0], y1 = sh_y[slot][1], y2 = sh_y[slot][2];
    const Real p00 = sh_sp[slot][0], p01 = sh_sp[slot][1], p02 = sh_sp[slot][2];
    const Real p11 = sh_sp[slot][3], p12 = sh_sp[slot][4], p22 = sh_sp[slot][5];
    const Real yx = (Real)y0, yy = (Real)y1, yz = (Real)y2;
    const Real rc2 = (Real)(rc * rc);
    const Real kexp = (Real)kexp_d;   // f = exp2(q * inv_det * kexp)
    const Real k2 = (Real)k2_d;
    LineDir<Real> ld = {};
    if constexpr (Mode == kModeLine) {
        // Direction in the recentred frame: w' = w, v' = v - c x w.
        const double w[3] = {dir[0], dir[1], dir[2]};
        const double v[3] = {dir[3] - (c1 * w[2] - c2 * w[1]), dir[4] - (c2 * w[0] - c0 * w[2]),
                             dir[5] - (c0 * w[1] - c1 * w[0])};
        double e[3] = {w[1] * y2 - w[2] * y1 + v[0], w[2] * y0 - w[0] * y2 + v[1], w[0] * y1 - w[1] * y0 + v[2]};
        for (int k = 0; k < 4; ++k) {
            for (int a = 0; a < 3; ++a) ld.e[k][a] = (Real)e[a];
            const double n[3] = {w[1] * e[2] - w[2] * e[1], w[2] * e[0] - w[0] * e[2], w[0] * e[1] - w[1] * e[0]};
            e[0] = n[0]; e[1] = n[1]; e[2] = n[2];
        }
    }

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
        // cell coordinates: y, z in units of h, x in units of hx (rows run along x)
        const float gx = (fy0 - G.lo[0]) * G.inv_hx, gy = (fy1 - G.lo[1]) * G.inv_h, gz = (fy2 - G.lo[2]) * G.inv_h;
        // radius in y-z cell units, padded for the FP32 rounding of cell coordinates
        const float rh = rcm * G.inv_h + 4e-7f * fmaxf(fabsf(gx), fmaxf(fabsf(gy), fabsf(gz)));
        const float xs = G.h * G.inv_hx, padx = 4e-7f * fabsf(gx);   // y-z units -> x units, x rounding
        const int y_lo = max(0, (int)floorf(gy - rh)), y_hi = min(G.n[1] - 1, (int)floorf(gy + rh));
        const int z_lo = max(0, (int)floorf(gz - rh)), z_hi = min(G.n[2] - 1, (int)floorf(gz + rh));
        const int nyr = (lane_valid && y_lo <= y_hi && z_lo <= z_hi) ? y_hi - y_lo + 1 : 0;
        const int nrows = (nyr > 0) ? nyr * (z_hi - z_lo + 1) : 0;
        int (*rs_t)[kMaxRows] = sh_rs[wave];
        int (*rl_t)[kMaxRows] = sh_rl[wave];
        // Row t of the list is (cy, cz) = (y_lo + t mod nyr, z_lo + t div nyr).  The
        // quotient comes from an FP32 product with 1/nyr (t and nyr are small: at
        // most ~5 cells either side of the point), which is off by at most one
        // and corrected, in place of an integer division.
        const float inv_nyr = nyr > 0 ? __builtin_amdgcn_rcpf((float)nyr) : 0.0f;
        // Walks are long only where the cutoff spans many cells along a row (the
        // coarse stages); the shorter ones skip the priority below, and so does
        // the FP64 kernel, whose launches it lengthens.
        const bool long_rows = sizeof(Real) == 4 && rcm * G.inv_hx >= 4.0f;
        for (int r0 = 0; r0 < nrows; r0 += kMaxRows) {
            const int nb = min(kMaxRows, nrows - r0);
            unsigned mylen = 0;   // candidates on this lane's rows of the chunk
            for (int r = q; r < nb; r += kGroupLanes) {
                const int t = r0 + r;
                int zi = (int)((float)t * inv_nyr);
                zi -= (zi * nyr > t) ? 1 : 0;
                zi += ((zi + 1) * nyr <= t) ? 1 : 0;
                const int cy = y_lo + (t - zi * nyr), cz = z_lo + zi;
                // distance (cell units) from the point to the row's y-z square
                const float dy = fmaxf(0.0f, fmaxf((float)cy - gy, gy - (float)(cy + 1)));
                const float dz = fmaxf(0.0f, fmaxf((float)cz - gz, gz - (float)(cz + 1)));
                const float rem = rh * rh - dy * dy - dz * dz;
                int b = 0, len = 0;
                if (rem >= 0.0f) {
                    const float ext = sqrtf(rem) * xs + padx;   // half-length of the ball's section, x cells
                    const int x_lo = max(0, (int)floorf(gx - ext)), x_hi = min(G.n[0] - 1, (int)floorf(gx + ext));
                    if (x_lo <= x_hi) {
                        const int row = G.n[0] * (cy + G.n[1] * cz);
                        b = cells[row + x_lo];
                        len = cells[row + x_hi + 1] - b;
                    }
                }
                rs_t[grp][r] = b;
                rl_t[grp][r] = len;
                mylen += (unsigned)len;
            }
            __builtin_amdgcn_wave_barrier();
            if (r0 == 0 && long_rows) {
                // Issue priority from the longest walk of the wave's groups: a launch
                // ends with its longest waves, so on a shared SIMD they go first
                // (longest-first scheduling; the sums do not depend on it).  The
                // group is one DPP row, all of it active here (nrows is the
                // group's); the ballots make each test a scalar branch of the wave.
                group_sum(mylen);
                const unsigned steps = (mylen + kGroupLanes - 1) / kGroupLanes;
                if (__ballot(steps >= 40) != 0ull) __builtin_amdgcn_s_setprio(3);
                else if (__ballot(steps >= 28) != 0ull) __builtin_amdgcn_s_setprio(2);
                else if (__ballot(steps >= 16) != 0ull) __builtin_amdgcn_s_setprio(1);
            }
            int r = 0, o = q, rs = rs_t[grp][0], rl = rl_t[grp][0];
            while (r < nb && o >= rl) {
                o -= rl;
                if (++r < nb) { rs = rs_t[grp][r]; rl = rl_t[grp][r]; }
            }
            // Isotropic FP32 passes need only the recentred coordinates (first 16 bytes).
            constexpr bool kXyzOnly = (Mode == kModeIso) && !kExact;
            // Byte offset of the current record from the stage's (uniform) base:
            // loads with a scalar base and a 32-bit offset, stepped by the lane
            // stride within a row and recomputed only at row changes.
            static_assert(GCVO_MAX_POINTS * 48LL < (1LL << 32), "record offsets fit in 32 bits");
            typedef const __attribute__((address_space(1))) char *GBytes;
            unsigned off = (unsigned)(rs + o) * 48u;
            while (r < nb) {
                vf4 ra = {}, rb = {}, rcc = {}, lx = {};
                {
                    const GRec4 rec = (GRec4)((GBytes)trec + off);
                    ra = rec[0];
                    if constexpr (!kXyzOnly) { rb = rec[1]; rcc = rec[2]; }
                    if constexpr (kLab) lx = tlab[rs + o];
                }
                o += kGroupLanes;
                off += 48u * kGroupLanes;
                if (o >= rl) {
                    while (r < nb && o >= rl) {
                        o -= rl;
                        if (++r < nb) { rs = rs_t[grp][r]; rl = rl_t[grp][r]; }
                    }
                    off = (unsigned)(rs + o) * 48u;
                }
                const Real xx = kExact ? (Real)((double)rcc.y - c0) : (Real)ra.x;
                const Real xy = kExact ? (Real)((double)rcc.z - c1) : (Real)ra.y;
                const Real xz = kExact ? (Real)((double)rcc.w - c2) : (Real)ra.z;
                const Real rx = xx - yx, ry = xy - yy, rz = xz - yz;
                if (rx * rx + ry * ry + rz * rz <= rc2) {
                    Real cw = (Real)1;
                    if constexpr (kLab)
                        cw = (Real)lx.x * (Real)lz.x + (Real)lx.y * (Real)lz.y + (Real)lx.z * (Real)lz.z +
                             (Real)lx.w * (Real)lz.w;
                    pair_heavy<Real, Mode>(s, rx, ry, rz, (Real)ra.w + p00, (Real)rb.x + p01, (Real)rb.y + p02,
                                           (Real)rb.z + p11, (Real)rb.w + p12, (Real)rcc.x + p22, kexp, k2, ld, cw);
                    ++cnt;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if constexpr (sizeof(Real) == 4) __builtin_amdgcn_s_setprio(0);
    }

    // Combine the 16 lanes of each point.
    group_sum(cnt);
    group_sum(s.F);
    if constexpr (Mode == kModeLine) {
        group_sum(s.L1); group_sum(s.L2); group_sum(s.L3); group_sum(s.L4);
    } else if constexpr (Mode == kModeIso) {
        group_sum(s.A0); group_sum(s.A1); group_sum(s.A2);
        group_sum(s.B00);
    } else {
        group_sum(s.A0); group_sum(s.A1); group_sum(s.A2);
        group_sum(s.B00); group_sum(s.B01); group_sum(s.B02);
        group_sum(s.B11); group_sum(s.B12); group_sum(s.B22);
        if constexpr (Mode == kModeExact) {
            group_sum(s.Q00); group_sum(s.Q01); group_sum(s.Q02);
            group_sum(s.Q11); group_sum(s.Q12); group_sum(s.Q22);
        }
    }

    // Each group's sums go to LDS (lane 0 of the group); after the barrier wave 0
    // finishes all the block's points, one lane per point, in the recentred frame.
    constexpr int NR = (Mode == kModeLine || Mode == kModeIso) ? 5 : Mode == kModeExact ? 16 : 10;
    __shared__ Real sh_raw[kPointsPerBlock][NR];
    __shared__ Real sh_pts[kPointsPerBlock][NS];
    __shared__ unsigned sh_cnt[kPointsPerBlock];   // pairs within the cutoff, per group
    if (q == 0) {
        Real r[NR];
        r[0] = s.F;
        if constexpr (Mode == kModeLine) {
            r[1] = s.L1; r[2] = s.L2; r[3] = s.L3; r[4] = s.L4;
        } else {
            r[1] = s.A0; r[2] = s.A1; r[3] = s.A2; r[4] = s.B00;
            if constexpr (Mode != kModeIso) {
                r[5] = s.B01; r[6] = s.B02; r[7] = s.B11; r[8] = s.B12; r[9] = s.B22;
            }
            if constexpr (Mode == kModeExact) {
                r[10] = s.Q00; r[11] = s.Q01; r[12] = s.Q02; r[13] = s.Q11; r[14] = s.Q12; r[15] = s.Q22;
            }
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) sh_raw[slot][k] = r[k];
        sh_cnt[slot] = cnt;
    }
    __syncthreads();
    if (wave != 0) return;
    if (lane < kPointsPerBlock) {
        const int pt = lane;
        const bool pv = task.block * kPointsPerBlock + pt < ns;
        PairSums<Real> t = {};
        t.F = sh_raw[pt][0];
        if constexpr (Mode == kModeLine) {
            t.L1 = sh_raw[pt][1]; t.L2 = sh_raw[pt][2]; t.L3 = sh_raw[pt][3]; t.L4 = sh_raw[pt][4];
        } else {
            t.A0 = sh_raw[pt][1]; t.A1 = sh_raw[pt][2]; t.A2 = sh_raw[pt][3]; t.B00 = sh_raw[pt][4];
            if constexpr (Mode != kModeIso) {
                t.B01 = sh_raw[pt][5]; t.B02 = sh_raw[pt][6]; t.B11 = sh_raw[pt][7];
                t.B12 = sh_raw[pt][8]; t.B22 = sh_raw[pt][9];
            }
            if constexpr (Mode == kModeExact) {
                t.Q00 = sh_raw[pt][10]; t.Q01 = sh_raw[pt][11]; t.Q02 = sh_raw[pt][12];
                t.Q11 = sh_raw[pt][13]; t.Q12 = sh_raw[pt][14]; t.Q22 = sh_raw[pt][15];
            }
        }
        const Real yx = (Real)sh_y[pt][0], yy = (Real)sh_y[pt][1], yz = (Real)sh_y[pt][2];
        Real v[NS];
        if constexpr (Mode == kModeLine) {
            v[0] = pv ? t.F : (Real)0;
            v[1] = pv ? t.L1 : (Real)0;
            v[2] = pv ? t.L2 : (Real)0;
            v[3] = pv ? t.L3 : (Real)0;
            v[4] = pv ? t.L4 : (Real)0;
        } else {
            const Real kk = pv ? k2 : (Real)0;
            const Real a0 = kk * t.A0, a1 = kk * t.A1, a2 = kk * t.A2;
            const Real b00 = kk * t.B00;
            const Real b01 = (Mode == kModeIso) ? (Real)0 : kk * t.B01, b02 = (Mode == kModeIso) ? (Real)0 : kk * t.B02;
            const Real b11 = (Mode == kModeIso) ? b00 : kk * t.B11, b12 = (Mode == kModeIso) ? (Real)0 : kk * t.B12;
            const Real b22 = (Mode == kModeIso) ? b00 : kk * t.B22;
            v[0] = pv ? t.F : (Real)0;
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
            if constexpr (Mode == kModeExact) {
                // T1 = J^T Q J = [[-Y Q Y, Y Q], [-Q Y, Q]], Q = (2/ell^2)^2 * sum (f/det^2) u' u'^T
                const Real k4 = kk * kk;
                const Real Qm[3][3] = {{k4 * t.Q00, k4 * t.Q01, k4 * t.Q02},
                                       {k4 * t.Q01, k4 * t.Q11, k4 * t.Q12},
                                       {k4 * t.Q02, k4 * t.Q12, k4 * t.Q22}};
                Real N[3][3];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) N[r][c] = Y[r][0] * Qm[0][c] + Y[r][1] * Qm[1][c] + Y[r][2] * Qm[2][c];
                for (int r = 0; r < 3; ++r)
                    for (int c = r; c < 3; ++c)
                        v[kNumSums + ut(r, c)] = -(N[r][0] * Y[0][c] + N[r][1] * Y[1][c] + N[r][2] * Y[2][c]);
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) v[kNumSums + ut(r, 3 + c)] = N[r][c];
                for (int r = 0; r < 3; ++r)
                    for (int c = r; c < 3; ++c) v[kNumSums + ut(3 + r, 3 + c)] = Qm[r][c];
                // sum_j y_j a_j^T
                const Real yv[3] = {yx, yy, yz}, av[3] = {a0, a1, a2};
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) v[kNumSums + 21 + 3 * r + c] = yv[r] * av[c];
            }
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) sh_pts[pt][k] = v[k];
    }
    // LDS operations of one wave complete in order: the sums below read what
    // the point lanes wrote.
    __builtin_amdgcn_wave_barrier();
    Real *part = reinterpret_cast<Real *>(partials) + (size_t)task.block * kPartialStride;
    if (tid < NS) {
        Real acc = 0;
        for (int pnt = 0; pnt < kPointsPerBlock; ++pnt) acc += sh_pts[pnt][tid];
        part[tid] = acc;
    }
    if (tid == NS) {
        unsigned long long c = 0;
        for (int g = 0; g < kPointsPerBlock; ++g) c += sh_cnt[g];
        *reinterpret_cast<unsigned long long *>(part + NS + (NS & 1) * (sizeof(Real) == 4)) = c;
    }
}

// Cross-block reduction of one pair's block sums, split over kReduceSplit
// blocks per pair.  Block s takes the pair-kernel blocks b = s (mod
// kReduceSplit); in it, thread t adds component t % W (the NS sums and the
// pair count) over every (1024 / W)-th of those blocks with a Kahan-compensated
// sum in the pair-term precision, and the slices are added in FP64 in a fixed
// order.  The step kernel adds the kReduceSplit results, again in fixed order.
// The descriptor fields go out in one batch ahead of the done/phase test, and
// each thread requests kAhead of its block partials at a time, so a pair of
// up to kAhead * 512 pair-kernel blocks costs two memory round trips.
constexpr int kReduceThreads = 1024;

template <typename Real, int Mode>
__global__ __launch_bounds__(kReduceThreads) void k_reduce(PairDev *pairs) {
    constexpr int NS = ModeInfo<Mode>::sums;
    constexpr int W = (NS + 1 <= 32) ? 32 : 64;
    constexpr int kSlices = kReduceThreads / W;
    constexpr int kCountAt = NS + (NS & 1) * (sizeof(Real) == 4);   // 8-byte aligned slot of the pair count
    constexpr int kAhead = 4;
    // Rows are read as raw words of the pair-term width, so that the sums'
    // lanes and the count's lanes (two 4-byte words in FP32 rows, one 8-byte
    // word in FP64 rows) share one load sequence: one memory round trip per
    // kAhead rows for every wave.
    typedef typename std::conditional<sizeof(Real) == 8, unsigned long long, unsigned>::type Word;
    constexpr int kCountWords = sizeof(Real) == 4 ? 2 : 1;
    static_assert(kCountAt + kCountWords <= W, "the count's words have lanes of their own");
    PairDev &P = pairs[blockIdx.y];
    State &St = P.st;
    typedef const __attribute__((address_space(1))) Word *GWord;
    const GWord words = (GWord)P.partials;
    const int nb = P.n_blocks;
    const int done = St.done, phase = St.phase;
    pin_s(words);
    pin_s(nb);
    if ((done != 0) | (phase != (Mode == kModeLine ? 1 : 0))) return;
    const int split = blockIdx.x;
    const int tid = threadIdx.x, ck = tid % W, slice = tid / W;
    __shared__ double sh[kSlices][W + 1];
    __shared__ unsigned long long sh_c[kCountWords][kSlices];
    const int step = kSlices * kReduceSplit;
    const bool is_sum = ck < NS, is_cnt = ck >= kCountAt && ck < kCountAt + kCountWords;
    Real sm = 0, cp = 0;
    unsigned long long cacc = 0;
    if (is_sum || is_cnt) {
        for (int b0 = split + kReduceSplit * slice; b0 < nb; b0 += kAhead * step) {
            Word y[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                const int b = b0 + u * step;
                y[u] = b < nb ? words[(size_t)b * kPartialStride + ck] : (Word)0;
            }
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                if (b0 + u * step < nb) {
                    if (is_sum) {
                        const Real yy = __builtin_bit_cast(Real, y[u]) - cp;
                        const Real t = sm + yy;
                        cp = (t - sm) - yy;
                        sm = t;
                    } else {
                        cacc += y[u];
                    }
                }
            }
        }
    }
    if (is_sum) sh[slice][ck] = (double)sm - (double)cp;
    else if (is_cnt) sh_c[ck - kCountAt][slice] = cacc;
    __syncthreads();
    if (tid < NS) {
        double acc = 0.0;
        for (int sl = 0; sl < kSlices; ++sl) acc += sh[sl][tid];
        St.sub[split][tid] = acc;
    } else if (tid == NS) {
        unsigned long long c = 0;
        for (int sl = 0; sl < kSlices; ++sl) {
            c += sh_c[0][sl];
            if constexpr (kCountWords == 2) c += sh_c[1][sl] << 32;   // high words of the FP32 rows' counts
        }
        St.sub[split][NS] = (double)c;   // exact: counts stay below 2^53
    }
}

// A double held by lane k of the wave, read by every lane (k uniform).
__device__ __forceinline__ double lane_read(double v, int k) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, k);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), k);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// The FP64 step of one pair, on one lane (its registers are not shared with
// any wide kernel).  Every lane first requests its column of the reduction
// splits (the sums, then the pair count in column NS), and the step's reads of
// the descriptor and state go out with them, ahead of the done/phase test:
// one memory round trip, after which the step reads only registers.
// The splits are added in a fixed order, one column per lane.  Step kinds:
// 0 Gauss-Newton, 1 Newton, 2 first-order direction (after a gradient pass),
// 3 first-order line step.  At the last pass of a chunk of iterations the host
// passes host_done (pinned host memory, one int per pair), and every pair
// stores its done flag there for the host to poll.
template <int Kind>
__global__ __launch_bounds__(64) void k_step(PairDev *pairs, int *host_done) {
    constexpr int Mode = Kind == 1 ? kModeExact : Kind == 3 ? kModeLine : kModeGN;
    constexpr int NS = ModeInfo<Mode>::sums;
    static_assert(NS < 64 && NS < kMaxSums, "one column per lane, the pair count after the sums");
    PairDev &P = pairs[blockIdx.x];
    State &St = P.st;
    const int lane = threadIdx.x;
    const int col = lane < NS ? lane : NS;
    double v[kReduceSplit];
#pragma unroll
    for (int sp = 0; sp < kReduceSplit; ++sp) v[sp] = St.sub[sp][col];
    const StepIn R = load_step_in(P);
    const int done = St.done, phase = St.phase;
    double acc = 0.0;
#pragma unroll
    for (int sp = 0; sp < kReduceSplit; ++sp) acc += v[sp];
    pin_v(acc);
    pin_step_in(R);
    if ((done != 0) | (phase != (Mode == kModeLine ? 1 : 0))) {
        if (host_done && lane == 0) host_done[blockIdx.x] = done;
        return;
    }
    // the column sums to the first lane by lane reads (no LDS round trip)
    double tot[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) tot[k] = lane_read(acc, k);
    const unsigned long long c = (unsigned long long)lane_read(acc, NS);
    if (lane != 0) return;
    int now_done;
    if constexpr (Kind == 0 || Kind == 1) now_done = finish_iteration(R, St, tot, c, Kind == 1);
    else if constexpr (Kind == 2) now_done = finish_direction(R, St, tot, c);
    else now_done = finish_line(R, St, tot);
    if (host_done) host_done[blockIdx.x] = now_done;
}

template <typename Real, int Mode, int Kind, bool kLab>
static void launch_pass(PairDev *pairs, int n_pairs, BlockTask *tasks, int n_tasks, int *host_done, hipStream_t s,
                        hipEvent_t *&ev) {
    if (n_pairs == 1) tasks = nullptr;   // block b is block b of pair 0
    if (ev) {
        // events attached to the dispatch itself: they time the kernel, not the queue
        hipExtLaunchKernelGGL((k_iterate<Real, Mode, kLab>), dim3(n_tasks), dim3(kBlock), 0, s, ev[0], ev[1], 0u,
                              pairs, tasks);
        ev += 2;
    } else {
        hipLaunchKernelGGL((k_iterate<Real, Mode, kLab>), dim3(n_tasks), dim3(kBlock), 0, s, pairs, tasks);
    }
    hipLaunchKernelGGL((k_reduce<Real, Mode>), dim3(kReduceSplit, n_pairs), dim3(kReduceThreads), 0, s, pairs);
    hipLaunchKernelGGL((k_step<Kind>), dim3(n_pairs), dim3(64), 0, s, pairs, host_done);
}

template <typename Real, bool kLab>
static void launch_iteration(PairDev *pairs, int n_pairs, BlockTask *tasks, int n_tasks, int solver, bool iso,
                             int *host_done, hipStream_t s, hipEvent_t *&ev) {
    if (solver == GCVO_SOLVER_NEWTON) {
        launch_pass<Real, kModeExact, 1, kLab>(pairs, n_pairs, tasks, n_tasks, host_done, s, ev);
    } else if (solver == GCVO_SOLVER_FIRST_ORDER) {
        launch_pass<Real, kModeGN, 2, kLab>(pairs, n_pairs, tasks, n_tasks, nullptr, s, ev);
        launch_pass<Real, kModeLine, 3, kLab>(pairs, n_pairs, tasks, n_tasks, host_done, s, ev);
    } else if (iso) {
        launch_pass<Real, kModeIso, 0, kLab>(pairs, n_pairs, tasks, n_tasks, host_done, s, ev);
    } else {
        launch_pass<Real, kModeGN, 0, kLab>(pairs, n_pairs, tasks, n_tasks, host_done, s, ev);
    }
}

int passes_per_iteration(int solver) { return solver == GCVO_SOLVER_FIRST_ORDER ? 2 : 1; }

hipError_t launch_iterations(PairDev *pairs, int n_pairs, BlockTask *tasks, int n_tasks, int n_iters,
                             int precision, int solver, bool labels, bool iso, int *host_done, hipStream_t s,
                             hipEvent_t *events) {
    if (n_tasks <= 0) return hipSuccess;
    hipEvent_t *ev = events;
    for (int it = 0; it < n_iters; ++it) {
        int *done = (it == n_iters - 1) ? host_done : nullptr;   // the chunk's last pass reports
        if (precision == GCVO_PRECISION_FP64) {
            if (labels) launch_iteration<double, true>(pairs, n_pairs, tasks, n_tasks, solver, iso, done, s, ev);
            else launch_iteration<double, false>(pairs, n_pairs, tasks, n_tasks, solver, iso, done, s, ev);
        } else {
            if (labels) launch_iteration<float, true>(pairs, n_pairs, tasks, n_tasks, solver, iso, done, s, ev);
            else launch_iteration<float, false>(pairs, n_pairs, tasks, n_tasks, solver, iso, done, s, ev);
        }
    }
    return hipGetLastError();
}

}  // namespace gcvo
