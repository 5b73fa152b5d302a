// Once-per-registration preparation on gfx950:
//   k_stats    bounding boxes, FP64 centroid sums, finiteness (one block per cloud)
//   k_setup    grids for every binning job, recentring shift, initial state
//   k_soa      AoS float32 input -> SoA original and recentred copies
//   k_keys     linear cell key of every point of every job
//   k_sort     stable LSD radix sort of (key, index), one 1024-thread block per job,
//              plus the cell_start table
//   k_knn      n nearest neighbours (FP64 distances, ties to the smaller index),
//              covariance about the point, cyclic Jacobi, eigenvalue floor
//              (eq. (covariance), Remark 1)
//   k_gather   sorted SoA arrays (recentred xyz + shape) for the pair kernel
#include <float.h>
#include <math.h>

#include "gcvo_dev.h"

namespace gcvo {

// ------------------------------------------------------------------ k_stats

__global__ __launch_bounds__(1024) void k_stats(PairDev *pairs) {
    const int pair = blockIdx.x >> 1, cloud = blockIdx.x & 1;
    PairDev &P = pairs[pair];
    const float *xyz = cloud == 0 ? P.tgt_xyz : P.src_xyz;
    const int n = cloud == 0 ? P.n_t : P.n_s;
    const int tid = threadIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    int bad = 0;
    for (int i = tid; i < n; i += 1024) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float v = xyz[3 * (size_t)i + d];
            if (!isfinite(v)) bad = 1;
            s[d] += (double)v;
            lo[d] = fminf(lo[d], v);
            hi[d] = fmaxf(hi[d], v);
        }
    }
    __shared__ double sh_s[3][16];
    __shared__ float sh_lo[3][16], sh_hi[3][16];
    __shared__ int sh_bad[16];
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        s[d] = wave_sum(s[d]);
        lo[d] = wave_min(lo[d]);
        hi[d] = wave_max(hi[d]);
    }
    bad = __any(bad) ? 1 : 0;
    if (lane == 0) {
        for (int d = 0; d < 3; ++d) {
            sh_s[d][wave] = s[d];
            sh_lo[d][wave] = lo[d];
            sh_hi[d][wave] = hi[d];
        }
        sh_bad[wave] = bad;
    }
    __syncthreads();
    if (tid == 0) {
        double ts[3] = {0, 0, 0};
        float tl[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, th[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
        int tb = 0;
        for (int w = 0; w < 16; ++w) {
            for (int d = 0; d < 3; ++d) {
                ts[d] += sh_s[d][w];
                tl[d] = fminf(tl[d], sh_lo[d][w]);
                th[d] = fmaxf(th[d], sh_hi[d][w]);
            }
            tb |= sh_bad[w];
        }
        for (int d = 0; d < 3; ++d) {
            if (cloud == 0) {
                P.sum_t[d] = ts[d];
                P.lo_t[d] = tl[d];
                P.hi_t[d] = th[d];
            } else {
                P.lo_s[d] = tl[d];
                P.hi_s[d] = th[d];
            }
        }
        if (tb) atomicOr(&P.nonfinite, 1);
    }
}

// ------------------------------------------------------------------ k_setup

__device__ int bits_for(int v) {   // bits needed to represent v (>= 1)
    int b = 1;
    while (b < 31 && (v >> b) != 0) ++b;
    return b;
}

// Grid over [lo, hi] with cell edge at least h_min, grown until it has at most
// max_cells cells (cell counts are evaluated in FP64 so nothing overflows).  A
// box that is not finite gets a single cell (its pair is flagged invalid).
__device__ void make_grid(Grid &G, const float lo[3], const float hi[3], double h_min, int max_cells) {
    double ext[3];
    bool finite = true;
    for (int d = 0; d < 3; ++d) {
        ext[d] = fmax(0.0, (double)hi[d] - (double)lo[d]);
        finite = finite && isfinite(ext[d]) && isfinite(lo[d]);
    }
    double h = h_min;
    if (!(h > 0.0) || !isfinite(h)) h = 1.0;
    int n[3] = {1, 1, 1};
    bool ok = false;
    for (int guard = 0; finite && guard < 400; ++guard) {
        double nd[3], nc = 1.0;
        for (int d = 0; d < 3; ++d) {
            nd[d] = floor(ext[d] / h) + 1.0;
            nc *= nd[d];
        }
        if (nc <= (double)max_cells) {
            for (int d = 0; d < 3; ++d) n[d] = (int)nd[d];
            ok = true;
            break;
        }
        h *= fmax(1.25, 0.5 * cbrt(nc / (double)max_cells));
    }
    for (int d = 0; d < 3; ++d) G.lo[d] = ok ? lo[d] : 0.0f;
    if (!ok) {
        n[0] = n[1] = n[2] = 1;
        h = 1.0;
    }
    for (int d = 0; d < 3; ++d) G.n[d] = n[d];
    G.h = (float)h;
    G.inv_h = ok ? (float)(1.0 / h) : 0.0f;
    G.ncells = n[0] * n[1] * n[2];
    G.key_bits = bits_for(G.ncells > 1 ? G.ncells - 1 : 1);
}

// Cell edge for a kNN grid: about one point per cell of the bounding volume
// (flat extents are widened to 1e-3 of the largest so the volume stays positive).
__device__ double knn_cell(const float lo[3], const float hi[3], int n) {
    double ext[3], emax = 0.0;
    for (int d = 0; d < 3; ++d) {
        ext[d] = fmax(0.0, (double)hi[d] - (double)lo[d]);
        emax = fmax(emax, ext[d]);
    }
    if (!(emax > 0.0)) return 1.0;
    double vol = 1.0;
    for (int d = 0; d < 3; ++d) vol *= fmax(ext[d], 1e-3 * emax);
    return cbrt(vol / (double)(n > 0 ? n : 1));
}

__global__ void k_setup(PairDev *pairs, int n_pairs) {
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= n_pairs) return;
    PairDev &P = pairs[pair];
    for (int d = 0; d < 3; ++d) P.centre[d] = P.n_t > 0 ? P.sum_t[d] / (double)P.n_t : 0.0;
    if (P.job_knn_t) make_grid(*P.job_knn_t->grid, P.lo_t, P.hi_t, knn_cell(P.lo_t, P.hi_t, P.n_t),
                               P.job_knn_t->max_cells);
    if (P.job_knn_s) make_grid(*P.job_knn_s->grid, P.lo_s, P.hi_s, knn_cell(P.lo_s, P.hi_s, P.n_s),
                               P.job_knn_s->max_cells);
    // Stage grids over the recentred target.  float(x - c) is monotone in x,
    // so the recentred box is the rounded original box.
    float lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = (float)((double)P.lo_t[d] - P.centre[d]);
        hi[d] = (float)((double)P.hi_t[d] - P.centre[d]);
    }
    for (int s = 0; s < P.n_stages; ++s)
        make_grid(*P.t_grid[s], lo, hi, (double)kCellMargin * P.cutoff_scale * P.ell[s],
                  P.job_stage0[s].max_cells);
    State &S = *P.st;
    for (int a = 0; a < 16; ++a) S.T[a] = P.T_init[a];
    S.f = 0.0;
    for (int a = 0; a < 6; ++a) S.g[a] = S.xi[a] = 0.0;
    for (int a = 0; a < 36; ++a) S.H[a] = 0.0;
    S.xi_l1 = 0.0;
    S.pairs_last = 0;
    S.iter = S.stage = S.stage_iter = S.converged = S.damped = 0;
    for (int s = 0; s < kMaxStages; ++s) S.stage_iters[s] = 0;
    S.counter = 0;
    S.status = P.nonfinite ? GCVO_ERR_INVALID : GCVO_OK;
    S.done = P.nonfinite ? 1 : 0;
}

// ------------------------------------------------------------------ k_soa

__global__ __launch_bounds__(kBlock) void k_soa(PairDev *pairs) {
    const int pair = blockIdx.y >> 1, cloud = blockIdx.y & 1;
    const PairDev &P = pairs[pair];
    const int n = cloud == 0 ? P.n_t : P.n_s;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float *xyz = cloud == 0 ? P.tgt_xyz : P.src_xyz;
    float *orig = cloud == 0 ? P.t_orig : P.s_orig;
    float *rec = cloud == 0 ? P.t_rec : P.s_rec;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float v = xyz[3 * (size_t)i + d];
        if (orig) orig[(size_t)d * n + i] = v;
        rec[(size_t)d * n + i] = (float)((double)v - P.centre[d]);
    }
}

// ------------------------------------------------------------------ k_keys

__device__ __forceinline__ int cell_coord(float p, float lo, float inv_h, int n) {
    int c = (int)floorf((p - lo) * inv_h);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

__global__ __launch_bounds__(kBlock) void k_keys(SortJob *jobs) {
    const SortJob &J = jobs[blockIdx.y];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= J.n) return;
    const Grid G = *J.grid;
    int cx = cell_coord(J.x[i], G.lo[0], G.inv_h, G.n[0]);
    int cy = cell_coord(J.y[i], G.lo[1], G.inv_h, G.n[1]);
    int cz = cell_coord(J.z[i], G.lo[2], G.inv_h, G.n[2]);
    J.keys[i] = (uint32_t)(cx + G.n[0] * (cy + G.n[1] * cz));
    J.idx[i] = (uint32_t)i;
}

// ------------------------------------------------------------------ k_sort
//
// Stable LSD radix sort with 8-bit digits, one block per job.  Each pass:
// digit histogram in LDS, exclusive scan, then the input is streamed in
// 1024-element tiles in order; inside a tile an element's rank among equal
// digits comes from ballots within its wave (9 ballots match the 8 digit bits
// plus a valid bit) and a per-digit prefix over the 16 waves.  Ranks therefore
// follow input order, so the sort is stable and deterministic.

__global__ __launch_bounds__(kSortThreads) void k_sort(SortJob *jobs) {
    const SortJob J = jobs[blockIdx.x];
    const int n = J.n;
    const int ncells = J.grid->ncells;
    const int passes = (J.grid->key_bits + 7) / 8;
    __shared__ unsigned s_hist[256];
    __shared__ unsigned s_base[256];
    __shared__ unsigned s_tot[256];
    __shared__ unsigned s_wcnt[16][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    uint32_t *kin = J.keys, *iin = J.idx, *kout = J.keys_tmp, *iout = J.idx_tmp;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        if (tid < 256) s_hist[tid] = 0;
        for (int c = tid; c < 16 * 256; c += kSortThreads) (&s_wcnt[0][0])[c] = 0;
        __syncthreads();
        for (int i = tid; i < n; i += kSortThreads) atomicAdd(&s_hist[(kin[i] >> shift) & 255u], 1u);
        __syncthreads();
        if (wave == 0) {
            unsigned v0 = s_hist[4 * lane], v1 = s_hist[4 * lane + 1], v2 = s_hist[4 * lane + 2],
                     v3 = s_hist[4 * lane + 3];
            unsigned loc = v0 + v1 + v2 + v3, inc = loc;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                unsigned o = __shfl_up(inc, off, 64);
                if (lane >= off) inc += o;
            }
            unsigned ex = inc - loc;
            s_base[4 * lane] = ex;
            s_base[4 * lane + 1] = ex + v0;
            s_base[4 * lane + 2] = ex + v0 + v1;
            s_base[4 * lane + 3] = ex + v0 + v1 + v2;
        }
        __syncthreads();
        for (int start = 0; start < n; start += kSortThreads) {
            const int i = start + tid;
            const bool valid = i < n;
            const uint32_t key = valid ? kin[i] : 0u;
            const uint32_t id = valid ? iin[i] : 0u;
            const unsigned d = valid ? ((key >> shift) & 255u) : 256u;
            unsigned long long same = ~0ull;
#pragma unroll
            for (int b = 0; b < 9; ++b) {
                const bool bit = (d >> b) & 1u;
                const unsigned long long bb = __ballot(bit);
                same &= bit ? bb : ~bb;
            }
            const unsigned rank = (unsigned)__popcll(same & below);
            if (valid && rank == 0) s_wcnt[wave][d] = (unsigned)__popcll(same);
            __syncthreads();
            if (tid < 256) {
                unsigned run = 0;
                for (int w = 0; w < 16; ++w) {
                    unsigned v = s_wcnt[w][tid];
                    s_wcnt[w][tid] = run;
                    run += v;
                }
                s_tot[tid] = run;
            }
            __syncthreads();
            if (valid) {
                const unsigned pos = s_base[d] + s_wcnt[wave][d] + rank;
                kout[pos] = key;
                iout[pos] = id;
            }
            __syncthreads();
            if (tid < 256) {
                s_base[tid] += s_tot[tid];
                for (int w = 0; w < 16; ++w) s_wcnt[w][tid] = 0;
            }
            __syncthreads();
        }
        uint32_t *t = kin; kin = kout; kout = t;
        t = iin; iin = iout; iout = t;
        __syncthreads();
    }
    if (passes & 1) {   // result sits in the tmp buffers: move it home
        for (int i = tid; i < n; i += kSortThreads) {
            J.keys[i] = kin[i];
            J.idx[i] = iin[i];
        }
        __syncthreads();
    }
    const uint32_t *K = J.keys;
    int *cs = J.cell_start;
    for (int i = tid; i < n; i += kSortThreads) {
        const int k = (int)K[i];
        const int from = (i == 0) ? 0 : (int)K[i - 1] + 1;
        for (int c = from; c <= k; ++c) cs[c] = i;
    }
    const int tail = (n == 0) ? 0 : (int)K[n - 1] + 1;
    for (int c = tail + tid; c <= ncells; c += kSortThreads) cs[c] = n;
}

// ------------------------------------------------------------------ k_knn

__device__ __forceinline__ bool nb_less(double d, uint32_t q, double bd, uint32_t bq) {
    return d < bd || (d == bd && q < bq);
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi sweeps (FP64).  On return
// a[] holds the eigenvalues on its diagonal and v's columns the eigenvectors.
__device__ void jacobi_cyclic(double a[3][3], double v[3][3]) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) v[r][c] = (r == c) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 12; ++sweep) {
        const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off <= 1e-34 * dia || off < 1e-300) break;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int p = (k == 2) ? 1 : 0, q = (k == 0) ? 1 : 2;
            const double apq = a[p][q];
            if (apq == 0.0) continue;
            const double tau = (a[q][q] - a[p][p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            const int r = 3 - p - q;
            const double arp = a[r][p], arq = a[r][q];
            a[p][p] -= t * apq;
            a[q][q] += t * apq;
            a[p][q] = a[q][p] = 0.0;
            a[r][p] = a[p][r] = c * arp - s * arq;
            a[r][q] = a[q][r] = s * arp + c * arq;
            for (int m = 0; m < 3; ++m) {
                const double vmp = v[m][p], vmq = v[m][q];
                v[m][p] = c * vmp - s * vmq;
                v[m][q] = s * vmp + c * vmq;
            }
        }
    }
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_knn(SortJob *jobs, const PairDev *pairs) {
    const SortJob &J = jobs[blockIdx.y];
    if (!J.want_shapes || pairs[J.pair].nonfinite) return;
    const int pos = blockIdx.x * kBlock + threadIdx.x;
    const int n = J.n;
    if (pos >= n) return;
    const double rho = pairs[J.pair].rho;
    const Grid G = *J.grid;
    const uint32_t p = J.idx[pos];
    const float fx = J.x[p], fy = J.y[p], fz = J.z[p];
    const double px = fx, py = fy, pz = fz;
    const int cx = cell_coord(fx, G.lo[0], G.inv_h, G.n[0]);
    const int cy = cell_coord(fy, G.lo[1], G.inv_h, G.n[1]);
    const int cz = cell_coord(fz, G.lo[2], G.inv_h, G.n[2]);
    double bd[K];
    uint32_t bq[K];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        bd[m] = DBL_MAX;
        bq[m] = 0xffffffffu;
    }
    const int *cs = J.cell_start;
    const uint32_t *idx = J.idx;
    auto visit_range = [&](int b, int e) {
        for (int s = b; s < e; ++s) {
            const uint32_t q = idx[s];
            // Exact differences of float32 values in FP64, products and sums in
            // written order without contraction, so the ranking is reproducible.
            const double dx = (double)J.x[q] - px, dy = (double)J.y[q] - py, dz = (double)J.z[q] - pz;
            const double d = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
            if (!nb_less(d, q, bd[K - 1], bq[K - 1])) continue;
            bool placed = false;
#pragma unroll
            for (int m = K - 1; m > 0; --m) {
                if (!placed) {
                    if (nb_less(d, q, bd[m - 1], bq[m - 1])) {
                        bd[m] = bd[m - 1];
                        bq[m] = bq[m - 1];
                    } else {
                        bd[m] = d;
                        bq[m] = q;
                        placed = true;
                    }
                }
            }
            if (!placed) {
                bd[0] = d;
                bq[0] = q;
            }
        }
    };
    // Shells of cells at Chebyshev distance R around p's cell, clamped to the
    // grid.  After shell R every unvisited point lies at least R cells beyond
    // p's cell along some axis.  Points still short of K close neighbours after
    // kMaxShell shells are finished by a scan of the whole cloud.
    constexpr int kMaxShell = 24;
    const int cover = max(max(max(cx, G.n[0] - 1 - cx), max(cy, G.n[1] - 1 - cy)), max(cz, G.n[2] - 1 - cz));
    bool settled = false;
    for (int R = 0; R <= kMaxShell; ++R) {
        const int z0 = max(-R, -cz), z1 = min(R, G.n[2] - 1 - cz);
        const int y0 = max(-R, -cy), y1 = min(R, G.n[1] - 1 - cy);
        for (int dz = z0; dz <= z1; ++dz) {
            const int z = cz + dz;
            for (int dy = y0; dy <= y1; ++dy) {
                const int y = cy + dy;
                const int row = G.n[0] * (y + G.n[1] * z);
                if (dz == -R || dz == R || dy == -R || dy == R) {
                    const int x0 = max(cx - R, 0), x1 = min(cx + R, G.n[0] - 1);
                    visit_range(cs[row + x0], cs[row + x1 + 1]);
                } else {
                    if (cx - R >= 0) visit_range(cs[row + cx - R], cs[row + cx - R + 1]);
                    if (R > 0 && cx + R < G.n[0]) visit_range(cs[row + cx + R], cs[row + cx + R + 1]);
                }
            }
        }
        const double reach = (double)R * (double)G.h * (1.0 - 1e-4);
        if ((bq[K - 1] != 0xffffffffu && bd[K - 1] < reach * reach) || R >= cover) {
            settled = true;
            break;
        }
    }
    if (!settled) {
#pragma unroll
        for (int m = 0; m < K; ++m) {
            bd[m] = DBL_MAX;
            bq[m] = 0xffffffffu;
        }
        visit_range(0, n);   // sorted positions 0..n-1 cover every point once
    }
    // Covariance about p (eq. (covariance)), FP64.
    double a[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const uint32_t q = bq[m];
        if (q >= (uint32_t)n) continue;   // unfilled slot (cannot happen for n >= K)
        const double d0 = (double)J.x[q] - px, d1 = (double)J.y[q] - py, d2 = (double)J.z[q] - pz;
        a[0][0] += d0 * d0; a[0][1] += d0 * d1; a[0][2] += d0 * d2;
        a[1][1] += d1 * d1; a[1][2] += d1 * d2; a[2][2] += d2 * d2;
    }
    const double inv = 1.0 / (double)(K - 1);
    a[0][0] *= inv; a[0][1] *= inv; a[0][2] *= inv; a[1][1] *= inv; a[1][2] *= inv; a[2][2] *= inv;
    a[1][0] = a[0][1]; a[2][0] = a[0][2]; a[2][1] = a[1][2];
    double v[3][3];
    jacobi_cyclic(a, v);
    double lam[3] = {a[0][0], a[1][1], a[2][2]};
    int o0 = 0, o1 = 1, o2 = 2, t;
    if (lam[o1] > lam[o0]) { t = o0; o0 = o1; o1 = t; }
    if (lam[o2] > lam[o1]) { t = o1; o1 = o2; o2 = t; }
    if (lam[o1] > lam[o0]) { t = o0; o0 = o1; o1 = t; }
    double S[6];
    const double l1 = lam[o0];
    if (!(l1 > 1e-300)) {
        S[0] = 1.0; S[1] = 0.0; S[2] = 0.0; S[3] = 1.0; S[4] = 0.0; S[5] = 1.0;
    } else {
        // Remark 1: bound the normal/tangential ratio by flooring lambda/lambda_max at rho.
        const double w1 = fmax(lam[o1] / l1, rho), w2 = fmax(lam[o2] / l1, rho);
        const int col[3] = {o0, o1, o2};
        const double w[3] = {1.0, w1, w2};
        for (int e = 0; e < 6; ++e) S[e] = 0.0;
        for (int m = 0; m < 3; ++m) {
            const double u0 = v[0][col[m]], u1 = v[1][col[m]], u2 = v[2][col[m]];
            S[0] += w[m] * u0 * u0; S[1] += w[m] * u0 * u1; S[2] += w[m] * u0 * u2;
            S[3] += w[m] * u1 * u1; S[4] += w[m] * u1 * u2; S[5] += w[m] * u2 * u2;
        }
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) J.shape_out[(size_t)e * n + p] = (float)S[e];
}

// ------------------------------------------------------------------ k_gather

__global__ __launch_bounds__(kBlock) void k_gather(SortJob *jobs, const PairDev *pairs) {
    const SortJob &J = jobs[blockIdx.y];
    if (J.kind == kJobKnnTarget) return;
    const int pos = blockIdx.x * kBlock + threadIdx.x;
    if (pos >= J.n) return;
    const PairDev &P = pairs[J.pair];
    const uint32_t p = J.idx[pos];
    const bool src = J.kind == kJobKnnSource;
    const int n = J.n;
    const float *rec = src ? P.s_rec : P.t_rec;
    const float *org = src ? P.s_orig : P.t_orig;
    const float *shp = src ? P.s_shape : P.t_shape;
    float *out = src ? P.s_sorted : P.t_sorted[J.kind - kJobStage];
#pragma unroll
    for (int d = 0; d < 3; ++d) out[(size_t)d * n + pos] = rec[(size_t)d * n + p];
#pragma unroll
    for (int e = 0; e < 6; ++e) out[(size_t)(3 + e) * n + pos] = shp[(size_t)e * n + p];
#pragma unroll
    for (int d = 0; d < 3; ++d) out[(size_t)(9 + d) * n + pos] = org[(size_t)d * n + p];
}

// ------------------------------------------------------------------ launcher

template <int K>
static void launch_knn(dim3 grid, SortJob *jobs, const PairDev *pairs, hipStream_t s) {
    hipLaunchKernelGGL(k_knn<K>, grid, dim3(kBlock), 0, s, jobs, pairs);
}

hipError_t launch_prepare(PairDev *pairs, int n_pairs, int max_n, SortJob *jobs, int n_jobs, int max_job_n,
                          int knn, hipStream_t s) {
    hipLaunchKernelGGL(k_stats, dim3(2 * n_pairs), dim3(1024), 0, s, pairs);
    hipLaunchKernelGGL(k_setup, dim3((n_pairs + 63) / 64), dim3(64), 0, s, pairs, n_pairs);
    const int bx = (max_n + kBlock - 1) / kBlock;
    if (bx > 0) hipLaunchKernelGGL(k_soa, dim3(bx, 2 * n_pairs), dim3(kBlock), 0, s, pairs);
    const int jx = (max_job_n + kBlock - 1) / kBlock;
    if (n_jobs > 0 && jx > 0) {
        hipLaunchKernelGGL(k_keys, dim3(jx, n_jobs), dim3(kBlock), 0, s, jobs);
        hipLaunchKernelGGL(k_sort, dim3(n_jobs), dim3(kSortThreads), 0, s, jobs);
        if (knn > 0) {
            dim3 g(jx, n_jobs);
            switch (knn) {
                case 2: launch_knn<2>(g, jobs, pairs, s); break;
                case 3: launch_knn<3>(g, jobs, pairs, s); break;
                case 4: launch_knn<4>(g, jobs, pairs, s); break;
                case 5: launch_knn<5>(g, jobs, pairs, s); break;
                case 6: launch_knn<6>(g, jobs, pairs, s); break;
                case 7: launch_knn<7>(g, jobs, pairs, s); break;
                case 8: launch_knn<8>(g, jobs, pairs, s); break;
                case 9: launch_knn<9>(g, jobs, pairs, s); break;
                case 10: launch_knn<10>(g, jobs, pairs, s); break;
                case 11: launch_knn<11>(g, jobs, pairs, s); break;
                case 12: launch_knn<12>(g, jobs, pairs, s); break;
                case 13: launch_knn<13>(g, jobs, pairs, s); break;
                case 14: launch_knn<14>(g, jobs, pairs, s); break;
                case 15: launch_knn<15>(g, jobs, pairs, s); break;
                case 16: launch_knn<16>(g, jobs, pairs, s); break;
                default: return hipErrorInvalidValue;
            }
        }
        hipLaunchKernelGGL(k_gather, dim3(jx, n_jobs), dim3(kBlock), 0, s, jobs, pairs);
    }
    return hipGetLastError();
}

}  // namespace gcvo
