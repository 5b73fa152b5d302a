// Once-per-registration preparation on gfx950:
//   k_stats    bounding boxes, FP64 centroid sums, finiteness (16 blocks per cloud)
//   k_setup    their combination, grids for every binning job, recentring
//              shift, initial state
//   k_soa      AoS float32 input -> SoA original and recentred copies
//   k_keys     linear cell key of every point of every job
//   k_sort_*   stable multi-block LSD radix sort of (key, index) for all jobs,
//   k_cells    the cell_start table of each grid (and a kNN job's sorted
//              point records)
//   k_knn      n nearest neighbours (FP64 distances, ties to the smaller index)
//   k_knn_shape  covariance about the point, cyclic Jacobi, eigenvalue floor
//              (eq. (covariance), Remark 1)
//   k_gather   sorted SoA arrays (recentred xyz + shape) for the pair kernel
#include <float.h>
#include <math.h>

#include "gcvo_dev.h"

namespace gcvo {

// ------------------------------------------------------------------ k_stats
//
// Bounds of each cloud, kStatBlocks blocks per cloud: block b takes the points
// b * 256 + tid + m * 256 * kStatBlocks and stores its FP64 coordinate sums,
// minima, maxima and a non-finite flag; the setup kernel combines the blocks in
// a fixed order.

__global__ __launch_bounds__(kBlock) void k_stats(PairDev *pairs) {
    const int cloud = blockIdx.x / kStatBlocks, part = blockIdx.x % kStatBlocks;
    const PairDev &P = pairs[blockIdx.y];
    const auto xyz = gmem<const float>(cloud == 0 ? P.tgt_xyz : P.src_xyz);
    const int n = cloud == 0 ? P.n_t : P.n_s;
    const int tid = threadIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    int bad = 0;
    // Eight points' loads in flight per trip; they are added in the same order
    // as one at a time.
    constexpr int kAhead = 8, kStride = kBlock * kStatBlocks;
    for (int i0 = part * kBlock + tid; i0 < n; i0 += kStride * kAhead) {
        float v[kAhead][3];
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            const int i = i0 + kStride * u;
#pragma unroll
            for (int d = 0; d < 3; ++d) v[u][d] = (i < n) ? xyz[3 * (size_t)i + d] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kAhead; ++u) {
            if (i0 + kStride * u >= n) break;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (!isfinite(v[u][d])) bad = 1;
                s[d] += (double)v[u][d];
                lo[d] = fminf(lo[d], v[u][d]);
                hi[d] = fmaxf(hi[d], v[u][d]);
            }
        }
    }
    constexpr int kWaves = kBlock / 64;
    __shared__ double sh_s[3][kWaves];
    __shared__ float sh_lo[3][kWaves], sh_hi[3][kWaves];
    __shared__ int sh_bad[kWaves];
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
        for (int w = 0; w < kWaves; ++w) {
            for (int d = 0; d < 3; ++d) {
                ts[d] += sh_s[d][w];
                tl[d] = fminf(tl[d], sh_lo[d][w]);
                th[d] = fmaxf(th[d], sh_hi[d][w]);
            }
            tb |= sh_bad[w];
        }
        const auto out = gmem(P.stat_part) + (size_t)blockIdx.x * kStatVals;
        for (int d = 0; d < 3; ++d) {
            out[d] = ts[d];
            out[3 + d] = tl[d];
            out[6 + d] = th[d];
        }
        out[9] = tb;
    }
}

// ------------------------------------------------------------------ k_setup

__device__ int bits_for(int v) {   // bits needed to represent v (>= 1)
    int b = 1;
    while (b < 31 && (v >> b) != 0) ++b;
    return b;
}

// Grid over [lo, hi] with cells of edge h >= h_min (x edge x_ratio * h), grown
// until it has at most max_cells cells (cell counts are evaluated in FP64 so
// nothing overflows).  A box that is not finite gets a single cell (its pair
// is flagged invalid).
__device__ void make_grid(Grid &G, const float lo[3], const float hi[3], double h_min, int max_cells,
                          double x_ratio = 1.0) {
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
            nd[d] = floor(ext[d] / (d == 0 ? x_ratio * h : h)) + 1.0;
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
    G.hx = ok ? (float)(x_ratio * h) : (float)h;
    G.inv_hx = ok ? (float)(1.0 / (x_ratio * h)) : 0.0f;
    G.ncells = n[0] * n[1] * n[2];
    G.key_bits = bits_for(G.ncells > 1 ? G.ncells - 1 : 1);
}

// Cell edge for a kNN grid: half the edge that would hold one point per cell of
// the bounding volume (points lie on surfaces, so most of that volume is empty;
// flat extents are widened to 1e-3 of the largest so the volume stays positive).
__device__ double knn_cell(const float lo[3], const float hi[3], int n) {
    double ext[3], emax = 0.0;
    for (int d = 0; d < 3; ++d) {
        ext[d] = fmax(0.0, (double)hi[d] - (double)lo[d]);
        emax = fmax(emax, ext[d]);
    }
    if (!(emax > 0.0)) return 1.0;
    double vol = 1.0;
    for (int d = 0; d < 3; ++d) vol *= fmax(ext[d], 1e-3 * emax);
    return 0.5 * cbrt(vol / (double)(n > 0 ? n : 1));
}

// A start pose given in device memory must be a rigid motion: finite, last
// row (0, 0, 0, 1), R^T R = I and det R = 1, each within 1e-6.
__device__ bool in_se3(const double T[16]) {
    for (int a = 0; a < 16; ++a)
        if (!isfinite(T[a])) return false;
    if (fabs(T[12]) > 1e-6 || fabs(T[13]) > 1e-6 || fabs(T[14]) > 1e-6 || fabs(T[15] - 1.0) > 1e-6) return false;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += T[4 * k + a] * T[4 * k + b];
            if (fabs(s - (a == b ? 1.0 : 0.0)) > 1e-6) return false;
        }
    const double det = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
                       T[2] * (T[4] * T[9] - T[5] * T[8]);
    return fabs(det - 1.0) <= 1e-6;
}

// One 32-thread block per pair, the grids built side by side (each is a short
// serial FP64 loop): thread 0 the centroid and the solver state, 1 and 2 the
// kNN grids, 3 the source's Morton grid, 4 + s the pair grid of stage s.
__global__ __launch_bounds__(32) void k_setup(PairDev *pairs) {
    PairDev &P = pairs[blockIdx.x];
    const int t = threadIdx.x;
    // The bounds kernel's partials: lane l < kStatBlocks holds the target's block
    // l, lane kStatBlocks + l the source's.  A butterfly over each half adds
    // every pair of values in both orders, so all its lanes hold bitwise the
    // same totals.
    static_assert(2 * kStatBlocks == 32, "one setup lane per bounds block");
    double v[kStatVals];
    for (int k = 0; k < kStatVals; ++k) v[k] = P.stat_part[t * kStatVals + k];
    for (int off = kStatBlocks / 2; off > 0; off >>= 1) {
        for (int k = 0; k < kStatVals; ++k) {
            const double o = __shfl_xor(v[k], off, kStatBlocks);
            v[k] = k < 3 ? v[k] + o : (k < 6 ? fmin(v[k], o) : fmax(v[k], o));
        }
    }
    double c[3];
    float lo_t[3], hi_t[3], lo_s[3], hi_s[3];
    for (int d = 0; d < 3; ++d) {
        const double sum_t = __shfl(v[d], 0);
        c[d] = P.n_t > 0 ? sum_t / (double)P.n_t : 0.0;
        lo_t[d] = (float)__shfl(v[3 + d], 0);
        hi_t[d] = (float)__shfl(v[6 + d], 0);
        lo_s[d] = (float)__shfl(v[3 + d], kStatBlocks);
        hi_s[d] = (float)__shfl(v[6 + d], kStatBlocks);
    }
    const bool nonfinite = __shfl(v[9], 0) != 0.0 || __shfl(v[9], kStatBlocks) != 0.0;
    if (t == 0) {
        for (int d = 0; d < 3; ++d) P.centre[d] = c[d];
        State &S = P.st;
        bool pose_ok = true;
        if (P.T_init_dev) {
            for (int a = 0; a < 16; ++a) S.T[a] = P.T_init_dev[a];
            pose_ok = in_se3(S.T);
        } else {
            for (int a = 0; a < 16; ++a) S.T[a] = P.T_init[a];
        }
        S.f = 0.0;
        for (int a = 0; a < 6; ++a) S.g[a] = S.xi[a] = 0.0;
        for (int a = 0; a < 36; ++a) S.H[a] = 0.0;
        S.xi_l1 = 0.0;
        S.pairs_last = 0;
        S.iter = S.stage = S.stage_iter = S.converged = S.damped = 0;
        S.phase = 0;
        S.gnorm = 0.0;
        for (int a = 0; a < 6; ++a) S.dir[a] = 0.0;
        for (int s = 0; s < kMaxStages; ++s) S.stage_iters[s] = 0;
        if (nonfinite) P.nonfinite = 1;
        const bool bad = nonfinite || !pose_ok;
        S.status = bad ? GCVO_ERR_INVALID : GCVO_OK;
        S.done = bad ? 1 : 0;
    } else if (t == 1) {
        if (P.job_knn_t)
            make_grid(*P.job_knn_t->grid, lo_t, hi_t, knn_cell(lo_t, hi_t, P.n_t), P.job_knn_t->max_cells);
    } else if (t == 2) {
        if (P.job_knn_s)
            make_grid(*P.job_knn_s->grid, lo_s, hi_s, knn_cell(lo_s, hi_s, P.n_s), P.job_knn_s->max_cells);
    } else if (t == 3) {
        if (P.job_order_s) {   // 256 cells along the longest axis; keys are Morton codes
            Grid &M = *P.job_order_s->grid;
            double emax = 0.0;
            for (int d = 0; d < 3; ++d) emax = fmax(emax, (double)hi_s[d] - (double)lo_s[d]);
            const double h = (isfinite(emax) && emax > 0.0) ? emax / 255.5 : 1.0;
            for (int d = 0; d < 3; ++d) {
                M.lo[d] = isfinite(lo_s[d]) ? lo_s[d] : 0.0f;
                M.n[d] = 256;
            }
            M.h = M.hx = (float)h;
            M.inv_h = M.inv_hx = (float)(1.0 / h);
            M.ncells = 0;
            M.key_bits = 24;
        }
    } else if (t - 4 < P.n_stages) {
        // Stage grids over the recentred target.  float(x - c) is monotone in
        // x, so the recentred box is the rounded original box.
        const int s = t - 4;
        float lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = (float)((double)lo_t[d] - c[d]);
            hi[d] = (float)((double)hi_t[d] - c[d]);
        }
        make_grid(P.t_grid[s], lo, hi, P.cell_fraction * P.cutoff_scale * P.ell[s], P.job_stage0[s].max_cells,
                  P.cell_fraction_x / P.cell_fraction);
    }
}

// ------------------------------------------------------------------ k_soa

__global__ __launch_bounds__(kBlock) void k_soa(PairDev *pairs) {
    const int pair = blockIdx.y >> 1, cloud = blockIdx.y & 1;
    const PairDev &P = pairs[pair];
    const int n = cloud == 0 ? P.n_t : P.n_s;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const auto xyz = gmem<const float>(cloud == 0 ? P.tgt_xyz : P.src_xyz);
    float *orig = cloud == 0 ? P.t_orig : P.s_orig;
    const auto rec = gmem(cloud == 0 ? P.t_rec : P.s_rec);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        float v = xyz[3 * (size_t)i + d];
        if (orig) gmem(orig)[(size_t)d * n + i] = v;
        rec[(size_t)d * n + i] = (float)((double)v - P.centre[d]);
    }
}

// ------------------------------------------------------------------ k_keys

__device__ __forceinline__ int cell_coord(float p, float lo, float inv_h, int n) {
    int c = (int)floorf((p - lo) * inv_h);
    return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

// The keys go to keys_tmp when the sort runs an odd number of passes, so that
// its last pass leaves them in keys.
__global__ __launch_bounds__(kBlock) void k_keys(SortJob *jobs, int to_tmp) {
    const SortJob &J = jobs[blockIdx.y];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= J.n) return;
    const Grid G = *J.grid;
    int cx = cell_coord(gmem<const float>(J.x)[i], G.lo[0], G.inv_hx, G.n[0]);
    int cy = cell_coord(gmem<const float>(J.y)[i], G.lo[1], G.inv_h, G.n[1]);
    int cz = cell_coord(gmem<const float>(J.z)[i], G.lo[2], G.inv_h, G.n[2]);
    if (J.morton) {
        uint32_t key = 0;
        for (int b = 7; b >= 0; --b)
            key = (key << 3) | ((((uint32_t)cz >> b) & 1u) << 2) | ((((uint32_t)cy >> b) & 1u) << 1) |
                  (((uint32_t)cx >> b) & 1u);
        gmem(to_tmp ? J.keys_tmp : J.keys)[i] = key;
    } else {
        gmem(to_tmp ? J.keys_tmp : J.keys)[i] = (uint32_t)(cx + G.n[0] * (cy + G.n[1] * cz));
    }
    gmem(to_tmp ? J.idx_tmp : J.idx)[i] = (uint32_t)i;
}

// ------------------------------------------------------------------ radix sort
//
// Stable LSD radix sort of (key, index) with 8-bit digits, all jobs at once.
// Each pass is three launches over tiles of kSortTile elements:
//   k_sort_up    per-tile digit histograms,
//   k_sort_scan  per job: exclusive offsets in digit-major, tile-minor order,
//   k_sort_down  per tile: stable scatter.  A tile is taken in 4 rounds of 256
//                elements in input order; an element's rank among equal digits
//                comes from 9 ballots inside its wave plus per-digit prefixes
//                over the earlier waves and rounds, so ranks follow input order.
// Jobs whose keys need fewer passes run the extra passes as stable no-ops.

constexpr int kSortTile = 1024;

__global__ __launch_bounds__(256) void k_sort_up(SortJob *jobs, int shift, int in_tmp) {
    const SortJob &J = jobs[blockIdx.y];
    const int ntile = (J.n + kSortTile - 1) / kSortTile;
    const int tile = blockIdx.x;
    if (tile >= ntile) return;
    const auto kin = gmem<const uint32_t>(in_tmp ? J.keys_tmp : J.keys);
    __shared__ unsigned hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int base = tile * kSortTile;
    for (int e = threadIdx.x; e < kSortTile; e += 256) {
        const int i = base + e;
        if (i < J.n) atomicAdd(&hist[(kin[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    gmem(J.tile_counts)[(size_t)tile * 256 + threadIdx.x] = hist[threadIdx.x];
}

__global__ __launch_bounds__(256) void k_sort_scan(SortJob *jobs) {
    constexpr int kChunk = 16;   // tile counts in flight per thread
    constexpr int kHeld = 64;    // jobs of up to kHeld tiles keep their row in registers
    const SortJob &J = jobs[blockIdx.x];
    const int ntile = (J.n + kSortTile - 1) / kSortTile;
    const int d = threadIdx.x, lane = d & 63, wave = d >> 6;
    // digit d of tile t at tc[t * 256 + d]: a wave's 64 digits of one tile are
    // one contiguous 256-byte access
    const auto tc = gmem(J.tile_counts) + d;
    const bool held = ntile <= kHeld;
    // total of digit d over the tiles: a held row in one round trip, a longer
    // one kChunk independent loads at a time
    unsigned run = 0;
    unsigned h[kHeld];
    if (held) {
#pragma unroll
        for (int u = 0; u < kHeld; ++u) h[u] = (u < ntile) ? tc[(size_t)u * 256] : 0u;
#pragma unroll
        for (int u = 0; u < kHeld; ++u) run += h[u];
    } else {
        for (int t0 = 0; t0 < ntile; t0 += kChunk) {
            unsigned v[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) v[u] = (t0 + u < ntile) ? tc[(size_t)(t0 + u) * 256] : 0u;
#pragma unroll
            for (int u = 0; u < kChunk; ++u) run += v[u];
        }
    }
    // exclusive scan of the 256 digit totals
    unsigned inc = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    __shared__ unsigned wsum[4];
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    unsigned before = 0;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    // tile t of digit d starts at the digit's base plus the counts of tiles < t
    unsigned acc = before + inc - run;
    if (held) {
#pragma unroll
        for (int u = 0; u < kHeld; ++u) {
            if (u < ntile) tc[(size_t)u * 256] = acc;
            acc += h[u];
        }
        return;
    }
    for (int t0 = 0; t0 < ntile; t0 += kChunk) {
        unsigned v[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) v[u] = (t0 + u < ntile) ? tc[(size_t)(t0 + u) * 256] : 0u;
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
            if (t0 + u < ntile) tc[(size_t)(t0 + u) * 256] = acc;
            acc += v[u];
        }
    }
}

__global__ __launch_bounds__(256) void k_sort_down(SortJob *jobs, int shift, int in_tmp) {
    const SortJob &J = jobs[blockIdx.y];
    const int ntile = (J.n + kSortTile - 1) / kSortTile;
    const int tile = blockIdx.x;
    if (tile >= ntile) return;
    const auto kin = gmem<const uint32_t>(in_tmp ? J.keys_tmp : J.keys);
    const auto iin = gmem<const uint32_t>(in_tmp ? J.idx_tmp : J.idx);
    const auto kout = gmem(in_tmp ? J.keys : J.keys_tmp);
    const auto iout = gmem(in_tmp ? J.idx : J.idx_tmp);
    __shared__ unsigned base_d[256];    // next free slot of each digit for this tile
    __shared__ unsigned wcnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    constexpr int kRounds = kSortTile / 256;
    // the tile's keys and indices are requested at once, with its offsets
    uint32_t keys[kRounds], ids[kRounds];
#pragma unroll
    for (int round = 0; round < kRounds; ++round) {
        const int i = tile * kSortTile + round * 256 + tid;
        keys[round] = i < J.n ? kin[i] : 0u;
        ids[round] = i < J.n ? iin[i] : 0u;
    }
    base_d[tid] = gmem(J.tile_counts)[(size_t)tile * 256 + tid];
    for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
    __syncthreads();
#pragma unroll
    for (int round = 0; round < kRounds; ++round) {
        const int i = tile * kSortTile + round * 256 + tid;
        const bool valid = i < J.n;
        const uint32_t key = keys[round];
        const uint32_t id = ids[round];
        const unsigned d = valid ? ((key >> shift) & 255u) : 256u;
        unsigned long long same = ~0ull;
#pragma unroll
        for (int b = 0; b < 9; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long bb = __ballot(bit);
            same &= bit ? bb : ~bb;
        }
        const unsigned rank = (unsigned)__popcll(same & below);
        if (valid && rank == 0) wcnt[wave][d] = (unsigned)__popcll(same);
        __syncthreads();
        {   // per digit: prefix over the 4 waves
            unsigned run = 0;
            for (int w = 0; w < 4; ++w) {
                const unsigned v = wcnt[w][tid];
                wcnt[w][tid] = run;
                run += v;
            }
            __syncthreads();
            if (valid) {
                const unsigned posn = base_d[d] + wcnt[wave][d] + rank;
                kout[posn] = key;
                iout[posn] = id;
            }
            __syncthreads();
            base_d[tid] += run;
            for (int w = 0; w < 4; ++w) wcnt[w][tid] = 0;
            __syncthreads();
        }
    }
}

// cell_start[c] = first sorted position whose key is >= c, for c = 0..ncells.
// Sorted position i (0 <= i <= n) is that position for the cells after the
// previous key up to its own key (position 0 from cell 0, position n, one past
// the end, up to cell ncells), so every cell is written once.  A lane writes a
// run of up to kShortRun cells itself; a wave writes its lanes' longer runs one
// after another, its 64 lanes storing consecutive cells; runs longer than
// kLongRun cells (empty stretches of the grid, up to ~50k cells in a LiDAR
// scene) are listed in LDS and written by the whole block.
// A kNN job also gets its sorted point records {x, y, z, index bits} here, so
// that a candidate of the kNN search is one 16-byte load instead of an index
// load followed by three coordinate loads.
__global__ __launch_bounds__(kBlock) void k_cells(SortJob *jobs) {
    const SortJob &J = jobs[blockIdx.y];
    if (J.morton || !J.cell_start) return;
    const int n = J.n, ncells = J.grid->ncells;
    if (blockIdx.x * kBlock > n) return;   // the whole block is past the end
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const auto keys = gmem<const uint32_t>(J.keys);
    const auto cs = gmem(J.cell_start);
    int first = 0, len = 0;     // cells [first, first + len) take position i
    if (i <= n) {
        const int prev = i > 0 ? (int)keys[i - 1] : -1;
        const int cur = i < n ? (int)keys[i] : ncells;
        first = prev + 1;
        len = cur - prev;
    }
    if (J.want_shapes && i < n) {
        const uint32_t c = gmem(J.idx)[i];
        gmem(reinterpret_cast<vf4 *>(J.pts))[i] =
            vf4{gmem<const float>(J.x)[c], gmem<const float>(J.y)[c], gmem<const float>(J.z)[c], __uint_as_float(c)};
    }
    constexpr int kShortRun = 8, kLongRun = 4 * 64;
    __shared__ int long_first[kBlock], long_len[kBlock], long_pos[kBlock];
    __shared__ int n_long;
    if (threadIdx.x == 0) n_long = 0;
    __syncthreads();
    const bool is_long = len > kLongRun;
    if (is_long) {   // list order is arbitrary: the runs are disjoint
        const int at = atomicAdd(&n_long, 1);
        long_first[at] = first;
        long_len[at] = len;
        long_pos[at] = i;
    }
    if (len <= kShortRun) {
#pragma unroll
        for (int c = 0; c < kShortRun; ++c)
            if (c < len) cs[first + c] = i;
    }
    unsigned long long m = __ballot(len > kShortRun && !is_long);
    while (m) {   // l is the same in every lane: its values come by lane reads
        const int l = __builtin_ctzll(m);
        m &= m - 1;
        const int f = __builtin_amdgcn_readlane(first, l), cnt = __builtin_amdgcn_readlane(len, l);
        const int pos = i - lane + l;
        for (int c = lane; c < cnt; c += 64) cs[f + c] = pos;
    }
    __syncthreads();
    const int nl = n_long;
    for (int r = 0; r < nl; ++r) {
        const int f = long_first[r], cnt = long_len[r], pos = long_pos[r];
        for (int c = threadIdx.x; c < cnt; c += 4 * kBlock) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (c + u * kBlock < cnt) cs[f + c + u * kBlock] = pos;
        }
    }
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

constexpr int kKnnMaxAttempts = 40;   // radius attempts 1.5 h 2^a, a < 40

// Lexicographic (distance, index) minimum of a lane's candidate and another's.
__device__ __forceinline__ void take_min(double &d, uint32_t &c, double od, uint32_t oc) {
    if (nb_less(od, oc, d, c)) {
        d = od;
        c = oc;
    }
}

// The K nearest neighbours of (fx, fy, fz) with kGroupLanes lanes per point
// (lane q of group grp of the wave): the group lists the x-rows of grid cells
// meeting a ball of radius r around the point, every lane keeps the K best
// candidates it sees within r (FP64 squared distances, ties to the smaller
// index), and the 16 lists are merged by K rounds of a group minimum.  If fewer
// than K points lie within r, r doubles (exactly) and the point is scanned
// again; the K-th merged distance never exceeds r, so no closer point was
// skipped.  Returns whether the K nearest were found; md/mq then hold them in
// order on every lane of the group.  All lanes of the wave take part (the loop
// ends when every group is done).
template <int K>
__device__ __forceinline__ bool knn_search(const SortJob &J, const Grid &G, int wave, int grp, int q, bool active,
                                           float fx, float fy, float fz, double md[K], uint32_t mq[K]) {
    constexpr int L = kGroupLanes;
    __shared__ int sh_rs[kBlock / 64][kGroupsPerWave][kMaxRows], sh_rl[kBlock / 64][kGroupsPerWave][kMaxRows];
    int *rs_t = sh_rs[wave][grp];
    int *rl_t = sh_rl[wave][grp];
    const double px = fx, py = fy, pz = fz;
    // kNN grids are isotropic (inv_hx == inv_h)
    const float gx = (fx - G.lo[0]) * G.inv_h, gy = (fy - G.lo[1]) * G.inv_h, gz = (fz - G.lo[2]) * G.inv_h;
    const auto cs = gmem<const int>(J.cell_start);
    const auto pts = gmem(reinterpret_cast<const vf4 *>(J.pts));
    bool done = !active;
    double rad = 1.5 * (double)G.h;
    for (int attempt = 0; attempt < kKnnMaxAttempts; ++attempt) {
        double bd[K];
        uint32_t bq[K];
#pragma unroll
        for (int m = 0; m < K; ++m) {
            bd[m] = DBL_MAX;
            bq[m] = 0xffffffffu;
        }
        if (!done) {
            const double r2 = rad * rad;
            const float rh = (float)(rad * (double)kCellMargin) * G.inv_h +
                             4e-7f * fmaxf(fabsf(gx), fmaxf(fabsf(gy), fabsf(gz)));
            const int y_lo = max(0, (int)floorf(gy - rh)), y_hi = min(G.n[1] - 1, (int)floorf(gy + rh));
            const int z_lo = max(0, (int)floorf(gz - rh)), z_hi = min(G.n[2] - 1, (int)floorf(gz + rh));
            const int nyr = (y_lo <= y_hi && z_lo <= z_hi) ? y_hi - y_lo + 1 : 0;
            const int nrows = (nyr > 0) ? nyr * (z_hi - z_lo + 1) : 0;
            for (int r0 = 0; r0 < nrows; r0 += kMaxRows) {
                const int nb = min(kMaxRows, nrows - r0);
                // The table keeps the non-empty rows only, in row order (their
                // position from a ballot of the group's lanes): the cursor below
                // then never steps through empty rows one LDS read at a time, and
                // every lane still sees the same candidates in the same order.
                int cnt = 0;
                for (int r1 = 0; r1 < nb; r1 += L) {
                    const int r = r1 + q;
                    int b = 0, len = 0;
                    if (r < nb) {
                        const int cy = y_lo + (r0 + r) % nyr, cz = z_lo + (r0 + r) / nyr;
                        const float dy = fmaxf(0.0f, fmaxf((float)cy - gy, gy - (float)(cy + 1)));
                        const float dz = fmaxf(0.0f, fmaxf((float)cz - gz, gz - (float)(cz + 1)));
                        const float rem = rh * rh - dy * dy - dz * dz;
                        if (rem >= 0.0f) {
                            const float ext = sqrtf(rem);
                            const int x_lo = max(0, (int)floorf(gx - ext)), x_hi = min(G.n[0] - 1, (int)floorf(gx + ext));
                            if (x_lo <= x_hi) {
                                const int row = G.n[0] * (cy + G.n[1] * cz);
                                b = cs[row + x_lo];
                                len = cs[row + x_hi + 1] - b;
                            }
                        }
                    }
                    const unsigned long long m = (__ballot(len > 0) >> (grp * L)) & ((1ull << L) - 1);
                    if (len > 0) {
                        const int at = cnt + __popcll(m & ((1ull << q) - 1));
                        rs_t[at] = b;
                        rl_t[at] = len;
                    }
                    cnt += __popcll(m);
                }
                __builtin_amdgcn_wave_barrier();   // LDS operations of one wave complete in order
                int r = 0, o = q, rs = rs_t[0], rl = rl_t[0];
                while (r < cnt && o >= rl) {
                    o -= rl;
                    if (++r < cnt) { rs = rs_t[r]; rl = rl_t[r]; }
                }
                while (r < cnt) {
                    const vf4 pc = pts[rs + o];
                    const uint32_t c = __float_as_uint(pc.w);
                    // Exact differences of float32 values in FP64, products and sums
                    // in written order without contraction: reproducible ranking.
                    const double dx = (double)pc.x - px, dyy = (double)pc.y - py, dzz = (double)pc.z - pz;
                    const double d = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dyy, dyy)), __dmul_rn(dzz, dzz));
                    if (d <= r2 && nb_less(d, c, bd[K - 1], bq[K - 1])) {
                        bool placed = false;
#pragma unroll
                        for (int m = K - 1; m > 0; --m) {
                            if (!placed) {
                                if (nb_less(d, c, bd[m - 1], bq[m - 1])) {
                                    bd[m] = bd[m - 1];
                                    bq[m] = bq[m - 1];
                                } else {
                                    bd[m] = d;
                                    bq[m] = c;
                                    placed = true;
                                }
                            }
                        }
                        if (!placed) {
                            bd[0] = d;
                            bq[0] = c;
                        }
                    }
                    o += L;
                    while (r < cnt && o >= rl) {
                        o -= rl;
                        if (++r < cnt) { rs = rs_t[r]; rl = rl_t[r]; }
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        // Merge: K rounds of a lexicographic group minimum over the lists' heads,
        // by DPP row permutations (a minimum is exact, so every lane of the
        // group ends with the same head).
#pragma unroll
        for (int m = 0; m < K; ++m) {
            double d = bd[0];
            uint32_t c = bq[0];
            take_min(d, c, dpp_row<kDppRowMirror>(d), dpp_row<kDppRowMirror>((unsigned)c));
            take_min(d, c, dpp_row<kDppRowHalfMirror>(d), dpp_row<kDppRowHalfMirror>((unsigned)c));
            take_min(d, c, dpp_row<kDppQuadSwap1>(d), dpp_row<kDppQuadSwap1>((unsigned)c));
            take_min(d, c, dpp_row<kDppQuadSwap2>(d), dpp_row<kDppQuadSwap2>((unsigned)c));
            if (!done) {
                md[m] = d;
                mq[m] = c;
            }
            if (bq[0] == c && bd[0] == d) {   // this lane supplied the minimum: pop it
#pragma unroll
                for (int k = 0; k < K - 1; ++k) {
                    bd[k] = bd[k + 1];
                    bq[k] = bq[k + 1];
                }
                bd[K - 1] = DBL_MAX;
                bq[K - 1] = 0xffffffffu;
            }
        }
        if (!done) {
            if (mq[K - 1] != 0xffffffffu) done = true;   // K points within rad: the K nearest
            else rad *= 2.0;
        }
        if (__all(done)) break;
    }
    return active && done;
}

// Shape of point p from its K nearest neighbours (one lane): covariance about p
// (eq. (covariance)) in FP64, cyclic Jacobi, and Remark 1's floor of the
// eigenvalue ratios at rho.
template <int K>
__device__ __forceinline__ void knn_shape(const SortJob &J, double rho, uint32_t p, double px, double py, double pz,
                                          const uint32_t mq[K]) {
    double a[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    const auto X = gmem<const float>(J.x), Y = gmem<const float>(J.y), Z = gmem<const float>(J.z);
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const uint32_t c = mq[m];
        const double d0 = (double)X[c] - px, d1 = (double)Y[c] - py, d2 = (double)Z[c] - pz;
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
    const int n = J.n;
    const auto out = gmem(J.shape_out);
#pragma unroll
    for (int e = 0; e < 6; ++e) out[(size_t)e * n + p] = (float)S[e];
}

// K nearest neighbours of a job's points, kGroupLanes lanes per point; the
// group's first lane stores them for the shape kernel.
// Register budget of five waves per SIMD (96 VGPRs, no spills; 112 VGPRs and
// four waves otherwise): 11 % shorter on a LiDAR cloud pair; six waves spill.
template <int K>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_knn(SortJob *jobs,
                                                                                     const PairDev *pairs) {
    const SortJob &J = jobs[blockIdx.y];
    if (!J.want_shapes || pairs[J.pair].nonfinite) return;
    const int n = J.n;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / kGroupLanes, q = lane % kGroupLanes;
    const int pos = (blockIdx.x * (kBlock / 64) + wave) * kGroupsPerWave + grp;
    if ((blockIdx.x * (kBlock / 64) + wave) * kGroupsPerWave >= n) return;   // whole wave idle
    const bool valid = pos < n;
    const Grid G = *J.grid;
    const uint32_t p = valid ? gmem(J.idx)[pos] : 0u;
    const float fx = gmem<const float>(J.x)[p], fy = gmem<const float>(J.y)[p], fz = gmem<const float>(J.z)[p];
    double md[K];    // merged K nearest (identical on the group's lanes)
    uint32_t mq[K];
    const bool done = knn_search<K>(J, G, wave, grp, q, valid, fx, fy, fz, md, mq);
    if (!valid || q != 0) return;
    const auto nb = gmem(J.nbr) + (size_t)pos * K;
    if (!done) {
        nb[0] = 0xffffffffu;
        return;
    }
#pragma unroll
    for (int m = 0; m < K; ++m) nb[m] = mq[m];
}

// Shapes of a kNN job's points from their stored neighbours, one point per
// thread (64 shapes per wave instead of one per 16-lane group).
template <int K>
__global__ __launch_bounds__(kBlock) void k_knn_shape(SortJob *jobs, const PairDev *pairs) {
    const SortJob &J = jobs[blockIdx.y];
    if (!J.want_shapes || pairs[J.pair].nonfinite) return;
    const int pos = blockIdx.x * kBlock + threadIdx.x;
    if (pos >= J.n) return;
    const auto nb = gmem<const uint32_t>(J.nbr) + (size_t)pos * K;
    uint32_t mq[K];
#pragma unroll
    for (int m = 0; m < K; ++m) mq[m] = nb[m];
    if (mq[0] == 0xffffffffu) return;
    const vf4 pt = gmem(reinterpret_cast<const vf4 *>(J.pts))[pos];
    knn_shape<K>(J, pairs[J.pair].rho, __float_as_uint(pt.w), pt.x, pt.y, pt.z, mq);
}

// ------------------------------------------------------------------ k_gather

__global__ __launch_bounds__(kBlock) void k_gather(SortJob *jobs, const PairDev *pairs) {
    const SortJob &J = jobs[blockIdx.y];
    if (J.kind == kJobKnnTarget || J.kind == kJobKnnSource) return;
    const int pos = blockIdx.x * kBlock + threadIdx.x;
    if (pos >= J.n) return;
    const PairDev &P = pairs[J.pair];
    const uint32_t p = gmem(J.idx)[pos];
    const bool src = J.kind == kJobOrderSource;
    const int n = J.n;
    const auto rec = gmem<const float>(src ? P.s_rec : P.t_rec);
    const auto org = gmem<const float>(src ? P.s_orig : P.t_orig);
    const auto shp = gmem<const float>(src ? P.s_shape : P.t_shape);
    // shape of point p (the identity for isotropic pairs, whose shapes are not computed)
    float sh[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) sh[e] = P.iso ? ((e == 0 || e == 3 || e == 5) ? 1.0f : 0.0f) : shp[(size_t)e * n + p];
    // label vector of point p, zero-padded to 4
    vf4 lab = {0.0f, 0.0f, 0.0f, 0.0f};
    if (P.label_dim > 0) {
        const auto l = gmem<const float>(src ? P.src_label : P.tgt_label) + (size_t)P.label_dim * p;
        lab.x = l[0];
        if (P.label_dim > 1) lab.y = l[1];
        if (P.label_dim > 2) lab.z = l[2];
        if (P.label_dim > 3) lab.w = l[3];
    }
    if (src) {   // source: structure of arrays, read once per point and iteration
        const auto out = gmem(P.s_sorted);
#pragma unroll
        for (int d = 0; d < 3; ++d) out[(size_t)d * n + pos] = rec[(size_t)d * n + p];
#pragma unroll
        for (int e = 0; e < 6; ++e) out[(size_t)(3 + e) * n + pos] = sh[e];
#pragma unroll
        for (int d = 0; d < 3; ++d) out[(size_t)(9 + d) * n + pos] = org[(size_t)d * n + p];
        if (P.label_dim > 0) gmem(reinterpret_cast<vf4 *>(P.s_lab))[pos] = lab;
    } else {     // target: 48-byte records, three float4 loads per candidate
        const int stage = J.kind - kJobStage;
        const auto out = gmem(reinterpret_cast<vf4 *>(P.t_sorted[stage])) + 3 * (size_t)pos;
        out[0] = vf4{rec[p], rec[(size_t)n + p], rec[2 * (size_t)n + p], sh[0]};
        out[1] = vf4{sh[1], sh[2], sh[3], sh[4]};
        out[2] = vf4{sh[5], org[p], org[(size_t)n + p], org[2 * (size_t)n + p]};
        if (P.label_dim > 0) gmem(reinterpret_cast<vf4 *>(P.t_lab[stage]))[pos] = lab;
    }
}

// ------------------------------------------------------------------ batch outputs

// One thread per caller pair: the pose (or the start pose when the pair failed
// or never ran) and the run summary.
__global__ __launch_bounds__(64) void k_output(const PairDev *pairs, const OutSlot *slots, int n_out,
                                               const double *T_init_dev, double *T_out, gcvo_info *info) {
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k >= n_out) return;
    const OutSlot o = slots[k];
    const State *S = o.run >= 0 ? &pairs[o.run].st : nullptr;
    const int status = S ? S->status : o.status;
    double *T = T_out + 16 * (size_t)k;
    for (int a = 0; a < 16; ++a) {
        const double start = T_init_dev ? T_init_dev[16 * (size_t)k + a] : ((a % 5 == 0) ? 1.0 : 0.0);
        T[a] = (S && status == GCVO_OK) ? S->T[a] : start;
    }
    if (!info) return;
    gcvo_info r = {};
    r.status = status;
    if (S) {
        r.converged = S->converged;
        r.iters = S->iter;
        r.stages = S->stage + 1;
        r.pairs_last = S->pairs_last;
        r.f = S->f;
        for (int a = 0; a < 6; ++a) r.g[a] = S->g[a];
        r.xi_l1 = S->xi_l1;
        for (int s = 0; s < kMaxStages; ++s) r.stage_iters[s] = S->stage_iters[s];
        r.damped = S->damped;
    }
    info[k] = r;
}

hipError_t launch_outputs(const PairDev *pairs, const OutSlot *slots, int n_out, const double *T_init_dev,
                          double *T_out, gcvo_info *info, hipStream_t s) {
    if (n_out <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_output, dim3((n_out + 63) / 64), dim3(64), 0, s, pairs, slots, n_out, T_init_dev, T_out,
                       info);
    return hipGetLastError();
}

__global__ __launch_bounds__(64) void k_eval_output(const PairDev *pairs, const OutSlot *slots, int n_out, double *f,
                                                    double *g, double *H, long long *n_pairs, int *status) {
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k >= n_out) return;
    const OutSlot o = slots[k];
    const State *S = o.run >= 0 ? &pairs[o.run].st : nullptr;
    const bool ok = S && S->status == GCVO_OK;
    if (status) status[k] = S ? S->status : o.status;
    if (f) f[k] = ok ? S->f : 0.0;
    if (g)
        for (int a = 0; a < 6; ++a) g[6 * (size_t)k + a] = ok ? S->g[a] : 0.0;
    if (H)
        for (int a = 0; a < 36; ++a) H[36 * (size_t)k + a] = ok ? S->H[a] : 0.0;
    if (n_pairs) n_pairs[k] = ok ? S->pairs_last : 0;
}

hipError_t launch_eval_outputs(const PairDev *pairs, const OutSlot *slots, int n_out, double *f, double *g,
                               double *H, long long *n_pairs, int *status, hipStream_t s) {
    if (n_out <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eval_output, dim3((n_out + 63) / 64), dim3(64), 0, s, pairs, slots, n_out, f, g, H,
                       n_pairs, status);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launcher

template <int K>
static void launch_knn(dim3 grid, dim3 grid_pts, SortJob *jobs, const PairDev *pairs, hipStream_t s) {
    hipLaunchKernelGGL(k_knn<K>, grid, dim3(kBlock), 0, s, jobs, pairs);
    hipLaunchKernelGGL(k_knn_shape<K>, grid_pts, dim3(kBlock), 0, s, jobs, pairs);
}

hipError_t launch_prepare(PairDev *pairs, int n_pairs, int max_n, SortJob *jobs, int n_jobs, int max_job_n,
                          int max_cells, int knn, hipStream_t s) {
    hipLaunchKernelGGL(k_stats, dim3(2 * kStatBlocks, n_pairs), dim3(kBlock), 0, s, pairs);
    static_assert(4 + kMaxStages <= 32, "one setup thread per grid");
    hipLaunchKernelGGL(k_setup, dim3(n_pairs), dim3(32), 0, s, pairs);
    const int bx = (max_n + kBlock - 1) / kBlock;
    if (bx > 0) hipLaunchKernelGGL(k_soa, dim3(bx, 2 * n_pairs), dim3(kBlock), 0, s, pairs);
    const int jx = (max_job_n + kBlock - 1) / kBlock;
    if (n_jobs > 0 && jx > 0) {
        // Cell keys are below max_cells and Morton keys below 2^24: three 8-bit
        // passes while every cell table has at most 2^24 cells, four otherwise
        // (a job with fewer key bits sorts stably on zero digits in its last
        // passes).  The passes alternate between the two buffers and end in keys.
        const int passes = max_cells <= (1 << 24) ? 3 : 4;
        hipLaunchKernelGGL(k_keys, dim3(jx, n_jobs), dim3(kBlock), 0, s, jobs, passes & 1);
        const int tiles = (max_job_n + kSortTile - 1) / kSortTile;
        for (int pass = 0; pass < passes; ++pass) {
            const int in_tmp = (passes - pass) & 1;
            hipLaunchKernelGGL(k_sort_up, dim3(tiles, n_jobs), dim3(256), 0, s, jobs, 8 * pass, in_tmp);
            hipLaunchKernelGGL(k_sort_scan, dim3(n_jobs), dim3(256), 0, s, jobs);
            hipLaunchKernelGGL(k_sort_down, dim3(tiles, n_jobs), dim3(256), 0, s, jobs, 8 * pass, in_tmp);
        }
        hipLaunchKernelGGL(k_cells, dim3((max_job_n + kBlock) / kBlock, n_jobs), dim3(kBlock), 0, s, jobs);
        if (knn > 0) {
            dim3 g((max_job_n + kPointsPerBlock - 1) / kPointsPerBlock, n_jobs), gp(jx, n_jobs);
            switch (knn) {
                case 2: launch_knn<2>(g, gp, jobs, pairs, s); break;
                case 3: launch_knn<3>(g, gp, jobs, pairs, s); break;
                case 4: launch_knn<4>(g, gp, jobs, pairs, s); break;
                case 5: launch_knn<5>(g, gp, jobs, pairs, s); break;
                case 6: launch_knn<6>(g, gp, jobs, pairs, s); break;
                case 7: launch_knn<7>(g, gp, jobs, pairs, s); break;
                case 8: launch_knn<8>(g, gp, jobs, pairs, s); break;
                case 9: launch_knn<9>(g, gp, jobs, pairs, s); break;
                case 10: launch_knn<10>(g, gp, jobs, pairs, s); break;
                case 11: launch_knn<11>(g, gp, jobs, pairs, s); break;
                case 12: launch_knn<12>(g, gp, jobs, pairs, s); break;
                case 13: launch_knn<13>(g, gp, jobs, pairs, s); break;
                case 14: launch_knn<14>(g, gp, jobs, pairs, s); break;
                case 15: launch_knn<15>(g, gp, jobs, pairs, s); break;
                case 16: launch_knn<16>(g, gp, jobs, pairs, s); break;
                default: return hipErrorInvalidValue;
            }
        }
        hipLaunchKernelGGL(k_gather, dim3(jx, n_jobs), dim3(kBlock), 0, s, jobs, pairs);
    }
    return hipGetLastError();
}

}  // namespace gcvo
