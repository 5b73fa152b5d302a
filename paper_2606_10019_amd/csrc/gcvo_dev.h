// Internal device/host structures of the gfx950 G-CVO library.
//
// Work is described by small POD descriptors that live in device memory inside
// the caller's workspace: one PairDev per registration problem, one SortJob per
// (cloud, uniform grid) binning, one BlockTask per block of kPointsPerBlock
// source points of the per-iteration pair kernel.  A single registration is a
// batch of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gcvo.h"

namespace gcvo {

constexpr int kBlock = 256;           // threads of point-parallel kernels (4 waves)
constexpr int kStatBlocks = 16;      // bounds kernel: blocks per cloud
constexpr int kStatVals = 10;        // per bounds block: 3 FP64 sums, 3 minima, 3 maxima, non-finite flag
constexpr int kMaxStages = GCVO_MAX_STAGES;
constexpr int kMaxKnn = GCVO_MAX_KNN;
constexpr int kNumSums = 28;          // f, g (6), upper triangle of H_main (21)
constexpr int kSumsExact = 58;        // + upper triangle of T1 (21) + sum_j y_j a_j^T (9)
constexpr int kSumsLine = 5;          // line-search polynomial coefficients c0..c4
constexpr int kMaxSums = 64;          // room per reduction slot
constexpr int kPartialStride = 64;    // elements per block partial: sums + pair count + pad
constexpr float kCellMargin = 1.001f; // pair-grid cell edge = margin * cutoff (see Grid)
constexpr int kSortedRows = 12;      // rows of the sorted per-point arrays (see PairDev)
constexpr int kGroupLanes = 16;      // pair kernel: lanes serving one source point
constexpr int kGroupsPerWave = 64 / kGroupLanes;
constexpr int kPointsPerBlock = (kBlock / 64) * kGroupsPerWave;   // source points per pair-kernel block
constexpr int kMaxRows = 64;         // pair kernel: cell rows listed per batch and point
constexpr int kReduceSplit = 16;     // blocks per pair of the cross-block reduction

// Uniform grid over an axis-aligned box.  Cell of a point p along axis d is
// clamp(floor((p_d - lo_d) * inv_h), 0, n_d - 1); cells are numbered x-fastest.
// The pair grid's edge is half the cutoff (grown when the box would need more
// cells than the workspace holds); the pair kernel finds candidates with a ball
// of radius 1.001 * cutoff, which absorbs FP32 rounding of cell coordinates.
struct Grid {
    float lo[3];
    float h;
    float inv_h;
    int n[3];
    int ncells;
    int key_bits;   // bits needed to hold ncells - 1 (24 for a Morton grid)
    float hx;       // cell edge along x (pair grids may use finer x cells; h otherwise)
    float inv_hx;
};

// Sort of one cloud's points into one grid: keys, a stable LSD radix sort of
// (key, index), and cell_start[c] = first sorted position of cell c
// (cell_start[ncells] = n), so cell c holds sorted positions
// [cell_start[c], cell_start[c + 1]).
struct SortJob {
    const float *x, *y, *z;   // SoA coordinates the grid is built over
    int n;
    int max_cells;            // capacity of cell_start minus one
    Grid *grid;               // written by the setup kernel
    uint32_t *keys, *keys_tmp, *idx, *idx_tmp;   // idx: sorted position -> point index
    int *cell_start;
    unsigned *tile_counts;    // radix sort scratch: [ceil(n / 1024)][256] digit counts per tile, then offsets
    int pair;                 // owning pair
    int kind;                 // kJobKnnTarget, kJobKnnSource or kJobStage + stage
    int want_shapes;          // kNN jobs: 1 = compute shapes into shape_out
    int morton;               // 1: key = 24-bit Morton code of the 256^3 grid cell (no cell table)
    float *shape_out;         // SoA [6][n], original point order
    float4 *pts;              // kNN jobs: {x, y, z, point index bits} in sorted order
    uint32_t *nbr;            // kNN jobs: [n][knn] neighbour indices in sorted order (first 0xffffffff: none)
};

constexpr int kJobKnnTarget = 0;    // grid for the target's kNN shapes
constexpr int kJobKnnSource = 1;    // grid for the source's kNN shapes
constexpr int kJobOrderSource = 2;  // Morton order of the source (pair-kernel point order)
constexpr int kJobStage = 3;        // kJobStage + s: pair grid of stage s over the target

// Per-pair solver state, FP64, owned by the device for the whole solve.
struct State {
    double T[16];          // current pose in the caller's frame (row-major 4x4; the pair kernel recentres it)
    double f, g[6], H[36]; // last evaluation (H = H_GN incl. connection term)
    double xi[6];
    double xi_l1;
    long long pairs_last;
    int iter, stage, stage_iter, done, status, converged, damped;
    int stage_iters[kMaxStages];
    int phase;                        // first-order solver: 0 = gradient pass next, 1 = line pass next
    int pad0;
    double dir[6];                    // first-order solver: unit ascent direction (caller frame)
    double gnorm;                     // its gradient's norm
    double sub[kReduceSplit][kMaxSums];   // cross-block sums of the current pass by reduction block; the pair count follows the sums
};

// Everything one registration problem needs on the device.
struct PairDev {
    // caller inputs
    const float *tgt_xyz, *src_xyz;   // AoS [n][3]
    const float *tgt_label, *src_label;   // AoS [n][label_dim] label vectors, or null
    int n_t, n_s;
    int label_dim;                    // 0: no labels (c_ij = 1)
    int iso;                          // 1: every shape is the identity (eig_ratio_min >= 1; no kNN)
    // solver parameters
    double ell[kMaxStages];
    // per-stage constants of the pair kernel, from ell in FP64 on the host (the
    // same correctly rounded values the device would compute): the cutoff
    // cutoff_scale * ell, -log2(e) / ell^2 and 2 / ell^2
    double cut[kMaxStages], kexp[kMaxStages], k2[kMaxStages];
    int n_stages;
    int knn;
    double rho, cutoff_scale, sigma2, tol, stage_tol;
    int max_iters, max_per_stage;
    int solver;                       // GCVO_SOLVER_*
    double min_step;                  // first-order solver: smallest step mu
    double cell_fraction;             // pair-grid cell edge (y, z) as a fraction of the cutoff
    double cell_fraction_x;           // pair-grid cell edge along x (the row direction), same unit
    double T_init[16];                // caller frame
    const double *T_init_dev;         // device [16] start pose (batch calls), checked to be in SE(3); or null: T_init
    // derived on device
    double centre[3];                 // target centroid, subtracted before the FP32 cast
    double *stat_part;                // [2][kStatBlocks][kStatVals] bounds of target and source, per block
    int nonfinite;                    // 1 if any input coordinate is NaN or Inf
    // workspace arrays
    float *t_orig, *s_orig;           // SoA [3][n] original coordinates (kNN grids)
    float *t_rec, *s_rec;             // SoA [3][n] recentred coordinates
    float *t_shape, *s_shape;         // SoA [6][n] shapes, original point order
    // Sorted per-point arrays of kSortedRows floats per point: recentred xyz
    // (float32), the 6 shape entries, original xyz (read by the FP64
    // instantiation, which recentres exactly in FP64).  The source is stored as
    // structure of arrays [12][n]; the target as 48-byte records
    // {x, y, z, s00 | s01, s02, s11, s12 | s22, x0, y0, z0} (three float4).
    float *s_sorted;                  // source, in Morton order
    float *t_sorted[kMaxStages];      // target, in each stage grid's order
    float4 *s_lab;                    // source labels padded to 4 with zeros, Morton order (labels only)
    float4 *t_lab[kMaxStages];        // target labels in each stage grid's order (labels only)
    int *t_cells[kMaxStages];         // cell_start of each stage grid
    Grid t_grid[kMaxStages];          // pair grid of each stage (held here: one load fewer per kernel)
    SortJob *job_knn_t, *job_knn_s, *job_order_s, *job_stage0;   // job_stage0[s] for s < n_stages

    long long *iter_pairs;            // [max_iters] pairs within the cutoff at each iteration
    void *partials;                   // [n_blocks][kPartialStride] block sums (pair-term precision)
    int n_blocks;                     // pair-kernel blocks (kPointsPerBlock source points each)
    int first_block;                  // index of the pair's first BlockTask
    int shapes_given;                 // 1: t_shape / s_shape are caller memory (eval path)
    int eval_only;                    // 1: stop after one evaluation, no step
    // Solver state, held in the descriptor so that a kernel reaches it with the
    // descriptor's own loads (no pointer to follow).
    State st;
};

// Where a caller's pair k of a batch call finds its result: run >= 0 is the
// index of the pair in the device batch; run < 0 means it never ran and
// `status` is its error.
struct OutSlot {
    int run;
    int status;
};

struct BlockTask {   // one block of the pair kernel: a pair and a kPointsPerBlock-point slice of its source
    int pair;
    int block;       // block index within the pair
};

// Native 4-float vector (float4 is a class whose members expect generic
// addresses; this type loads and stores through any address space).
typedef float __attribute__((ext_vector_type(4))) vf4;

// Global-memory view of a generic pointer to device memory: accesses through it
// are global instructions, not flat ones (a flat access also counts against the
// counter of LDS and scalar loads, so waiting for it waits for those as well).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// ---------------------------------------------------------------- wave helpers

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// DPP lane permutations within a 16-lane row (one point's group of lanes):
// the row mirrored (lane i with 15 - i), each half-row mirrored (i with 7 - i),
// neighbours of a quad swapped, pairs of a quad swapped.  Applied in this order,
// each step combines two equal-sized disjoint sets of lanes, so after the four
// steps every lane of the row has combined all 16 values.
constexpr int kDppRowMirror = 0x140, kDppRowHalfMirror = 0x141, kDppQuadSwap1 = 0xB1, kDppQuadSwap2 = 0x4E;
static_assert(kGroupLanes == 16, "a group of lanes is one DPP row");
template <int Ctrl>
__device__ __forceinline__ unsigned dpp_row(unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, Ctrl, 0xF, 0xF, true);
}
template <int Ctrl>
__device__ __forceinline__ float dpp_row(float v) {
    return __builtin_bit_cast(float, dpp_row<Ctrl>(__builtin_bit_cast(unsigned, v)));
}
template <int Ctrl>
__device__ __forceinline__ double dpp_row(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = dpp_row<Ctrl>((unsigned)b), hi = dpp_row<Ctrl>((unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// ---------------------------------------------------------------- host launchers

// Enqueue the per-registration preparation: bounds and centroid, grids, SoA
// copies, cell keys, radix sorts, kNN shapes and the sorted per-stage arrays.
// knn selects the kNN kernel instantiation (0: no shapes are computed).
hipError_t launch_prepare(PairDev *pairs_dev, int n_pairs, int max_n, SortJob *jobs_dev, int n_jobs,
                          int max_job_n, int max_cells, int knn, hipStream_t s);
// Enqueue n_iters solver iterations (each a no-op for pairs already done) of
// the given solver (GCVO_SOLVER_*; all pairs of a batch share it).  With
// host_done non-null (pinned host memory, n_pairs ints), the last pass stores
// every pair's done flag there.
// With `events` non-null, every pair-kernel launch is bracketed by two of them
// (2 * passes_per_iteration(solver) * n_iters events, recorded in order).
// labels: the pairs carry label vectors (all pairs of a batch or none);
// iso: every pair's shapes are the identity (the isotropic pair kernel is used
// for Gauss-Newton).
hipError_t launch_iterations(PairDev *pairs_dev, int n_pairs, BlockTask *tasks_dev, int n_tasks, int n_iters,
                             int precision, int solver, bool labels, bool iso, int *host_done, hipStream_t s,
                             hipEvent_t *events = nullptr);
// Pair-kernel passes per solver iteration (2 for the first-order solver).
int passes_per_iteration(int solver);
// Enqueue the outputs of a batch call: for caller pair k, T_out[k] (device
// [16]) = the solved pose, or the start pose (T_init_dev + 16 k, identity when
// null) when the pair failed or never ran; info[k] (device, may be null) = the
// run summary or {status, 0...}.
hipError_t launch_outputs(const PairDev *pairs, const OutSlot *slots, int n_out, const double *T_init_dev,
                          double *T_out, gcvo_info *info, hipStream_t s);
// Enqueue the outputs of a batch of evaluations: for caller pair k, f[k],
// g[k][6], H[k][36], n_pairs[k] and status[k] (each device, may be null) from
// the evaluation, or zeros (an empty double sum) when the pair never ran.
hipError_t launch_eval_outputs(const PairDev *pairs, const OutSlot *slots, int n_out, double *f, double *g,
                               double *H, long long *n_pairs, int *status, hipStream_t s);

}  // namespace gcvo
