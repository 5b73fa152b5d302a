// Host side of the C ABI declared in include/gcvo.h.
//
// Every entry point lays its device data out in the caller's workspace with a
// bump allocator (a sizing pass with no base pointer gives *_workspace_size),
// uploads the POD descriptors of gcvo_dev.h in one copy, enqueues the
// preparation kernels and then the Gauss-Newton iterations in chunks.  The last
// step kernel of a chunk stores each pair's done flag in pinned host memory
// (no copy in the stream); while a chunk runs, the host reads the previous
// chunk's flags, so the device never idles between chunks and at most one
// chunk of no-op launches follows convergence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "gcvo_dev.h"

using namespace gcvo;

namespace {

constexpr int kChunk = 4;   // iterations enqueued per poll

struct Arena {
    char *base;
    size_t off = 0;
    explicit Arena(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Length-scale schedule: ell_0 = ell, ell_{s+1} = max(alpha ell_s, ell_min) until ell_min.
int stage_schedule(const gcvo_params &p, double ells[kMaxStages]) {
    double l = p.length_scale;
    int n = 0;
    for (;;) {
        if (n >= kMaxStages) return -1;
        ells[n++] = l;
        if (!(l > p.length_scale_min)) break;
        l = std::max(p.anneal_factor * l, p.length_scale_min);
    }
    return n;
}

bool params_ok(const gcvo_params *p) {
    if (!p) return false;
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(p->length_scale) || !pos(p->length_scale_min) || p->length_scale_min > p->length_scale) return false;
    if (!(p->anneal_factor > 0.0 && p->anneal_factor <= 1.0)) return false;
    if (p->length_scale_min < p->length_scale && !(p->anneal_factor < 1.0)) return false;
    if (!pos(p->cutoff_scale) || !pos(p->sigma2) || !pos(p->tol) || !pos(p->stage_tol)) return false;
    if (p->knn < 2 || p->knn > kMaxKnn) return false;
    if (!(p->eig_ratio_min > 0.0 && p->eig_ratio_min <= 1.0)) return false;
    if (p->max_iters < 1 || p->max_iters_per_stage < 1) return false;
    if (p->precision != GCVO_PRECISION_FP32 && p->precision != GCVO_PRECISION_FP64) return false;
    if (p->solver != GCVO_SOLVER_GN && p->solver != GCVO_SOLVER_NEWTON && p->solver != GCVO_SOLVER_FIRST_ORDER)
        return false;
    if (p->solver == GCVO_SOLVER_FIRST_ORDER && !pos(p->min_step)) return false;
    if (!(p->cell_fraction >= 0.2 && p->cell_fraction <= 1.0)) return false;
    if (!(p->cell_fraction_x >= 0.1 && p->cell_fraction_x <= 1.0)) return false;
    double e[kMaxStages];
    return stage_schedule(*p, e) > 0;
}

bool pose_ok(const double *T) {
    if (!T) return true;
    for (int a = 0; a < 16; ++a)
        if (!std::isfinite(T[a])) return false;
    if (std::fabs(T[12]) > 1e-6 || std::fabs(T[13]) > 1e-6 || std::fabs(T[14]) > 1e-6 ||
        std::fabs(T[15] - 1.0) > 1e-6)
        return false;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += T[4 * k + a] * T[4 * k + b];
            if (std::fabs(s - (a == b ? 1.0 : 0.0)) > 1e-6) return false;
        }
    const double det = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
                       T[2] * (T[4] * T[9] - T[5] * T[8]);
    return std::fabs(det - 1.0) <= 1e-6;
}

enum class Mode { Register, Eval, Shapes };

struct PairInput {
    const float *tgt, *src;
    long long n_t, n_s;
    gcvo_params p;
    double T0[16];
    const float *tgt_shape = nullptr, *src_shape = nullptr;   // Eval
    float *shape_out = nullptr;                               // Shapes
    double eval_ell = 0.0, eval_cutoff = 0.0;                 // Eval
    const float *tgt_label = nullptr, *src_label = nullptr;   // [n][label_dim] or null
    int label_dim = 0;
    const double *T0_dev = nullptr;                           // device start pose (batch calls) or null: T0
};

// Register mode with eig_ratio_min = 1: every shape is the identity (Remark 3),
// so no neighbourhoods are computed.
bool isotropic(Mode mode, const PairInput &I) { return mode == Mode::Register && I.p.eig_ratio_min >= 1.0; }

struct Plan {
    size_t bytes = 0;
    std::vector<PairDev> pairs;
    std::vector<SortJob> jobs;
    std::vector<BlockTask> tasks;
    PairDev *d_pairs = nullptr;
    SortJob *d_jobs = nullptr;
    BlockTask *d_tasks = nullptr;
    char *desc_begin = nullptr;
    size_t desc_bytes = 0;
    int max_n = 0, max_job_n = 0, max_cells = 0;
    bool labels = false;   // the pairs carry label vectors
    bool iso = false;      // every pair is isotropic
    // batch calls: one output slot per caller pair (set before build_plan)
    std::vector<OutSlot> out;
    OutSlot *d_out = nullptr;
    gcvo_profile *profile = nullptr;   // measurement of the call, or null
};

// Lays out (base == nullptr: sizes) every device array of a batch.
void build_plan(void *base, Mode mode, const std::vector<PairInput> &in, Plan &pl) {
    Arena A(base);
    const int np = (int)in.size();
    // job count and task count first (descriptor block is contiguous)
    int n_jobs = 0, n_tasks = 0;
    std::vector<int> nst(np);
    std::vector<double> ells((size_t)np * kMaxStages);
    for (int k = 0; k < np; ++k) {
        if (mode == Mode::Register) {
            nst[k] = stage_schedule(in[k].p, &ells[(size_t)k * kMaxStages]);
            n_jobs += (isotropic(mode, in[k]) ? 1 : 3) + nst[k];
        } else if (mode == Mode::Eval) {
            nst[k] = 1;
            ells[(size_t)k * kMaxStages] = in[k].eval_ell;
            n_jobs += 2;
        } else {
            nst[k] = 0;
            n_jobs += 1;
        }
        if (mode != Mode::Shapes) n_tasks += (int)((in[k].n_s + kPointsPerBlock - 1) / kPointsPerBlock);
    }
    pl.d_pairs = A.take<PairDev>(np);
    pl.desc_begin = reinterpret_cast<char *>(pl.d_pairs);
    size_t desc_start = A.off - sizeof(PairDev) * np;
    pl.d_jobs = A.take<SortJob>(std::max(n_jobs, 1));
    pl.d_tasks = A.take<BlockTask>(std::max(n_tasks, 1));
    pl.d_out = A.take<OutSlot>(std::max<size_t>(pl.out.size(), 1));
    pl.desc_bytes = A.off - desc_start;
    pl.labels = np > 0 && in[0].label_dim > 0;
    pl.iso = np > 0;
    for (int k = 0; k < np; ++k) pl.iso = pl.iso && isotropic(mode, in[k]);
    if (base) {
        pl.pairs.assign(np, PairDev{});
        pl.jobs.assign(std::max(n_jobs, 1), SortJob{});
        pl.tasks.assign(std::max(n_tasks, 1), BlockTask{});
    }
    int job = 0, task = 0;
    pl.max_n = pl.max_job_n = 0;
    for (int k = 0; k < np; ++k) {
        const PairInput &I = in[k];
        const int nt = (int)I.n_t, ns = (int)I.n_s;
        pl.max_n = std::max(pl.max_n, std::max(nt, ns));
        PairDev P{};
        P.tgt_xyz = I.tgt;
        P.src_xyz = I.src;
        P.n_t = nt;
        P.n_s = ns;
        const bool iso = isotropic(mode, I);
        P.iso = iso ? 1 : 0;
        P.label_dim = (mode == Mode::Shapes) ? 0 : I.label_dim;
        P.tgt_label = I.tgt_label;
        P.src_label = I.src_label;
        P.n_stages = nst[k];
        for (int s = 0; s < nst[k]; ++s) P.ell[s] = ells[(size_t)k * kMaxStages + s];
        P.knn = I.p.knn;
        P.rho = I.p.eig_ratio_min;
        P.cutoff_scale = (mode == Mode::Eval) ? I.eval_cutoff / I.eval_ell : I.p.cutoff_scale;
        for (int s = 0; s < nst[k]; ++s) {
            const double l = P.ell[s];
            P.cut[s] = P.cutoff_scale * l;
            P.kexp[s] = -1.4426950408889634 / (l * l);
            P.k2[s] = 2.0 / (l * l);
        }
        P.sigma2 = I.p.sigma2;
        P.tol = I.p.tol;
        P.stage_tol = I.p.stage_tol;
        P.max_iters = I.p.max_iters;
        P.max_per_stage = I.p.max_iters_per_stage;
        P.solver = (mode == Mode::Eval) ? GCVO_SOLVER_GN : I.p.solver;
        P.min_step = I.p.min_step;
        P.cell_fraction = I.p.cell_fraction;
        P.cell_fraction_x = I.p.cell_fraction_x;
        std::memcpy(P.T_init, I.T0, sizeof P.T_init);
        P.T_init_dev = I.T0_dev;
        P.stat_part = A.take<double>(2 * kStatBlocks * kStatVals);
        P.t_orig = A.take<float>(3 * (size_t)nt);
        P.s_orig = A.take<float>(3 * (size_t)ns);
        P.t_rec = A.take<float>(3 * (size_t)nt);
        P.s_rec = A.take<float>(3 * (size_t)ns);
        if (mode == Mode::Eval) {
            P.t_shape = const_cast<float *>(I.tgt_shape);
            P.s_shape = const_cast<float *>(I.src_shape);
            P.shapes_given = 1;
            P.eval_only = 1;
        } else if (mode == Mode::Register && !iso) {
            P.t_shape = A.take<float>(6 * (size_t)nt);
            P.s_shape = A.take<float>(6 * (size_t)ns);
        }
        if (mode != Mode::Shapes) P.s_sorted = A.take<float>(kSortedRows * (size_t)ns);
        if (P.label_dim > 0) P.s_lab = A.take<float4>((size_t)ns);
        P.iter_pairs = A.take<long long>((size_t)std::max(I.p.max_iters, 1));
        P.n_blocks = (ns + kPointsPerBlock - 1) / kPointsPerBlock;
        P.first_block = task;
        P.partials = A.take<float>((size_t)std::max(P.n_blocks, 1) * kPartialStride * 2);
        // device address of this pair's descriptor (the stage grids and the state live in it)
        PairDev *P_dev = pl.d_pairs ? pl.d_pairs + k : nullptr;
        auto make_job = [&](int kind, int n, const float *x, int max_cells, bool own_grid = true, Grid *grid = nullptr) {
            SortJob J{};
            J.x = x;
            J.y = x ? x + n : nullptr;
            J.z = x ? x + 2 * (size_t)n : nullptr;
            J.n = n;
            J.max_cells = max_cells;
            J.grid = own_grid ? A.take<Grid>(1) : grid;
            J.keys = A.take<uint32_t>(n);
            J.keys_tmp = A.take<uint32_t>(n);
            J.idx = A.take<uint32_t>(n);
            J.idx_tmp = A.take<uint32_t>(n);
            J.cell_start = max_cells > 0 ? A.take<int>((size_t)max_cells + 1) : nullptr;
            J.tile_counts = A.take<unsigned>(256 * (size_t)std::max(1, (n + 1023) / 1024));
            J.pair = k;
            J.kind = kind;
            pl.max_job_n = std::max(pl.max_job_n, n);
            pl.max_cells = std::max(pl.max_cells, max_cells);
            return J;
        };
        // cell tables: at most 16 cells per point (keys stay below 2^30, four radix
        // passes; below 2^24, three passes, for clouds of up to ~1M points)
        const int knn_cells_t = (int)std::min<long long>(16LL * nt + 64, (1 << 30) - 1);
        const int knn_cells_s = (int)std::min<long long>(16LL * ns + 64, (1 << 30) - 1);
        const int stage_cells = knn_cells_t;
        // neighbour lists of the kNN jobs: the shape-only calls' workspace sizes
        // do not know K, so their plans hold room for the largest
        const int nbr_k = (mode == Mode::Shapes) ? kMaxKnn : I.p.knn;
        if ((mode == Mode::Register && !iso) || mode == Mode::Shapes) {
            SortJob J = make_job(kJobKnnTarget, nt, P.t_orig, knn_cells_t);
            J.want_shapes = 1;
            J.pts = A.take<float4>((size_t)J.n);
            J.nbr = A.take<uint32_t>((size_t)J.n * nbr_k);
            J.shape_out = (mode == Mode::Shapes) ? I.shape_out : P.t_shape;
            P.job_knn_t = pl.d_jobs + job;
            if (base) pl.jobs[job] = J;
            ++job;
        }
        if (mode == Mode::Register && !iso) {
            SortJob J = make_job(kJobKnnSource, ns, P.s_orig, knn_cells_s);
            J.want_shapes = 1;
            J.pts = A.take<float4>((size_t)J.n);
            J.nbr = A.take<uint32_t>((size_t)J.n * nbr_k);
            J.shape_out = P.s_shape;
            P.job_knn_s = pl.d_jobs + job;
            if (base) pl.jobs[job] = J;
            ++job;
        }
        if (mode != Mode::Shapes) {
            SortJob J = make_job(kJobOrderSource, ns, P.s_orig, 0);
            J.morton = 1;
            P.job_order_s = pl.d_jobs + job;
            if (base) pl.jobs[job] = J;
            ++job;
            P.job_stage0 = pl.d_jobs + job;
            for (int s = 0; s < nst[k]; ++s) {
                SortJob Js = make_job(kJobStage + s, nt, P.t_rec, stage_cells, false,
                                      P_dev ? &P_dev->t_grid[s] : nullptr);
                P.t_sorted[s] = A.take<float>(kSortedRows * (size_t)nt);
                if (P.label_dim > 0) P.t_lab[s] = A.take<float4>((size_t)nt);
                P.t_cells[s] = Js.cell_start;
                if (base) pl.jobs[job] = Js;
                ++job;
            }
            for (int b = 0; b < P.n_blocks; ++b) {
                if (base) pl.tasks[task] = BlockTask{k, b};
                ++task;
            }
        }
        if (base) pl.pairs[k] = P;
    }
    pl.bytes = A.off + 256;
}

// Pinned host buffers for the completion flags the device writes (two slots
// of one int per pair) and, for calls that report to the host, each pair's
// final state up to its reduction splits, pooled per device.  Each buffer carries an event
// recorded after the last work of the call that used it: it is handed out
// again only once that event has completed, so the tail of one call's no-op
// launches can never write into the next call's flags.  Buffers stay in the
// pool until the process ends (the device may have written them).
struct FlagBuf {
    int *p = nullptr;
    int cap = 0;                 // ints
    hipEvent_t last = nullptr;   // recorded after the last work that writes p
    bool busy = false;
};

class FlagPool {
   public:
    FlagBuf *acquire(int n_flags) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
        std::lock_guard<std::mutex> lock(m_);
        if ((int)per_dev_.size() <= dev) per_dev_.resize(dev + 1);
        auto &bufs = per_dev_[dev];
        for (auto &b : bufs)
            if (!b->busy && b->cap >= n_flags && hipEventQuery(b->last) == hipSuccess) {
                b->busy = true;
                return b.get();
            }
        auto b = std::make_unique<FlagBuf>();
        b->cap = std::max(n_flags, 256);
        void *q = nullptr;
        if (hipHostMalloc(&q, sizeof(int) * (size_t)b->cap, hipHostMallocDefault) != hipSuccess) return nullptr;
        b->p = static_cast<int *>(q);
        if (hipEventCreateWithFlags(&b->last, hipEventDisableTiming) != hipSuccess) return nullptr;
        b->busy = true;
        bufs.push_back(std::move(b));
        return bufs.back().get();
    }
    // Marks b free once the stream passes the work enqueued so far.
    hipError_t release(FlagBuf *b, hipStream_t s) {
        const hipError_t e = hipEventRecord(b->last, s);
        std::lock_guard<std::mutex> lock(m_);
        b->busy = false;
        return e;
    }

   private:
    std::mutex m_;
    std::vector<std::vector<std::unique_ptr<FlagBuf>>> per_dev_;
};

FlagPool g_flag_pool;

#define HIP_OK(expr)                                        \
    do {                                                    \
        if ((expr) != hipSuccess) return GCVO_ERR_HIP;      \
    } while (0)

// pinned: the blob may be staged in the pinned pool (registrations); the
// evaluation calls, the no-allocation one among them, pass false and never
// touch the pool.
int upload_and_prepare(Plan &pl, int knn, hipStream_t s, bool pinned) {
    // Descriptors are contiguous from d_pairs: the host vectors are laid out
    // in one buffer and copied in one transfer (a single pair's launches read
    // no task table, so its blob stops before the table).
    char *d0 = reinterpret_cast<char *>(pl.d_pairs);
    const size_t task_at = reinterpret_cast<char *>(pl.d_tasks) - d0;
    const bool whole = pl.pairs.size() != 1 || !pl.out.empty();
    const size_t bytes = whole ? pl.desc_bytes : task_at;
    // Blobs of up to kPinnedBlob bytes go through the pinned pool; larger ones
    // (batches of many pairs: mostly task table) through pageable memory, so
    // that the pool keeps small buffers only.
    constexpr size_t kPinnedBlob = 256 << 10;
    std::vector<char> pageable;
    FlagBuf *fb = nullptr;
    char *blob;
    if (pinned && bytes <= kPinnedBlob) {
        fb = g_flag_pool.acquire((int)((bytes + sizeof(int) - 1) / sizeof(int)));
        if (!fb) return GCVO_ERR_HIP;
        blob = reinterpret_cast<char *>(fb->p);
    } else {
        pageable.resize(bytes);
        blob = pageable.data();
    }
    std::memset(blob, 0, bytes);
    std::memcpy(blob, pl.pairs.data(), pl.pairs.size() * sizeof(PairDev));
    std::memcpy(blob + (reinterpret_cast<char *>(pl.d_jobs) - d0), pl.jobs.data(), pl.jobs.size() * sizeof(SortJob));
    if (whole) {
        std::memcpy(blob + task_at, pl.tasks.data(), pl.tasks.size() * sizeof(BlockTask));
        std::memcpy(blob + (reinterpret_cast<char *>(pl.d_out) - d0), pl.out.data(), pl.out.size() * sizeof(OutSlot));
    }
    const hipError_t ce = hipMemcpyAsync(d0, blob, bytes, hipMemcpyHostToDevice, s);
    if ((fb && g_flag_pool.release(fb, s) != hipSuccess) || ce != hipSuccess) return GCVO_ERR_HIP;
    if (pl.pairs.empty()) return GCVO_OK;
    const int n_jobs = (int)pl.jobs.size();
    HIP_OK(launch_prepare(pl.d_pairs, (int)pl.pairs.size(), pl.max_n, pl.d_jobs, n_jobs, pl.max_job_n, pl.max_cells,
                          knn, s));
    return GCVO_OK;
}

// After a measured run (the stream synchronised): launches in which some pair
// iterated are the first max_k(iterations of pair k) ones; their
// event-bracketed durations and the pairs logged by the device are added to
// the caller's profile.
int profile_collect(Plan &pl, int launched, int solver, const std::vector<hipEvent_t> &ev) {
    const int passes = passes_per_iteration(solver);
    const int np = (int)pl.pairs.size();
    int active = 0;
    long long pairs = 0, points = 0;
    for (int k = 0; k < np; ++k) {
        State st;
        if (hipMemcpy(&st, &pl.d_pairs[k].st, sizeof st, hipMemcpyDeviceToHost) != hipSuccess) return GCVO_ERR_HIP;
        const int it = std::min(st.iter + ((st.status != GCVO_OK) ? 1 : 0), pl.pairs[k].max_iters);
        active = std::max(active, it);
        if (it > 0) {
            std::vector<long long> log(it);
            if (hipMemcpy(log.data(), pl.pairs[k].iter_pairs, it * sizeof(long long), hipMemcpyDeviceToHost) !=
                hipSuccess)
                return GCVO_ERR_HIP;
            for (long long v : log) pairs += v;
            points += (long long)it * pl.pairs[k].n_s;
        }
    }
    active = std::min(active, launched) * passes;
    pairs *= passes;
    points *= passes;
    double ms = 0.0;
    for (int i = 0; i < active && 2 * i + 1 < (int)ev.size(); ++i) {
        float e = 0.0f;
        if (hipEventElapsedTime(&e, ev[2 * i], ev[2 * i + 1]) != hipSuccess) return GCVO_ERR_HIP;
        ms += e;
    }
    pl.profile->pair_kernel_ms += ms;
    pl.profile->launches += active;
    pl.profile->pairs += pairs;
    pl.profile->source_points += points;
    return GCVO_OK;
}

// Enqueues the iterations chunk by chunk until every pair is done (or
// max_iters).  With wait, or when the call is measured, it returns after the
// stream has finished them; otherwise the last chunk may still be queued.
// Bytes of a pair's state the host reads back: everything before the
// reduction splits (pose, last evaluation, counters, stage record).
constexpr size_t kReportBytes = offsetof(State, sub);
static_assert(kReportBytes % 8 == 0, "the report keeps the state's 8-byte alignment");

// With `report` (np States, host), the pairs' final states are copied there:
// enqueued right after the iterations into the pinned buffer, so that one
// synchronisation covers the iterations still in flight and the copy.
int run_iterations(Plan &pl, int max_iters, int precision, int solver, hipStream_t s, bool wait,
                   State *report = nullptr) {
    const int np = (int)pl.pairs.size();
    if (np == 0) return GCVO_OK;
    const int report_at = 2 * np;   // ints after the flags: 8 bytes per pair, so the report stays 8-byte aligned
    const int n_ints = report ? report_at + (int)(kReportBytes / sizeof(int)) * np : 2 * np;
    FlagBuf *fb = g_flag_pool.acquire(n_ints);
    if (!fb) return GCVO_ERR_HIP;
    int *flags = fb->p;
    hipEvent_t ev[2];
    if (hipEventCreateWithFlags(&ev[0], hipEventDisableTiming) != hipSuccess) {
        g_flag_pool.release(fb, s);
        return GCVO_ERR_HIP;
    }
    if (hipEventCreateWithFlags(&ev[1], hipEventDisableTiming) != hipSuccess) {
        hipEventDestroy(ev[0]);
        g_flag_pool.release(fb, s);
        return GCVO_ERR_HIP;
    }
    std::vector<hipEvent_t> pev;   // measured calls: two events per pair-kernel launch
    const int n_tasks = (int)pl.tasks.size();
    int launched = 0, slot = 0, rc = GCVO_OK;
    bool pending[2] = {false, false};
    auto enqueue = [&](int c) -> hipError_t {
        int *done = flags + (size_t)slot * np;
        if (!pl.profile)
            return launch_iterations(pl.d_pairs, np, pl.d_tasks, n_tasks, c, precision, solver, pl.labels, pl.iso,
                                     done, s);
        const size_t first = pev.size(), per = 2 * (size_t)passes_per_iteration(solver) * c;
        for (size_t i = 0; i < per; ++i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return hipErrorOutOfMemory;
            pev.push_back(e);
        }
        return launch_iterations(pl.d_pairs, np, pl.d_tasks, n_tasks, c, precision, solver, pl.labels, pl.iso,
                                 done, s, pev.data() + first);
    };
    while (rc == GCVO_OK && launched < max_iters) {
        const int c = std::min(kChunk, max_iters - launched);
        if (enqueue(c) != hipSuccess || hipEventRecord(ev[slot], s) != hipSuccess) {
            rc = GCVO_ERR_HIP;
            break;
        }
        launched += c;
        pending[slot] = true;
        const int other = slot ^ 1;
        if (pending[other]) {
            if (hipEventSynchronize(ev[other]) != hipSuccess) {
                rc = GCVO_ERR_HIP;
                break;
            }
            pending[other] = false;
            bool all_done = true;
            for (int k = 0; k < np && all_done; ++k) all_done = flags[(size_t)other * np + k] != 0;
            if (all_done) break;
        }
        slot = other;
    }
    char *rep_buf = reinterpret_cast<char *>(fb->p + report_at);
    if (report && rc == GCVO_OK &&
        hipMemcpy2DAsync(rep_buf, kReportBytes, &pl.d_pairs[0].st, sizeof(PairDev), kReportBytes, np,
                         hipMemcpyDeviceToHost, s) != hipSuccess)
        rc = GCVO_ERR_HIP;
    if ((wait || pl.profile || report) && hipStreamSynchronize(s) != hipSuccess) rc = GCVO_ERR_HIP;
    if (report && rc == GCVO_OK)
        for (int k = 0; k < np; ++k) std::memcpy(&report[k], rep_buf + kReportBytes * (size_t)k, kReportBytes);
    if (g_flag_pool.release(fb, s) != hipSuccess) rc = GCVO_ERR_HIP;
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
    if (rc == GCVO_OK && pl.profile) rc = profile_collect(pl, launched, solver, pev);
    for (hipEvent_t e : pev) hipEventDestroy(e);
    return rc;
}

void fill_info(const State &S, gcvo_info *info) {
    if (!info) return;
    std::memset(info, 0, sizeof *info);
    info->status = S.status;
    info->converged = S.converged;
    info->iters = S.iter;
    info->stages = S.stage + 1;
    info->pairs_last = S.pairs_last;
    info->f = S.f;
    std::memcpy(info->g, S.g, sizeof info->g);
    info->xi_l1 = S.xi_l1;
    for (int s = 0; s < kMaxStages; ++s) info->stage_iters[s] = S.stage_iters[s];
    info->damped = S.damped;
}

bool ws_ok(void *ws, size_t ws_bytes, size_t need) {
    return ws && (reinterpret_cast<uintptr_t>(ws) & 255u) == 0 && ws_bytes >= need;
}

int register_many(Mode mode, std::vector<PairInput> &in, double *T_out, gcvo_info *info, void *ws,
                  size_t ws_bytes, hipStream_t s, int shared_knn, int precision, int solver, int max_iters,
                  gcvo_profile *profile) {
    Plan sizing;
    build_plan(nullptr, mode, in, sizing);
    if (!ws_ok(ws, ws_bytes, sizing.bytes)) return GCVO_ERR_WORKSPACE;
    Plan pl;
    pl.profile = profile;
    build_plan(ws, mode, in, pl);
    int rc = upload_and_prepare(pl, shared_knn, s, true);
    if (rc) return rc;
    const int np = (int)in.size();
    std::vector<State> st(np);
    rc = run_iterations(pl, max_iters, precision, solver, s, true, st.data());
    if (rc) return rc;
    int first_err = GCVO_OK;
    for (int k = 0; k < np; ++k) {
        if (st[k].status == GCVO_OK) std::memcpy(T_out + 16 * (size_t)k, st[k].T, 16 * sizeof(double));
        else if (first_err == GCVO_OK) first_err = st[k].status;
        if (info) fill_info(st[k], info + k);
    }
    return first_err;
}

const double kIdentity[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};

}  // namespace

extern "C" {

void gcvo_default_params(gcvo_params *p) {
    if (!p) return;
    p->length_scale = 0.3;
    p->length_scale_min = 0.3;
    p->anneal_factor = 0.5;
    p->cutoff_scale = 3.0;
    p->knn = 10;
    p->eig_ratio_min = 0.01;
    p->sigma2 = 1.0;
    p->max_iters = 30;
    p->max_iters_per_stage = 30;
    p->tol = 1e-6;
    p->stage_tol = 1e-4;
    p->precision = GCVO_PRECISION_FP32;
    p->solver = GCVO_SOLVER_GN;
    p->min_step = 1e-10;
    p->cell_fraction = 0.5;
    p->cell_fraction_x = 0.125;
    p->profile = nullptr;
}

int gcvo_abi_version(void) { return 200; }

const char *gcvo_strerror(int status) {
    switch (status) {
        case GCVO_OK: return "ok";
        case GCVO_ERR_INVALID: return "invalid argument (null pointer, size, non-finite input, pose or parameter)";
        case GCVO_ERR_TOO_FEW_POINTS: return "a cloud has fewer points than knn";
        case GCVO_ERR_NO_PAIRS: return "no point pair within the cutoff";
        case GCVO_ERR_SINGULAR: return "the damped Gauss-Newton system is singular";
        case GCVO_ERR_WORKSPACE: return "workspace missing, too small or not 256-byte aligned";
        case GCVO_ERR_HIP: return "HIP runtime error";
        case GCVO_ERR_CAPACITY: return "size beyond the library limits";
        default: return "unknown status";
    }
}

size_t gcvo_workspace_size(long long n_tgt, long long n_src, const gcvo_params *p) {
    if (!params_ok(p) || n_tgt < 1 || n_src < 1 || n_tgt > GCVO_MAX_POINTS || n_src > GCVO_MAX_POINTS) return 0;
    std::vector<PairInput> in(1);
    in[0] = PairInput{nullptr, nullptr, n_tgt, n_src, *p, {}};
    Plan pl;
    build_plan(nullptr, Mode::Register, in, pl);
    return pl.bytes;
}

int gcvo_register(const float *tgt_xyz, long long n_tgt, const float *src_xyz, long long n_src,
                  const double *T_init, const gcvo_params *p, double *T_out, gcvo_info *info, void *workspace,
                  size_t workspace_bytes, void *stream) {
    auto fail = [&](int st) {
        if (info) {
            std::memset(info, 0, sizeof *info);
            info->status = st;
        }
        return st;
    };
    if (!tgt_xyz || !src_xyz || !T_out || !params_ok(p) || !pose_ok(T_init) || n_tgt < 0 || n_src < 0)
        return fail(GCVO_ERR_INVALID);
    if (n_tgt > GCVO_MAX_POINTS || n_src > GCVO_MAX_POINTS) return fail(GCVO_ERR_CAPACITY);
    if (n_tgt < p->knn || n_src < p->knn) return fail(GCVO_ERR_TOO_FEW_POINTS);
    std::vector<PairInput> in(1);
    in[0] = PairInput{tgt_xyz, src_xyz, n_tgt, n_src, *p, {}};
    std::memcpy(in[0].T0, T_init ? T_init : kIdentity, sizeof in[0].T0);
    double T[16];
    int rc = register_many(Mode::Register, in, T, info, workspace, workspace_bytes, (hipStream_t)stream, p->knn,
                           p->precision, p->solver, p->max_iters, p->profile);
    if (rc == GCVO_ERR_HIP || rc == GCVO_ERR_WORKSPACE) return fail(rc);   // info not filled by the run
    if (rc != GCVO_OK) return rc;                                           // info holds the run's summary
    std::memcpy(T_out, T, sizeof T);
    return GCVO_OK;
}

}  // extern "C"

namespace {

// The pairs of a batch that run on the device (the others fail before any
// device work: too few points for the neighbourhoods) and every caller pair's
// output slot.
struct BatchSplit {
    std::vector<PairInput> run;
    std::vector<OutSlot> out;
};

// Host validation and the split.  Returns GCVO_OK, or the call's error.
int split_batch(int n_pairs, const float *tgt_xyz, const float *tgt_label, const long long *tgt_off,
                const float *src_xyz, const float *src_label, const long long *src_off, int label_dim,
                const double *T_init_dev, const gcvo_params *p, int shared_params, BatchSplit &B) {
    if (n_pairs < 1 || !tgt_off || !src_off || !p) return GCVO_ERR_INVALID;
    if (label_dim < 0 || label_dim > GCVO_MAX_LABEL_DIM) return GCVO_ERR_INVALID;
    const int knn = p[0].knn, prec = p[0].precision, solver = p[0].solver;
    B.run.clear();
    B.out.assign(n_pairs, OutSlot{-1, GCVO_OK});
    for (int k = 0; k < n_pairs; ++k) {
        const gcvo_params &pk = shared_params ? p[0] : p[k];
        if (!params_ok(&pk) || pk.knn != knn || pk.precision != prec || pk.solver != solver) return GCVO_ERR_INVALID;
        const long long nt = tgt_off[k + 1] - tgt_off[k], ns = src_off[k + 1] - src_off[k];
        if (nt < 0 || ns < 0 || tgt_off[k] < 0 || src_off[k] < 0) return GCVO_ERR_INVALID;
        if (nt > GCVO_MAX_POINTS || ns > GCVO_MAX_POINTS) return GCVO_ERR_CAPACITY;
        if (nt < knn || ns < knn) {
            B.out[k].status = GCVO_ERR_TOO_FEW_POINTS;
            continue;
        }
        PairInput I{tgt_xyz ? tgt_xyz + 3 * tgt_off[k] : nullptr, src_xyz ? src_xyz + 3 * src_off[k] : nullptr,
                    nt, ns, pk, {}};
        std::memcpy(I.T0, kIdentity, sizeof I.T0);
        I.T0_dev = T_init_dev ? T_init_dev + 16 * (size_t)k : nullptr;
        if (label_dim > 0) {
            I.tgt_label = tgt_label ? tgt_label + (size_t)label_dim * tgt_off[k] : nullptr;
            I.src_label = src_label ? src_label + (size_t)label_dim * src_off[k] : nullptr;
            I.label_dim = label_dim;
        }
        B.out[k].run = (int)B.run.size();
        B.run.push_back(I);
    }
    return GCVO_OK;
}

size_t batch_workspace(int n_pairs, const long long *tgt_off, const long long *src_off, const gcvo_params *p,
                       int shared_params, int label_dim) {
    BatchSplit B;
    if (split_batch(n_pairs, nullptr, nullptr, tgt_off, nullptr, nullptr, src_off, label_dim, nullptr, p,
                    shared_params, B) != GCVO_OK)
        return 0;
    Plan pl;
    pl.out = B.out;
    build_plan(nullptr, Mode::Register, B.run, pl);
    return pl.bytes;
}

int register_batch(int n_pairs, const float *tgt_xyz, const float *tgt_label, const long long *tgt_off,
                   const float *src_xyz, const float *src_label, const long long *src_off, int label_dim,
                   const double *T_init, const gcvo_params *p, int shared_params, double *T_out, gcvo_info *info,
                   void *workspace, size_t workspace_bytes, void *stream) {
    if (n_pairs < 1 || !tgt_xyz || !tgt_off || !src_xyz || !src_off || !p || !T_out) return GCVO_ERR_INVALID;
    if (label_dim < 0 || label_dim > GCVO_MAX_LABEL_DIM || (label_dim > 0 && (!tgt_label || !src_label)))
        return GCVO_ERR_INVALID;
    BatchSplit B;
    int rc = split_batch(n_pairs, tgt_xyz, tgt_label, tgt_off, src_xyz, src_label, src_off, label_dim, T_init, p,
                         shared_params, B);
    if (rc) return rc;
    int max_it = 0;
    for (const PairInput &I : B.run) max_it = std::max(max_it, I.p.max_iters);
    hipStream_t s = (hipStream_t)stream;
    Plan sizing;
    sizing.out = B.out;
    build_plan(nullptr, Mode::Register, B.run, sizing);
    if (!ws_ok(workspace, workspace_bytes, sizing.bytes)) return GCVO_ERR_WORKSPACE;
    Plan pl;
    pl.out = B.out;
    pl.profile = p[0].profile;
    build_plan(workspace, Mode::Register, B.run, pl);
    rc = upload_and_prepare(pl, p[0].knn, s, true);
    if (rc) return rc;
    rc = run_iterations(pl, max_it, p[0].precision, p[0].solver, s, false);
    if (rc) return rc;
    HIP_OK(launch_outputs(pl.d_pairs, pl.d_out, n_pairs, T_init, T_out, info, s));
    return GCVO_OK;
}

size_t eval_workspace(long long n_tgt, long long n_src, int label_dim) {
    if (n_tgt < 0 || n_src < 0 || n_tgt > GCVO_MAX_POINTS || n_src > GCVO_MAX_POINTS) return 0;
    if (label_dim < 0 || label_dim > GCVO_MAX_LABEL_DIM) return 0;
    std::vector<PairInput> in(1);
    gcvo_params p;
    gcvo_default_params(&p);
    in[0] = PairInput{nullptr, nullptr, n_tgt, n_src, p, {}};
    in[0].eval_ell = 1.0;
    in[0].eval_cutoff = 3.0;
    in[0].label_dim = label_dim;
    Plan pl;
    build_plan(nullptr, Mode::Eval, in, pl);
    return pl.bytes;
}

int eval_fgh(const float *tgt_xyz, const float *tgt_shape6, const float *tgt_label, long long n_tgt,
             const float *src_xyz, const float *src_shape6, const float *src_label, long long n_src, int label_dim,
             const double *T, double length_scale, double cutoff, double sigma2, int precision, double *f, double *g,
             double *H, long long *n_pairs, void *workspace, size_t workspace_bytes, void *stream) {
    if (!T || !f || !g || !H || n_tgt < 0 || n_src < 0) return GCVO_ERR_INVALID;
    if (label_dim < 0 || label_dim > GCVO_MAX_LABEL_DIM) return GCVO_ERR_INVALID;
    if (label_dim > 0 && ((n_tgt > 0 && !tgt_label) || (n_src > 0 && !src_label))) return GCVO_ERR_INVALID;
    if ((n_tgt > 0 && (!tgt_xyz || !tgt_shape6)) || (n_src > 0 && (!src_xyz || !src_shape6))) return GCVO_ERR_INVALID;
    if (!pose_ok(T) || !(std::isfinite(length_scale) && length_scale > 0.0) || !(cutoff > 0.0) ||
        !(std::isfinite(sigma2) && sigma2 > 0.0))
        return GCVO_ERR_INVALID;
    if (precision != GCVO_PRECISION_FP32 && precision != GCVO_PRECISION_FP64) return GCVO_ERR_INVALID;
    if (n_tgt > GCVO_MAX_POINTS || n_src > GCVO_MAX_POINTS) return GCVO_ERR_CAPACITY;
    if (n_tgt == 0 || n_src == 0) {   // empty double sum
        *f = 0.0;
        std::memset(g, 0, 6 * sizeof(double));
        std::memset(H, 0, 36 * sizeof(double));
        if (n_pairs) *n_pairs = 0;
        return GCVO_OK;
    }
    std::vector<PairInput> in(1);
    gcvo_params p;
    gcvo_default_params(&p);
    p.sigma2 = sigma2;
    p.precision = precision;
    in[0] = PairInput{tgt_xyz, src_xyz, n_tgt, n_src, p, {}};
    std::memcpy(in[0].T0, T, sizeof in[0].T0);
    in[0].tgt_shape = tgt_shape6;
    in[0].src_shape = src_shape6;
    in[0].eval_ell = length_scale;
    in[0].eval_cutoff = cutoff;
    in[0].tgt_label = tgt_label;
    in[0].src_label = src_label;
    in[0].label_dim = label_dim;
    hipStream_t s = (hipStream_t)stream;
    Plan sizing;
    build_plan(nullptr, Mode::Eval, in, sizing);
    if (!ws_ok(workspace, workspace_bytes, sizing.bytes)) return GCVO_ERR_WORKSPACE;
    Plan pl;
    build_plan(workspace, Mode::Eval, in, pl);
    int rc = upload_and_prepare(pl, 0, s, false);
    if (rc) return rc;
    HIP_OK(launch_iterations(pl.d_pairs, 1, pl.d_tasks, (int)pl.tasks.size(), 1, precision, GCVO_SOLVER_GN,
                             pl.labels, false, nullptr, s));
    State st;
    HIP_OK(hipMemcpyAsync(&st, &pl.d_pairs[0].st, sizeof st, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (st.status != GCVO_OK) return st.status;
    *f = st.f;
    std::memcpy(g, st.g, 6 * sizeof(double));
    std::memcpy(H, st.H, 36 * sizeof(double));
    if (n_pairs) *n_pairs = st.pairs_last;
    return GCVO_OK;
}

}  // namespace

extern "C" {

size_t gcvo_batch_workspace_size(int n_pairs, const long long *tgt_off, const long long *src_off,
                                 const gcvo_params *p, int shared_params) {
    return batch_workspace(n_pairs, tgt_off, src_off, p, shared_params, 0);
}

int gcvo_register_batch(int n_pairs, const float *tgt_xyz, const long long *tgt_off, const float *src_xyz,
                        const long long *src_off, const double *T_init, const gcvo_params *p, int shared_params,
                        double *T_out, gcvo_info *info, void *workspace, size_t workspace_bytes, void *stream) {
    return register_batch(n_pairs, tgt_xyz, nullptr, tgt_off, src_xyz, nullptr, src_off, 0, T_init, p,
                          shared_params, T_out, info, workspace, workspace_bytes, stream);
}

size_t gcvo_batch_workspace_size_labeled(int n_pairs, const long long *tgt_off, const long long *src_off,
                                         const gcvo_params *p, int shared_params, int label_dim) {
    if (label_dim < 1) return 0;
    return batch_workspace(n_pairs, tgt_off, src_off, p, shared_params, label_dim);
}

int gcvo_register_batch_labeled(int n_pairs, const float *tgt_xyz, const float *tgt_label,
                                const long long *tgt_off, const float *src_xyz, const float *src_label,
                                const long long *src_off, int label_dim, const double *T_init,
                                const gcvo_params *p, int shared_params, double *T_out, gcvo_info *info,
                                void *workspace, size_t workspace_bytes, void *stream) {
    if (label_dim < 1) return GCVO_ERR_INVALID;
    return register_batch(n_pairs, tgt_xyz, tgt_label, tgt_off, src_xyz, src_label, src_off, label_dim, T_init, p,
                          shared_params, T_out, info, workspace, workspace_bytes, stream);
}

size_t gcvo_eval_workspace_size(long long n_tgt, long long n_src) { return eval_workspace(n_tgt, n_src, 0); }

}  // extern "C"

// ---------------------------------------------------------------- evaluation without allocation

namespace {

// Device scratch of gcvo_eval_fgh_noalloc: one array per GPU, in place of the
// caller's workspace.  Host code never passes the array's name to a kernel or
// a copy (on the host it only stands for the device symbol); it uses the
// device address resolved once per device below.
constexpr size_t kScratchBytes = size_t(GCVO_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's scratch address (resolved on the first call there).
int scratch_of_current_device(void **ptr) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GCVO_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GCVO_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return GCVO_OK;
}

}  // namespace

extern "C" {

int gcvo_eval_fgh_noalloc(const float *tgt_xyz, const float *tgt_shape6, long long n_tgt, const float *src_xyz,
                          const float *src_shape6, long long n_src, const double *T, double length_scale,
                          double cutoff, double sigma2, int precision, double *f, double *g, double *H,
                          long long *n_pairs, void *stream) {
    if (n_tgt < 0 || n_src < 0) return GCVO_ERR_INVALID;
    const size_t need = eval_workspace(n_tgt, n_src, 0);
    if (need == 0 || need > kScratchBytes) return GCVO_ERR_CAPACITY;
    void *ws = nullptr;
    const int rc = scratch_of_current_device(&ws);
    if (rc) return rc;
    return eval_fgh(tgt_xyz, tgt_shape6, nullptr, n_tgt, src_xyz, src_shape6, nullptr, n_src, 0, T, length_scale,
                    cutoff, sigma2, precision, f, g, H, n_pairs, ws, kScratchBytes, stream);
}

int gcvo_eval_fgh(const float *tgt_xyz, const float *tgt_shape6, long long n_tgt, const float *src_xyz,
                  const float *src_shape6, long long n_src, const double *T, double length_scale, double cutoff,
                  double sigma2, int precision, double *f, double *g, double *H, long long *n_pairs,
                  void *workspace, size_t workspace_bytes, void *stream) {
    return eval_fgh(tgt_xyz, tgt_shape6, nullptr, n_tgt, src_xyz, src_shape6, nullptr, n_src, 0, T, length_scale,
                    cutoff, sigma2, precision, f, g, H, n_pairs, workspace, workspace_bytes, stream);
}

size_t gcvo_eval_workspace_size_labeled(long long n_tgt, long long n_src, int label_dim) {
    if (label_dim < 1) return 0;
    return eval_workspace(n_tgt, n_src, label_dim);
}

int gcvo_eval_fgh_labeled(const float *tgt_xyz, const float *tgt_shape6, const float *tgt_label, long long n_tgt,
                          const float *src_xyz, const float *src_shape6, const float *src_label, long long n_src,
                          int label_dim, const double *T, double length_scale, double cutoff, double sigma2,
                          int precision, double *f, double *g, double *H, long long *n_pairs, void *workspace,
                          size_t workspace_bytes, void *stream) {
    if (label_dim < 1) return GCVO_ERR_INVALID;
    return eval_fgh(tgt_xyz, tgt_shape6, tgt_label, n_tgt, src_xyz, src_shape6, src_label, n_src, label_dim, T,
                    length_scale, cutoff, sigma2, precision, f, g, H, n_pairs, workspace, workspace_bytes, stream);
}

// ---------------------------------------------------------------- batched shapes and evaluations

namespace {

// Clouds of a shapes batch, or the error of the call.
int shapes_inputs(int n_clouds, const float *xyz, const long long *off, int knn, double rho, float *out,
                  std::vector<PairInput> &in) {
    if (n_clouds < 1 || !off || knn < 2 || knn > kMaxKnn || !(rho > 0.0 && rho <= 1.0)) return GCVO_ERR_INVALID;
    gcvo_params p;
    gcvo_default_params(&p);
    p.knn = knn;
    p.eig_ratio_min = rho;
    in.clear();
    for (int k = 0; k < n_clouds; ++k) {
        const long long n = off[k + 1] - off[k];
        if (off[k] < 0 || n < 0) return GCVO_ERR_INVALID;
        if (n > GCVO_MAX_POINTS) return GCVO_ERR_CAPACITY;
        if (n < knn) return GCVO_ERR_TOO_FEW_POINTS;
        PairInput I{xyz ? xyz + 3 * off[k] : nullptr, xyz ? xyz + 3 * off[k] : nullptr, n, 0, p, {}};
        std::memcpy(I.T0, kIdentity, sizeof I.T0);
        I.shape_out = out ? out + 6 * off[k] : nullptr;
        in.push_back(I);
    }
    return GCVO_OK;
}

// Pairs of an evaluation batch: pairs with an empty cloud never run (their
// sums are zero); the rest evaluate at their pose.
int eval_inputs(int n_pairs, const float *tgt_xyz, const float *tgt_shape6, const long long *tgt_off,
                const float *src_xyz, const float *src_shape6, const long long *src_off, const double *T_dev,
                const double *ell, double cutoff_scale, double sigma2, int precision, std::vector<PairInput> &in,
                std::vector<OutSlot> &out) {
    if (n_pairs < 1 || !tgt_off || !src_off || !ell) return GCVO_ERR_INVALID;
    if (!(std::isfinite(cutoff_scale) && cutoff_scale > 0.0) || !(std::isfinite(sigma2) && sigma2 > 0.0))
        return GCVO_ERR_INVALID;
    if (precision != GCVO_PRECISION_FP32 && precision != GCVO_PRECISION_FP64) return GCVO_ERR_INVALID;
    gcvo_params p;
    gcvo_default_params(&p);
    p.sigma2 = sigma2;
    p.precision = precision;
    in.clear();
    out.assign(n_pairs, OutSlot{-1, GCVO_OK});
    for (int k = 0; k < n_pairs; ++k) {
        const long long nt = tgt_off[k + 1] - tgt_off[k], ns = src_off[k + 1] - src_off[k];
        if (tgt_off[k] < 0 || src_off[k] < 0 || nt < 0 || ns < 0) return GCVO_ERR_INVALID;
        if (nt > GCVO_MAX_POINTS || ns > GCVO_MAX_POINTS) return GCVO_ERR_CAPACITY;
        if (!(std::isfinite(ell[k]) && ell[k] > 0.0)) return GCVO_ERR_INVALID;
        if (nt == 0 || ns == 0) continue;
        PairInput I{tgt_xyz ? tgt_xyz + 3 * tgt_off[k] : nullptr, src_xyz ? src_xyz + 3 * src_off[k] : nullptr,
                    nt, ns, p, {}};
        std::memcpy(I.T0, kIdentity, sizeof I.T0);
        I.T0_dev = T_dev ? T_dev + 16 * (size_t)k : nullptr;
        I.tgt_shape = tgt_shape6 ? tgt_shape6 + 6 * tgt_off[k] : nullptr;
        I.src_shape = src_shape6 ? src_shape6 + 6 * src_off[k] : nullptr;
        I.eval_ell = ell[k];
        I.eval_cutoff = cutoff_scale * ell[k];
        out[k].run = (int)in.size();
        in.push_back(I);
    }
    return GCVO_OK;
}

}  // namespace

size_t gcvo_shapes_batch_workspace_size(int n_clouds, const long long *off) {
    std::vector<PairInput> in;
    if (shapes_inputs(n_clouds, nullptr, off, 2, 0.5, nullptr, in) != GCVO_OK) return 0;
    Plan pl;
    build_plan(nullptr, Mode::Shapes, in, pl);
    return pl.bytes;
}

int gcvo_point_shapes_batch(int n_clouds, const float *xyz, const long long *off, int knn, double rho,
                            float *shape6_out, void *workspace, size_t workspace_bytes, void *stream) {
    if (!xyz || !shape6_out) return GCVO_ERR_INVALID;
    std::vector<PairInput> in;
    int rc = shapes_inputs(n_clouds, xyz, off, knn, rho, shape6_out, in);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Plan sizing;
    build_plan(nullptr, Mode::Shapes, in, sizing);
    if (!ws_ok(workspace, workspace_bytes, sizing.bytes)) return GCVO_ERR_WORKSPACE;
    Plan pl;
    build_plan(workspace, Mode::Shapes, in, pl);
    return upload_and_prepare(pl, knn, s, true);
}

size_t gcvo_eval_batch_workspace_size(int n_pairs, const long long *tgt_off, const long long *src_off) {
    std::vector<PairInput> in;
    std::vector<OutSlot> out;
    if (n_pairs < 1 || !tgt_off || !src_off) return 0;
    std::vector<double> ell(n_pairs, 1.0);
    if (eval_inputs(n_pairs, nullptr, nullptr, tgt_off, nullptr, nullptr, src_off, nullptr, ell.data(), 3.0, 1.0,
                    GCVO_PRECISION_FP32, in, out) != GCVO_OK)
        return 0;
    Plan pl;
    pl.out = out;
    build_plan(nullptr, Mode::Eval, in, pl);
    return pl.bytes;
}

int gcvo_eval_fgh_batch(int n_pairs, const float *tgt_xyz, const float *tgt_shape6, const long long *tgt_off,
                        const float *src_xyz, const float *src_shape6, const long long *src_off, const double *T,
                        const double *length_scale, double cutoff_scale, double sigma2, int precision, double *f,
                        double *g, double *H, long long *n_pairs_out, int *status, void *workspace,
                        size_t workspace_bytes, void *stream) {
    if (!tgt_xyz || !tgt_shape6 || !src_xyz || !src_shape6) return GCVO_ERR_INVALID;
    std::vector<PairInput> in;
    std::vector<OutSlot> out;
    int rc = eval_inputs(n_pairs, tgt_xyz, tgt_shape6, tgt_off, src_xyz, src_shape6, src_off, T, length_scale,
                         cutoff_scale, sigma2, precision, in, out);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Plan sizing;
    sizing.out = out;
    build_plan(nullptr, Mode::Eval, in, sizing);
    if (!ws_ok(workspace, workspace_bytes, sizing.bytes)) return GCVO_ERR_WORKSPACE;
    Plan pl;
    pl.out = out;
    build_plan(workspace, Mode::Eval, in, pl);
    rc = upload_and_prepare(pl, 0, s, false);
    if (rc) return rc;
    if (!in.empty())
        HIP_OK(launch_iterations(pl.d_pairs, (int)in.size(), pl.d_tasks, (int)pl.tasks.size(), 1, precision,
                                 GCVO_SOLVER_GN, false, false, nullptr, s));
    HIP_OK(launch_eval_outputs(pl.d_pairs, pl.d_out, n_pairs, f, g, H, n_pairs_out, status, s));
    return GCVO_OK;
}

size_t gcvo_shapes_workspace_size(long long n) {
    if (n < 1 || n > GCVO_MAX_POINTS) return 0;
    std::vector<PairInput> in(1);
    gcvo_params p;
    gcvo_default_params(&p);
    in[0] = PairInput{nullptr, nullptr, n, 0, p, {}};
    Plan pl;
    build_plan(nullptr, Mode::Shapes, in, pl);
    return pl.bytes;
}

int gcvo_point_shapes(const float *xyz, long long n, int knn, double rho, float *shape6_out, void *workspace,
                      size_t workspace_bytes, void *stream) {
    if (!xyz || !shape6_out || n < 0 || knn < 2 || knn > kMaxKnn || !(rho > 0.0 && rho <= 1.0))
        return GCVO_ERR_INVALID;
    if (n > GCVO_MAX_POINTS) return GCVO_ERR_CAPACITY;
    if (n < knn) return GCVO_ERR_TOO_FEW_POINTS;
    std::vector<PairInput> in(1);
    gcvo_params p;
    gcvo_default_params(&p);
    p.knn = knn;
    p.eig_ratio_min = rho;
    in[0] = PairInput{xyz, xyz, n, 0, p, {}};
    std::memcpy(in[0].T0, kIdentity, sizeof in[0].T0);
    in[0].shape_out = shape6_out;
    hipStream_t s = (hipStream_t)stream;
    Plan sizing;
    build_plan(nullptr, Mode::Shapes, in, sizing);
    if (!ws_ok(workspace, workspace_bytes, sizing.bytes)) return GCVO_ERR_WORKSPACE;
    Plan pl;
    build_plan(workspace, Mode::Shapes, in, pl);
    return upload_and_prepare(pl, knn, s, true);
}

}  // extern "C"
