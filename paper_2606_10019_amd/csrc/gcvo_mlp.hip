// Warm-start point-set network: forward, loss gradient and Adam, all in HIP.
//
// Kernels (B pairs, P points per cloud, 2B clouds; cloud 2b is pair b's source,
// 2b + 1 its target):
//   k_points      grid (2B, 4), 256 threads.  Each block owns one cloud and 32
//                 of the 128 output channels: both per-point layers run in
//                 registers from LDS copies of the weights, with a running
//                 per-channel maximum (first point wins ties), then a wave and
//                 block argmax reduction.  Writes g = relu(max) and the argmax.
//   k_head        grid B, 128 threads: hid = relu(W3 [g_s, g_t] + b3),
//                 out = W4 hid + b4.
//   k_head_back   grid B, 256 threads: residual, d_out, d_pre3, d_in.
//   k_head_grad   one thread per head parameter, fixed-order sum over pairs.
//   k_points_back grid 2B, 128 threads: channel c routes its gradient to its
//                 argmax point, recomputes that point's first layer, writes the
//                 cloud's W2/b2 gradient rows and sums the W1/b1 gradient over
//                 the channels in channel order (LDS).
//   k_points_grad one thread per per-point parameter, fixed-order sum over clouds.
//   k_poses       one thread per pair: T0 = exp(xi^) in FP64.
//   k_adam        one thread per parameter.
// The per-point layer is a dense 64 x 128 contraction per point, but at P = 1024
// points and B ~ 100 pairs the whole forward is ~4 GFLOP; it runs on FP32 VALU
// with weights broadcast from LDS, which keeps the max-pool and argmax fused
// into the producing loop.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <vector>

#include "gcvo.h"
#include "gcvo_mlp.h"

namespace gcvo_mlp {

constexpr int kIn = 3, kH1 = 64, kH2 = 128, kFeat = 256, kHid = 128, kOut = 6;
constexpr int oW1 = 0, ob1 = oW1 + kH1 * kIn, oW2 = ob1 + kH1, ob2 = oW2 + kH2 * kH1;
constexpr int oW3 = ob2 + kH2, ob3 = oW3 + kHid * kFeat, oW4 = ob3 + kHid, ob4 = oW4 + kOut * kHid;
constexpr int kNParams = ob4 + kOut;
constexpr int kPointParams = oW3;                 // W1, b1, W2, b2: the per-point layers
constexpr int kChunk = 32;                        // channels per k_points block
static_assert(kNParams == GCVO_MLP_N_PARAMS, "parameter layout");

struct Args {
    int B, P;
    const float *tgt_xyz, *src_xyz;
    const long long *off;       // device [4][B]: target starts, target counts, source starts, source counts
    const int *tgt_idx, *src_idx;
    const float *tmotion;       // [B][12] or null
    const float *smotion;       // [B][12] or null
    float inv_scale;
    const uint16_t *w;          // bf16 parameters
    float *g;                   // [B][256]
    int *arg;                   // [B][256]
    float *hid;                 // [B][128]
    float *out;                 // [B][6]
    float *dout;                // [B][6]
    float *dpre3;               // [B][128]
    float *din;                 // [B][256]
    float *sq;                  // [B] squared residual per pair
    float *cgrad;               // [2B][kPointParams]
    int *bad;                   // index error flag
};

__device__ __forceinline__ float bf(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t to_bf16(float x) {
    const uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// The network input of point k of cloud (b, is_tgt): gathered, moved, scaled.  An out-of-range index raises the error flag and reads row 0.
__device__ __forceinline__ void input_point(const Args &a, int b, int is_tgt, int k, float &px, float &py, float &pz) {
    const long long o0 = a.off[(is_tgt ? 0 : 2 * a.B) + b], n = a.off[(is_tgt ? a.B : 3 * a.B) + b];
    int r = (is_tgt ? a.tgt_idx : a.src_idx)[(size_t)b * a.P + k];
    if (r < 0 || (long long)r >= n) {
        a.bad[0] = 1;
        r = 0;
    }
    const float *q = (is_tgt ? a.tgt_xyz : a.src_xyz) + 3 * (o0 + r);
    float x = q[0], y = q[1], z = q[2];
    const float *mot = is_tgt ? a.tmotion : a.smotion;
    if (mot) {
        const float *M = mot + 12 * b;
        const float X = M[0] * x + M[1] * y + M[2] * z + M[3];
        const float Y = M[4] * x + M[5] * y + M[6] * z + M[7];
        const float Z = M[8] * x + M[9] * y + M[10] * z + M[11];
        x = X; y = Y; z = Z;
    }
    px = x * a.inv_scale;
    py = y * a.inv_scale;
    pz = z * a.inv_scale;
}

// (value, index) maximum; ties keep the smaller index.
__device__ __forceinline__ void take_max(float &v, int &i, float ov, int oi) {
    if (ov > v || (ov == v && oi < i)) {
        v = ov;
        i = oi;
    }
}

__global__ __launch_bounds__(256) void k_points(Args a) {
    const int cloud = blockIdx.x, b = cloud >> 1, is_tgt = cloud & 1, c0 = blockIdx.y * kChunk;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ float w1[kH1 * kIn], b1[kH1], w2[kChunk][kH1], b2[kChunk];
    __shared__ float sv[4][kChunk];
    __shared__ int si[4][kChunk];
    for (int i = tid; i < kH1 * kIn; i += 256) w1[i] = bf(a.w[oW1 + i]);
    for (int i = tid; i < kH1; i += 256) b1[i] = bf(a.w[ob1 + i]);
    for (int i = tid; i < kChunk * kH1; i += 256) w2[i / kH1][i % kH1] = bf(a.w[oW2 + c0 * kH1 + i]);
    if (tid < kChunk) b2[tid] = bf(a.w[ob2 + c0 + tid]);
    __syncthreads();

    float best[kChunk];
    int barg[kChunk];
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
        best[c] = -INFINITY;
        barg[c] = 0x7fffffff;
    }
    for (int k = tid; k < a.P; k += 256) {
        float px, py, pz;
        input_point(a, b, is_tgt, k, px, py, pz);
        float h1[kH1];
#pragma unroll
        for (int j = 0; j < kH1; ++j)
            h1[j] = fmaxf(0.0f, fmaf(w1[3 * j + 2], pz, fmaf(w1[3 * j + 1], py, fmaf(w1[3 * j], px, b1[j]))));
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
            float acc = b2[c];
#pragma unroll
            for (int j = 0; j < kH1; ++j) acc = fmaf(w2[c][j], h1[j], acc);
            if (acc > best[c]) {          // k increases per thread: the first maximum stays
                best[c] = acc;
                barg[c] = k;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
        float v = best[c];
        int i = barg[c];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) take_max(v, i, __shfl_xor(v, off, 64), __shfl_xor(i, off, 64));
        if (lane == 0) {
            sv[wave][c] = v;
            si[wave][c] = i;
        }
    }
    __syncthreads();
    if (tid < kChunk) {
        float v = sv[0][tid];
        int i = si[0][tid];
        for (int w = 1; w < 4; ++w) take_max(v, i, sv[w][tid], si[w][tid]);
        const int slot = b * kFeat + is_tgt * kH2 + c0 + tid;
        a.g[slot] = fmaxf(v, 0.0f);
        a.arg[slot] = i;
    }
}

__global__ __launch_bounds__(128) void k_head(Args a) {
    const int b = blockIdx.x, t = threadIdx.x;
    __shared__ float x[kFeat], h[kHid];
    for (int i = t; i < kFeat; i += 128) x[i] = a.g[b * kFeat + i];
    __syncthreads();
    float acc = bf(a.w[ob3 + t]);
    const uint16_t *row = a.w + oW3 + t * kFeat;
    for (int i = 0; i < kFeat; ++i) acc = fmaf(bf(row[i]), x[i], acc);
    const float hv = fmaxf(acc, 0.0f);
    h[t] = hv;
    a.hid[b * kHid + t] = hv;
    __syncthreads();
    if (t < kOut) {
        float o = bf(a.w[ob4 + t]);
        for (int i = 0; i < kHid; ++i) o = fmaf(bf(a.w[oW4 + t * kHid + i]), h[i], o);
        a.out[b * kOut + t] = o;
    }
}

__global__ __launch_bounds__(256) void k_head_back(Args a, const float *y) {
    const int b = blockIdx.x, t = threadIdx.x;
    __shared__ float dout[kOut], dp[kHid];
    if (t == 0) {
        float s = 0.0f;
        for (int m = 0; m < kOut; ++m) {
            const float r = a.out[b * kOut + m] - y[b * kOut + m];
            s = fmaf(r, r, s);
            dout[m] = 2.0f * r / (float)a.B;
            a.dout[b * kOut + m] = dout[m];
        }
        a.sq[b] = s;
    }
    __syncthreads();
    if (t < kHid) {
        float d = 0.0f;
        for (int m = 0; m < kOut; ++m) d = fmaf(bf(a.w[oW4 + m * kHid + t]), dout[m], d);
        d = (a.hid[b * kHid + t] > 0.0f) ? d : 0.0f;
        dp[t] = d;
        a.dpre3[b * kHid + t] = d;
    }
    __syncthreads();
    float s = 0.0f;
    for (int o = 0; o < kHid; ++o) s = fmaf(bf(a.w[oW3 + o * kFeat + t]), dp[o], s);
    a.din[b * kFeat + t] = s;
}

// Head parameter gradients: one thread per parameter, sum over pairs in order.
// Thread 0 also sums the loss.
__global__ __launch_bounds__(256) void k_head_grad(Args a, float *grad, float *loss) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int n_head = kNParams - oW3;
    if (e == 0 && loss) {
        float s = 0.0f;
        for (int b = 0; b < a.B; ++b) s += a.sq[b];
        loss[0] = s / (float)a.B;
    }
    if (e >= n_head) return;
    const int p = oW3 + e;
    float s = 0.0f;
    if (p < ob3) {
        const int o = (p - oW3) / kFeat, i = (p - oW3) % kFeat;
        for (int b = 0; b < a.B; ++b) s = fmaf(a.dpre3[b * kHid + o], a.g[b * kFeat + i], s);
    } else if (p < oW4) {
        const int o = p - ob3;
        for (int b = 0; b < a.B; ++b) s += a.dpre3[b * kHid + o];
    } else if (p < ob4) {
        const int m = (p - oW4) / kHid, o = (p - oW4) % kHid;
        for (int b = 0; b < a.B; ++b) s = fmaf(a.dout[b * kOut + m], a.hid[b * kHid + o], s);
    } else {
        const int m = p - ob4;
        for (int b = 0; b < a.B; ++b) s += a.dout[b * kOut + m];
    }
    grad[p] = s;
}

// Per-cloud gradients of the per-point layers.  Thread c = channel.
__global__ __launch_bounds__(kH2) void k_points_back(Args a) {
    const int cloud = blockIdx.x, b = cloud >> 1, is_tgt = cloud & 1, c = threadIdx.x;
    __shared__ float u[kH2][kH1 + 1];
    __shared__ float xk[kH2][kIn];
    const int slot = b * kFeat + is_tgt * kH2 + c;
    const float delta = (a.g[slot] > 0.0f) ? a.din[slot] : 0.0f;
    float *cg = a.cgrad + (size_t)cloud * kPointParams;
    float px = 0.0f, py = 0.0f, pz = 0.0f;
    if (delta != 0.0f) input_point(a, b, is_tgt, a.arg[slot], px, py, pz);
    xk[c][0] = px; xk[c][1] = py; xk[c][2] = pz;
    for (int j = 0; j < kH1; ++j) {
        const float pre = fmaf(bf(a.w[oW1 + 3 * j + 2]), pz,
                               fmaf(bf(a.w[oW1 + 3 * j + 1]), py, fmaf(bf(a.w[oW1 + 3 * j]), px, bf(a.w[ob1 + j]))));
        const float h1 = fmaxf(pre, 0.0f);
        cg[oW2 + c * kH1 + j] = delta * h1;
        u[c][j] = (pre > 0.0f) ? delta * bf(a.w[oW2 + c * kH1 + j]) : 0.0f;
    }
    cg[ob2 + c] = delta;
    __syncthreads();
    if (c < kH1) {
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, sb = 0.0f;
        for (int ch = 0; ch < kH2; ++ch) {
            const float v = u[ch][c];
            s0 = fmaf(v, xk[ch][0], s0);
            s1 = fmaf(v, xk[ch][1], s1);
            s2 = fmaf(v, xk[ch][2], s2);
            sb += v;
        }
        cg[oW1 + 3 * c] = s0;
        cg[oW1 + 3 * c + 1] = s1;
        cg[oW1 + 3 * c + 2] = s2;
        cg[ob1 + c] = sb;
    }
}

__global__ __launch_bounds__(256) void k_points_grad(Args a, float *grad) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kPointParams) return;
    float s = 0.0f;
    for (int cl = 0; cl < 2 * a.B; ++cl) s += a.cgrad[(size_t)cl * kPointParams + e];
    grad[e] = s;
}

// exp of the twist (w, v): Rodrigues and the left Jacobian, series below 1e-4 rad.
__global__ void k_poses(const float *out, int B, double *T) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double w0 = GCVO_MLP_ROT_SCALE * (double)out[6 * b], w1 = GCVO_MLP_ROT_SCALE * (double)out[6 * b + 1],
                 w2 = GCVO_MLP_ROT_SCALE * (double)out[6 * b + 2];
    const double v[3] = {GCVO_MLP_TRANS_SCALE * (double)out[6 * b + 3], GCVO_MLP_TRANS_SCALE * (double)out[6 * b + 4],
                         GCVO_MLP_TRANS_SCALE * (double)out[6 * b + 5]};
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2, th = sqrt(th2);
    double A, Bc, C;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0;
        Bc = 0.5 - th2 / 24.0;
        C = 1.0 / 6.0 - th2 / 120.0;
    } else {
        const double s = sin(th), hs = sin(0.5 * th);
        A = s / th;
        Bc = 2.0 * hs * hs / th2;
        C = (th - s) / (th2 * th);
    }
    const double W[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
    const double w[3] = {w0, w1, w2};
    double *Tb = T + 16 * b;
    for (int r = 0; r < 3; ++r) {
        double t = 0.0;
        for (int q = 0; q < 3; ++q) {
            const double W2 = w[r] * w[q] - (r == q ? th2 : 0.0);
            const double I = (r == q) ? 1.0 : 0.0;
            Tb[4 * r + q] = I + A * W[r][q] + Bc * W2;
            t += (I + Bc * W[r][q] + C * W2) * v[q];
        }
        Tb[4 * r + 3] = t;
    }
    Tb[12] = Tb[13] = Tb[14] = 0.0;
    Tb[15] = 1.0;
}

__global__ void k_adam(float *w, uint16_t *wb, float *m, float *v, const float *g, long long n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float wi = w[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[e] = wi;
    wb[e] = to_bf16(wi);
}

// ------------------------------------------------------------------ host side

struct Layout {
    size_t off, g, arg, hid, dout, dpre3, din, sq, cgrad, T, bad, total;
};

static size_t up(size_t x) { return (x + 255) & ~size_t(255); }

static bool layout(int B, int P, Layout &L) {
    if (B < 1 || P < 1 || B > GCVO_MLP_MAX_PAIRS || P > GCVO_MLP_MAX_POINTS) return false;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t r = o; o += up(bytes); return r; };
    L.off = take(sizeof(long long) * 4 * B);
    L.g = take(sizeof(float) * B * kFeat);
    L.arg = take(sizeof(int) * B * kFeat);
    L.hid = take(sizeof(float) * B * kHid);
    L.dout = take(sizeof(float) * B * kOut);
    L.dpre3 = take(sizeof(float) * B * kHid);
    L.din = take(sizeof(float) * B * kFeat);
    L.sq = take(sizeof(float) * B);
    L.cgrad = take(sizeof(float) * 2 * (size_t)B * kPointParams);
    L.T = take(sizeof(double) * 16 * B);
    L.bad = take(sizeof(int) * 64);
    L.total = o;
    return true;
}

static int prepare(const gcvo_mlp_batch *bt, const uint16_t *w, void *ws, size_t ws_bytes, hipStream_t s, Args &a,
                   Layout &L) {
    if (!bt || !w || !bt->tgt_xyz || !bt->src_xyz || !bt->tgt_start || !bt->tgt_count || !bt->src_start ||
        !bt->src_count || !bt->tgt_idx || !bt->src_idx || !(bt->input_scale > 0.0f) || !isfinite(bt->input_scale))
        return GCVO_ERR_INVALID;
    if (!layout(bt->n_pairs, bt->n_points, L)) return GCVO_ERR_CAPACITY;
    if (!ws || ws_bytes < L.total || ((uintptr_t)ws & 255)) return GCVO_ERR_WORKSPACE;
    const int B = bt->n_pairs;
    for (int b = 0; b < B; ++b) {
        const long long ts = bt->tgt_start[b], tc = bt->tgt_count[b], ss = bt->src_start[b], sc = bt->src_count[b];
        if (ts < 0 || tc < 1 || ts + tc > bt->n_tgt_rows || ss < 0 || sc < 1 || ss + sc > bt->n_src_rows)
            return GCVO_ERR_INVALID;
    }
    char *base = static_cast<char *>(ws);
    std::vector<long long> offs(4 * (size_t)B);
    for (int b = 0; b < B; ++b) {
        offs[b] = bt->tgt_start[b];
        offs[B + b] = bt->tgt_count[b];
        offs[2 * B + b] = bt->src_start[b];
        offs[3 * B + b] = bt->src_count[b];
    }
    if (hipMemcpyAsync(base + L.off, offs.data(), sizeof(long long) * offs.size(), hipMemcpyHostToDevice, s) !=
        hipSuccess)
        return GCVO_ERR_HIP;
    if (hipMemsetAsync(base + L.bad, 0, sizeof(int), s) != hipSuccess) return GCVO_ERR_HIP;
    // The offsets vector must stay alive until the copy has read it.
    if (hipStreamSynchronize(s) != hipSuccess) return GCVO_ERR_HIP;
    a.B = B;
    a.P = bt->n_points;
    a.tgt_xyz = bt->tgt_xyz;
    a.src_xyz = bt->src_xyz;
    a.off = reinterpret_cast<const long long *>(base + L.off);
    a.tgt_idx = bt->tgt_idx;
    a.src_idx = bt->src_idx;
    a.tmotion = bt->tgt_motion;
    a.smotion = bt->src_motion;
    a.inv_scale = 1.0f / bt->input_scale;
    a.w = w;
    a.g = reinterpret_cast<float *>(base + L.g);
    a.arg = reinterpret_cast<int *>(base + L.arg);
    a.hid = reinterpret_cast<float *>(base + L.hid);
    a.out = nullptr;
    a.dout = reinterpret_cast<float *>(base + L.dout);
    a.dpre3 = reinterpret_cast<float *>(base + L.dpre3);
    a.din = reinterpret_cast<float *>(base + L.din);
    a.sq = reinterpret_cast<float *>(base + L.sq);
    a.cgrad = reinterpret_cast<float *>(base + L.cgrad);
    a.bad = reinterpret_cast<int *>(base + L.bad);
    return GCVO_OK;
}

static int check_bad(const Args &a, hipStream_t s) {
    int bad = 0;
    if (hipMemcpyAsync(&bad, a.bad, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return GCVO_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return GCVO_ERR_HIP;
    return bad ? GCVO_ERR_INVALID : GCVO_OK;
}

static void launch_forward(const Args &a, hipStream_t s) {
    hipLaunchKernelGGL(k_points, dim3(2 * a.B, kH2 / kChunk), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_head, dim3(a.B), dim3(kHid), 0, s, a);
}

}  // namespace gcvo_mlp

using namespace gcvo_mlp;

extern "C" {

long long gcvo_mlp_param_count(void) { return kNParams; }

size_t gcvo_mlp_workspace_size(int n_pairs, int n_points) {
    Layout L;
    return layout(n_pairs, n_points, L) ? L.total : 0;
}

int gcvo_mlp_forward(const gcvo_mlp_batch *batch, const uint16_t *w_bf16, float *out6, double *T_out, void *ws,
                     size_t ws_bytes, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!out6) return GCVO_ERR_INVALID;
    Args a;
    Layout L;
    int rc = prepare(batch, w_bf16, ws, ws_bytes, s, a, L);
    if (rc != GCVO_OK) return rc;
    a.out = out6;
    launch_forward(a, s);
    if (hipGetLastError() != hipSuccess) return GCVO_ERR_HIP;
    if (T_out) {
        hipLaunchKernelGGL(k_poses, dim3((a.B + 63) / 64), dim3(64), 0, s, out6, a.B, T_out);
        if (hipGetLastError() != hipSuccess) return GCVO_ERR_HIP;
    }
    return check_bad(a, s);
}

int gcvo_mlp_loss_grad(const gcvo_mlp_batch *batch, const uint16_t *w_bf16, const float *y6, float *out6,
                       float *loss, float *grad, void *ws, size_t ws_bytes, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!y6 || !loss || !grad) return GCVO_ERR_INVALID;
    Args a;
    Layout L;
    int rc = prepare(batch, w_bf16, ws, ws_bytes, s, a, L);
    if (rc != GCVO_OK) return rc;
    a.out = out6 ? out6 : reinterpret_cast<float *>(static_cast<char *>(ws) + L.T);   // T area holds >= 6B floats
    launch_forward(a, s);
    hipLaunchKernelGGL(k_head_back, dim3(a.B), dim3(kFeat), 0, s, a, y6);
    hipLaunchKernelGGL(k_head_grad, dim3((kNParams - oW3 + 255) / 256), dim3(256), 0, s, a, grad, loss);
    hipLaunchKernelGGL(k_points_back, dim3(2 * a.B), dim3(kH2), 0, s, a);
    hipLaunchKernelGGL(k_points_grad, dim3((kPointParams + 255) / 256), dim3(256), 0, s, a, grad);
    if (hipGetLastError() != hipSuccess) return GCVO_ERR_HIP;
    return check_bad(a, s);
}

int gcvo_mlp_adam(float *w, uint16_t *w_bf16, float *m, float *v, const float *grad, long long n, int step, float lr,
                  float beta1, float beta2, float eps, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!w || !w_bf16 || !m || !v || !grad || n < 1 || step < 1 || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
        !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return GCVO_ERR_INVALID;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, w_bf16, m, v, grad, n, lr, beta1,
                       beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? GCVO_OK : GCVO_ERR_HIP;
}

}  // extern "C"
