/*
 * gcvo_mlp.h - C ABI of the learned warm start: a point-set network that
 * predicts an initial pose for the registration from two subsampled clouds.
 *
 * The paper has no learned component: it warm-starts consecutive LiDAR frames
 * only with a constant-velocity guess (Sec. "LiDAR odometry" experiments) and
 * names learning as future work (Sec. "Conclusion").  This network is the
 * project's addition; the registration it feeds (gcvo.h) is the paper's
 * method, which refines the prediction and judges it.
 *
 * Network (per pair b; P input points per cloud):
 *     per point p of each cloud:   h1 = relu(W1 p + b1)    3 -> 64
 *                                  h2 = relu(W2 h1 + b2)   64 -> 128
 *     per cloud:                   g = channel-wise max of h2 over the P points
 *     per pair:                    hid = relu(W3 [g_source, g_target] + b3)   256 -> 128
 *                                  out = W4 hid + b4                          128 -> 6
 * The output is a normalised twist: xi = (GCVO_MLP_ROT_SCALE * out[0..2],
 * GCVO_MLP_TRANS_SCALE * out[3..5]) (rotation first), and the predicted
 * registration pose is T0 = exp(xi^) (the same convention as gcvo.h: x ~ T^{-1} z).
 * Training minimises L = (1/B) sum_b ||out_b - y_b||^2 with y_b the normalised
 * twist of the label pose.
 *
 * Parameters.  One flat vector of GCVO_MLP_N_PARAMS values: W1 [64][3], b1 [64],
 * W2 [128][64], b2 [128], W3 [128][256], b3 [128], W4 [6][128], b4 [6],
 * row-major, in that order.  The forward pass reads them as bfloat16 (raw
 * 16-bit patterns, device memory); all sums run in FP32.  Training keeps FP32
 * master weights and Adam moments (device memory) and rewrites the bfloat16
 * copy after every step (round to nearest, ties to even).
 *
 * Inputs (gcvo_mlp_batch).  Clouds live in two device arrays, float32
 * [rows][3]; sample b's target is rows tgt_start[b] .. tgt_start[b] +
 * tgt_count[b] - 1 of the target array (host int64 arrays; ranges may repeat or
 * overlap, so a training batch can draw the same pair twice), likewise for the
 * source.  For every sample, tgt_idx / src_idx (device int32,
 * [n_pairs][n_points]) list the rows of that sample's cloud fed to the network
 * (a subsample drawn by the caller; indices are relative to the range start).
 * tgt_motion / src_motion (device float32 [n_pairs][12], row-major 3x4 [R | t],
 * or NULL) move that cloud's points, p -> R p + t, before they enter the
 * network (used to re-pose training pairs; the label moves with them).  Every
 * coordinate is then divided by input_scale (metres).
 *
 * Gradients of the max over points go to the first point (lowest position in
 * the index list) attaining the maximum; relu'(0) = 0.
 *
 * Memory, streams, errors and determinism follow gcvo.h: device work is
 * enqueued on `stream`; the calls return without waiting, except for the index
 * check below.  An index
 * outside its cloud makes the call return GCVO_ERR_INVALID (the kernels read row
 * 0 of that cloud instead, so nothing is read out of bounds); that check waits
 * for the stream.  Sums over points, pairs and clouds run in a fixed order
 * without atomics, so results are bitwise repeatable.
 */
#ifndef GCVO_MLP_H
#define GCVO_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GCVO_MLP_N_PARAMS 42246
#define GCVO_MLP_ROT_SCALE 0.3   /* rad per unit of out[0..2] */
#define GCVO_MLP_TRANS_SCALE 3.0 /* m per unit of out[3..5]   */
#define GCVO_MLP_MAX_POINTS 65536
#define GCVO_MLP_MAX_PAIRS 65536

typedef struct {
    int n_pairs;                 /* B >= 1                                             */
    int n_points;                /* P >= 1 points per cloud fed to the network         */
    const float *tgt_xyz;        /* device float32 [n_tgt_rows][3]                     */
    long long n_tgt_rows;
    const long long *tgt_start;  /* host int64 [B], 0 <= start, start + count <= rows  */
    const long long *tgt_count;  /* host int64 [B], count >= 1                         */
    const float *src_xyz;        /* device float32 [n_src_rows][3]                     */
    long long n_src_rows;
    const long long *src_start;  /* host int64 [B]                                     */
    const long long *src_count;  /* host int64 [B]                                     */
    const int *tgt_idx;          /* device int32 [B][P], rows within the pair's cloud  */
    const int *src_idx;          /* device int32 [B][P]                                */
    const float *tgt_motion;     /* device float32 [B][12] or NULL (identity)          */
    const float *src_motion;     /* device float32 [B][12] or NULL (identity)          */
    float input_scale;           /* metres per network input unit, > 0                 */
} gcvo_mlp_batch;

/* Number of parameters (GCVO_MLP_N_PARAMS). */
long long gcvo_mlp_param_count(void);

/* Device workspace (bytes) for a batch of n_pairs pairs with n_points points per
 * cloud; 0 for sizes outside the limits. */
size_t gcvo_mlp_workspace_size(int n_pairs, int n_points);

/* Forward pass.  out6: device float32 [B][6] (the normalised twists), required.
 * T_out: device double [B][16], or NULL; when given, the predicted poses
 * exp(xi^) (FP64, row-major) are written there on the stream, ready to be the
 * start poses of gcvo_register_batch. */
int gcvo_mlp_forward(const gcvo_mlp_batch *batch, const uint16_t *w_bf16, float *out6, double *T_out,
                     void *ws, size_t ws_bytes, void *stream);

/* Forward pass, loss and its gradient with respect to the (bfloat16-valued)
 * parameters.  y6: device float32 [B][6] normalised label twists.  loss: device
 * float32 [1].  grad: device float32 [GCVO_MLP_N_PARAMS] (overwritten).
 * out6: device float32 [B][6] or NULL (receives the forward outputs). */
int gcvo_mlp_loss_grad(const gcvo_mlp_batch *batch, const uint16_t *w_bf16, const float *y6, float *out6,
                       float *loss, float *grad, void *ws, size_t ws_bytes, void *stream);

/* One Adam step (Kingma and Ba, bias-corrected moments) on n device float32
 * master weights w with moments m, v and gradient grad; step >= 1 is the
 * 1-based step count.  Rewrites w_bf16 (device, n values) from the new w. */
int gcvo_mlp_adam(float *w, uint16_t *w_bf16, float *m, float *v, const float *grad, long long n, int step,
                  float lr, float beta1, float beta2, float eps, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GCVO_MLP_H */
