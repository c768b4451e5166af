/*
 * homog.h -- C ABI of libhomog, an MI355X (gfx950) implementation of the
 * minimal 4-point homography solvers of Cai et al., "Fast and Interpretable 2D
 * Homography Decomposition: Similarity-Kernel-Similarity and
 * Affine-Core-Affine Transformations" (arXiv 2402.18008), the RANSAC scoring
 * that consumes them and a differentiable 4-point-offset pipeline.
 *
 * Conventions shared by every call
 *  - Every array pointer is a DEVICE pointer owned by the caller unless stated
 *    otherwise; the library never frees or keeps one (a graph keeps the
 *    pointers it captured until hg_graph_destroy).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls are asynchronous on that stream unless stated otherwise.
 *  - Arguments are validated on the host before any HIP call; invalid ones
 *    return HG_EINVAL and launch nothing. A HIP failure returns HG_EHIP.
 *    hg_last_error() gives the detail of the last failing call of the calling
 *    thread. No C++ exception crosses this interface.
 *  - Degenerate inputs are not errors: they are reported through flags (solver)
 *    or by excluding the hypothesis (RANSAC).
 *  - Point order of a 4-point problem: M, N, P, Q. In the ACA decomposition
 *    (Sec. 4) M, N, P are the three anchor points and Q the fourth point; in
 *    SKS (Sec. 3) M, N are the two anchor points.
 *  - H is 3x3 row-major up to scale: h11 h12 h13 h21 h22 h23 h31 h32 h33.
 */
#ifndef HOMOG_H
#define HOMOG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status ------------------------------------------------------------ */
enum {
  HG_OK = 0,
  HG_EINVAL = -1,       /* invalid argument (host-side check)            */
  HG_EHIP = -2,         /* a HIP runtime call failed                     */
  HG_EWORKSPACE = -3,   /* workspace missing or smaller than required    */
  HG_EUNSUPPORTED = -4  /* valid request the library does not implement  */
};

/* Static text for a status code. */
const char *hg_status_str(int status);
/* Detail of the last failing call on this thread ("" if none). */
const char *hg_last_error(void);
/* Library version, major * 10000 + minor * 100 + patch. */
int hg_version(void);

/* ---- batched 4-point solver ---------------------------------------------
 * Solves n independent 4-point problems x2_i ~ H x1_i (i = M, N, P, Q): the
 * minimal homography problem of Sec. 2.1.
 *   method  HG_ACA: affine-core-affine, H = H_A2^-1 H_C H_A1 (Sec. 4,
 *                   eq. ACA, the division-free core of eqs. H_C_2 / C_11);
 *           HG_SKS: similarity-kernel-similarity, H = H_S2^-1 H_K H_S1
 *                   (Sec. 3, eq. HS).
 *   src, dst  8 planes each of n floats, plane k at offset k*ld:
 *             x_M y_M x_N y_N x_P y_P x_Q y_Q (source resp. target points).
 *   ld        plane stride in elements, ld >= n.
 *   H         9 planes of n floats at stride ld (output): the solution scaled
 *             by the power of two that brings max|h_ij| into [0.5, 1), then
 *             rounded to float (arithmetic inside is double precision).
 *   flags     n bytes (output, may be NULL): bit0 = near-degenerate (one of the
 *             8 triangles of either side has minimum height <= 1e-2 px);
 *             bit1 = non-finite input; bit2 = H was zero or non-finite and
 *             has been written as zeros.
 * Any alignment and any ld >= n are accepted (one quadruple per lane, 4-byte
 * accesses). n == 0 is a no-op. Errors: NULL pointer (other than flags), n < 0, ld < n,
 * unknown method -> HG_EINVAL.                                               */
enum { HG_ACA = 0, HG_SKS = 1 };
enum { HG_FLAG_NEAR_DEGENERATE = 1, HG_FLAG_NONFINITE_INPUT = 2, HG_FLAG_ZERO_H = 4 };
int hg_solve4(int method, const float *src, const float *dst, int64_t n, int64_t ld,
              float *H, uint8_t *flags, void *stream);

/* ---- simplified SK: one known pattern, many images ----------------------
 * The homography up to a similarity of Sec. 3.4 (eq. SK), for the case of a
 * known planar pattern seen in n images: Hbar = H_S2^-1 H_K = H H_S1^-1, where
 * H_S1 is the similarity of eq. 3_2_4 that takes the pattern's anchors M, N to
 * (-1, 0) and (1, 0). The pattern's constants are computed once per call on
 * the host, so each image costs the per-image steps of Table III (second row).
 *   obj     HOST array of 8 doubles: the pattern's x_M y_M x_N y_N x_P y_P
 *           x_Q y_Q in object coordinates (read during the call only).
 *   dst     8 planes of n floats at stride ld: the images of M, N, P, Q.
 *   H       9 planes of n floats at stride ld (output): Hbar, which maps the
 *           pattern's canonical frame to the image, scaled as in hg_solve4.
 *           The object-to-image homography is Hbar * H_S1 up to scale.
 *   flags   n bytes (output, may be NULL), bits as in hg_solve4; bit0 is set
 *           on every problem when a triangle of the pattern itself has height
 *           <= 1e-2 (in object units).
 *   frame   HOST array of 9 doubles (output, may be NULL): H_S1 row-major.
 * A pattern with three collinear points makes every Hbar non-finite: those
 * are written as zeros with bit2. n == 0 is a no-op (frame is still written).
 * Errors: NULL obj, a non-finite pattern coordinate, NULL dst or H when
 * n > 0, n < 0, ld < n -> HG_EINVAL.                                        */
int hg_solve_sk(const double *obj, const float *dst, int64_t n, int64_t ld, float *H,
                uint8_t *flags, double *frame, void *stream);

/* ---- three-point affine ---------------------------------------------------
 * The affine map through three correspondences M, N, P as H_A2^-1 H_A1
 * (Sec. 5.2, eq. AffineACA, 33 operations up to scale), normalised by its
 * third-row entry f_A1 (one division, six multiplications), in double
 * precision on float inputs.
 *   src, dst  6 planes each of n floats at stride ld: x_M y_M x_N y_N x_P y_P.
 *   A         6 planes of n floats at stride ld (output): a11 a12 a13 a21 a22
 *             a23 with (x', y') = A (x, y, 1).
 *   flags     n bytes (output, may be NULL): bit0 = the triangle M N P of
 *             either side has height <= 1e-2 px; bit1 = non-finite input;
 *             bit2 = A was not finite (source triangle of zero area) and has
 *             been written as zeros.
 * n == 0 is a no-op. Errors: NULL pointer (other than flags), n < 0, ld < n
 * -> HG_EINVAL.                                                              */
int hg_solve3_affine(const float *src, const float *dst, int64_t n, int64_t ld, float *A,
                     uint8_t *flags, void *stream);

/* Plain device copy of n floats (16 bytes per lane when both pointers are
 * 16-byte aligned, one float per lane for the rest; 512-thread workgroups,
 * non-temporal loads and stores). Not part of the method: it is the reference
 * for calibrating hardware byte counters and the plain-copy streaming rate.
 * n == 0 is a no-op; NULL pointer or n < 0 -> HG_EINVAL.                    */
int hg_stream_copy(const float *src, float *dst, int64_t n, void *stream);

/* Streaming ceiling of a solver's access pattern. Not part of the method: it
 * moves the bytes of one solver kernel without its arithmetic, with the same
 * launch shape (one element per lane, 512-thread workgroups, a grid covering
 * the batch once, non-temporal loads and stores). in: n_in float planes of n
 * elements, plane stride ld; out: n_out float planes, stride ld, where out
 * plane j = in[j mod n_in] + in[j + n_out] (second term only if
 * j + n_out < n_in); flags (optional, n bytes) = (in plane 0 < 0). Supported
 * shapes: 16 -> 9 (hg_solve4), 8 -> 9 (hg_solve_sk), 12 -> 6
 * (hg_solve3_affine). n == 0 is a no-op; other shapes, NULL in/out or
 * ld < n -> HG_EINVAL.                                                      */
int hg_stream_planes(const float *in, int32_t n_in, float *out, int32_t n_out, uint8_t *flags,
                     int64_t n, int64_t ld, void *stream);

/* ---- single-pair RANSAC --------------------------------------------------
 * Hypothesise and verify (RANSAC stage of the experiments): hypothesis j
 * draws 4 distinct correspondences with Philox4x32-10 (key = seed, counter =
 * (j, 0, 0, 0)) and Floyd's algorithm, solves ACA on them (as hg_solve4) and
 * counts the points with one-way transfer error ||pi(H x1) - x2|| <= thresh
 * (evaluated division-free in float). Degenerate samples (any flag bit) are
 * skipped. best = largest count, ties to the lowest j.
 *   corr        4 planes x1 y1 x2 y2 of n_pts floats at stride ld (>= n_pts).
 *   n_pts >= 4, n_hyp >= 1, thresh finite and > 0 with 1/thresh finite in float.
 *   best_H      9 floats (output); zeros if no hypothesis is valid.
 *   best_count, best_hyp  1 int32 each (output); best_hyp = -1 if none valid.
 *   inlier_mask n_pts bytes (output): 1 for inliers of best_H.
 *   hyp_counts  n_hyp int32 (output, may be NULL): per-hypothesis counts,
 *               0 for degenerate samples.
 *   ws          device workspace of at least hg_ransac_ws_bytes(...) bytes.
 * hg_ransac is the fused form (sampling, solving and scoring in one kernel,
 * then one kernel that reduces the per-workgroup winners and writes the
 * mask); hg_ransac_plain runs the same arithmetic as separate kernels (solve
 * all -> H buffer, score -> counts, argmax, mask) and returns identical
 * results.                                                                    */
size_t hg_ransac_ws_bytes(int32_t n_pts, int32_t n_hyp);
int hg_ransac(const float *corr, int32_t n_pts, int64_t ld, int32_t n_hyp, float thresh,
              uint64_t seed, float *best_H, int32_t *best_count, int32_t *best_hyp,
              uint8_t *inlier_mask, int32_t *hyp_counts, void *ws, size_t ws_bytes,
              void *stream);
int hg_ransac_plain(const float *corr, int32_t n_pts, int64_t ld, int32_t n_hyp, float thresh,
                    uint64_t seed, float *best_H, int32_t *best_count, int32_t *best_hyp,
                    uint8_t *inlier_mask, int32_t *hyp_counts, void *ws, size_t ws_bytes,
                    void *stream);

/* hg_ransac without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). Arguments and results are those of hg_ransac; the
 * workspace is the library's own static device array of 622592 bytes, one per
 * GPU, held until the process ends (its address is looked up on the first
 * call on each device). n_hyp <= 16384 (HG_EINVAL beyond). No allocation of
 * any kind happens in the call. Every call on a GPU uses that GPU's one
 * array: calls that overlap on one GPU (concurrent streams or threads) race
 * and must be serialised by the caller.                                       */
int hg_ransac_noalloc(const float *corr, int32_t n_pts, int64_t ld, int32_t n_hyp, float thresh,
                      uint64_t seed, float *best_H, int32_t *best_count, int32_t *best_hyp,
                      uint8_t *inlier_mask, int32_t *hyp_counts, void *stream);

/* ---- batched RANSAC over many uneven pairs --------------------------------
 * Pair p owns points [off[p], off[p+1]) of the concatenated planes (corr at
 * stride ld >= off[n_pairs]); every pair runs n_hyp hypotheses with Philox
 * counter (j, p, 0, 0). One persistent kernel drains a queue of (pair,
 * hypothesis block) items, largest pairs first, each folding its best key
 * into the pair's; a finish kernel then writes every pair's best outputs and
 * mask. Per pair, the arithmetic is that of hg_ransac (same
 * device functions) with Philox counter word 1 = p; results do not depend
 * on the tuning.
 *   off         n_pairs + 1 int64 (device); every pair needs >= 4 points.
 *   n_pairs * ceil(n_hyp / 16) <= 2^31 (the work queue's counter is 32-bit;
 *               HG_EINVAL beyond).
 *   best_H      n_pairs x 9 floats; best_count, best_hyp n_pairs int32;
 *   inlier_mask off[n_pairs] bytes; hyp_counts n_pairs x n_hyp or NULL.
 *   tune        launch shape, NULL = the cached autotuned or default choice.
 *   ws          >= hg_ransac_batched_ws_bytes(n_pairs, n_hyp) bytes.       */
typedef struct {
  int32_t pts_per_lane;    /* points held in registers per lane: 8 or 16    */
  int32_t hyps_per_block;  /* hypotheses per work item: 16, 32 or 64         */
  int32_t blocks_per_cu;   /* persistent blocks per compute unit: 1..8       */
  int32_t reserved;        /* 0                                              */
} hg_ransac_tuning;

size_t hg_ransac_batched_ws_bytes(int32_t n_pairs, int32_t n_hyp);
int hg_ransac_batched(const float *corr, int64_t ld, const int64_t *off, int32_t n_pairs,
                      int32_t n_hyp, float thresh, uint64_t seed, const hg_ransac_tuning *tune,
                      float *best_H, int32_t *best_count, int32_t *best_hyp,
                      uint8_t *inlier_mask, int32_t *hyp_counts, void *ws, size_t ws_bytes,
                      void *stream);

/* Adaptive termination (the RANSAC loop rule of the experiments): each pair
 * evaluates its hypotheses in rounds of 64 in index order and stops after the
 * first round at which, with eps = best count / N_p and m hypotheses
 * evaluated, (1 - eps^4)^m <= 1 - confidence (i.e. m >= log(1 - confidence) /
 * log(1 - eps^4)), or when m reaches n_hyp_max (the cap). The result is the
 * best hypothesis among the m evaluated; n_evaluated[p] = m. Rounds of all
 * pairs run in one persistent launch, queued by (2r + 1) / N_p (round r of a
 * pair of N_p points; large pairs' rounds spread through the queue) when
 * n_pairs^2 * rounds <= 2^27, else round-major. Rounds past a pair's stopping
 * point (or past the bound that the best count so far gives) are skipped, or
 * abandoned once a wave sees it (checked every 8 hypotheses); the finish
 * kernel applies the rule to the published round keys in order, so results
 * do not depend on order or timing. Same arguments as hg_ransac_batched
 * otherwise (no per-hypothesis counts); 0 < confidence < 1;
 * tune->hyps_per_block is ignored (64); with tune NULL the cached batched
 * choice is used with at most 4 blocks per compute unit.
 * ws >= hg_ransac_adaptive_ws_bytes(n_pairs, n_hyp_max) bytes.               */
size_t hg_ransac_adaptive_ws_bytes(int32_t n_pairs, int32_t n_hyp_max);
int hg_ransac_adaptive(const float *corr, int64_t ld, const int64_t *off, int32_t n_pairs,
                       int32_t n_hyp_max, float thresh, uint64_t seed, double confidence,
                       const hg_ransac_tuning *tune, float *best_H, int32_t *best_count,
                       int32_t *best_hyp, uint8_t *inlier_mask, int32_t *n_evaluated, void *ws,
                       size_t ws_bytes, void *stream);

/* ---- n-point refit on inliers (HO-SVD) ------------------------------------
 * Least-squares homography of each pair over the points whose mask byte is
 * non-zero (all points when mask is NULL), by the HO-SVD method that the paper
 * recommends for n points (Sec. 3.5): both sides normalised about their
 * centroids with RMS distance sqrt(2), the first two rows of H eliminated in
 * the least-squares sense, the last row h3 minimising ||A h|| / ||h3||
 * (smallest eigenvector of the 3 x 3 reduced Gram matrix),
 * all in double precision; then denormalised.
 *   corr, ld, off  as hg_ransac_batched (points [off[p], off[p+1]) of the
 *                  planes x1 y1 x2 y2); H maps (x1, y1) to (x2, y2).
 *   mask           off[n_pairs] bytes (e.g. hg_ransac_batched's inlier mask)
 *                  or NULL.
 *   H              n_pairs x 9 floats (output), scaled as hg_solve4.
 *   n_used         n_pairs int32 (output, may be NULL): points used.
 *   flags          n_pairs bytes (output, may be NULL): bit2 = fewer than 4
 *                  points or a singular normalised system; H written as 0.
 * One workgroup per pair (suited to sets of up to ~10^5 points).
 * Errors: n_pairs < 0, NULL corr/off/H with n_pairs > 0, ld < 1 ->
 * HG_EINVAL. n_pairs == 0 is a no-op.                                       */
int hg_refit_ho(const float *corr, int64_t ld, const int64_t *off, int32_t n_pairs,
                const uint8_t *mask, float *H, int32_t *n_used, uint8_t *flags, void *stream);

/* Times the tunings {8, 16} points per lane x {16, 32, 64} hypotheses per
 * block x {1, 2, 4, 5, 6} blocks per compute unit on the given problem (7 and
 * 8 blocks per unit do not fit in the registers at once); allocates temporary
 * outputs and synchronises the stream. Stores the fastest in *out and in the
 * process-wide cache used when tune == NULL; also written to the JSON file
 * named by HG_AUTOTUNE_CACHE if that variable is set. off_host mirrors off. */
int hg_ransac_autotune(const float *corr, int64_t ld, const int64_t *off,
                       const int64_t *off_host, int32_t n_pairs, int32_t n_hyp, float thresh,
                       uint64_t seed, void *ws, size_t ws_bytes, void *stream,
                       hg_ransac_tuning *out);

/* Captures hg_ransac_batched (queue reset + persistent kernel) with these
 * exact pointers and scalars into a HIP graph (allocates, synchronises).
 * hg_graph_launch replays it on `stream`; buffer contents may change between
 * launches, pointers may not. */
typedef struct hg_graph hg_graph;
int hg_ransac_batched_graph_create(const float *corr, int64_t ld, const int64_t *off,
                                   int32_t n_pairs, int32_t n_hyp, float thresh, uint64_t seed,
                                   const hg_ransac_tuning *tune, float *best_H,
                                   int32_t *best_count, int32_t *best_hyp, uint8_t *inlier_mask,
                                   int32_t *hyp_counts, void *ws, size_t ws_bytes,
                                   void *stream, hg_graph **out);
int hg_graph_launch(hg_graph *g, void *stream);
void hg_graph_destroy(hg_graph *g);

/* ---- differentiable 4-point-offset pipeline -------------------------------
 * Source: the rectangle with upper-left vertex (x0, y0), width w and aspect
 * ratio r = width / height (Sec. 5.3). offsets: B x 4 x 2 floats, corner
 * order TL, TR, BR, BL; target corners = source corners + offsets.
 * hg_aca_rect_fwd: H (B x 9 doubles) mapping the rectangle to the target
 *   quadrilateral (the rectangle case of ACA that Algorithm 1 tensorises,
 *   Sec. 5.3): ACA (Sec. 4) with the source points M N P Q at the corners TL,
 *   TR, BL, BR, at ACA's own scale (no rescaling, as hg_aca_fwd), double
 *   precision inside.
 * hg_aca_rect_bwd: grad_offsets (B x 8 floats) = (dH/d offsets)^T grad_H,
 *   grad_H B x 9 doubles (ACA's reverse mode in the target points).
 * Errors: B outside [0, 2^27], w or r not finite and > 0, non-finite x0/y0,
 * NULL pointer with B > 0 -> HG_EINVAL; B == 0 is a no-op.                   */
int hg_aca_rect_fwd(const float *offsets, int32_t B, float x0, float y0, float w, float r,
                    double *H, void *stream);
int hg_aca_rect_bwd(const float *offsets, const double *grad_H, int32_t B, float x0, float y0,
                    float w, float r, float *grad_offsets, void *stream);

/* General quadrilaterals (the tensorised general ACA of the deep-pipeline
 * experiments, Sec. 4): src, dst B x 8 floats, rows x_M y_M x_N y_N x_P y_P
 * x_Q y_Q (point order as hg_solve4).
 * hg_aca_fwd: H (B x 9 doubles) = H_A2^-1 H_C H_A1 at ACA's own scale (no
 *   rescaling), double precision inside; no degeneracy test.
 * hg_aca_bwd: grad_src, grad_dst (B x 8 floats each, either may be NULL) =
 *   (dH/dsrc)^T grad_H and (dH/ddst)^T grad_H, grad_H B x 9 doubles; the
 *   forward quantities are recomputed (nothing is stored between the calls).
 * Errors: B outside [0, 2^30], a NULL input, both outputs NULL -> HG_EINVAL;
 * B == 0 is a no-op.                                                        */
int hg_aca_fwd(const float *src, const float *dst, int32_t B, double *H, void *stream);
int hg_aca_bwd(const float *src, const float *dst, const double *grad_H, int32_t B,
               float *grad_src, float *grad_dst, void *stream);

/* Photometric loss of the warp by H (B x 9 doubles): for every pixel
 * p = (x, y) of an h x w output (x = column), sample img at pi(adj(H) p)
 * (adj(H) ~ H^-1) bilinearly, x0 = floor(x), taps outside the image reading
 * 0; loss[b] = mean_p |I_w(p) - tgt(p)| (float). img, tgt: B x h x w floats.
 * The sample position and the floor are double precision (the reciprocal to
 * ~2^-46 relative); bilinear weights, taps, residual and gradient terms are
 * float, with per-patch sums accumulated in double.
 * hg_warp_l1_bwd recomputes everything from H (nothing per pixel is stored)
 * and writes grad_H (B x 9 doubles) = grad_loss[b] * dloss[b]/dH_b, with
 * d|r|/dr = sign(r) (0 at 0) and the floor treated as constant.
 * Errors: B outside [0, 2^27], h or w outside [1, 32768], h w > 2^29, NULL
 * pointer with B > 0 -> HG_EINVAL; B == 0 is a no-op.                                             */
int hg_warp_l1_fwd(const double *H, const float *img, const float *tgt, int32_t B, int32_t h,
                   int32_t w, float *loss, void *stream);
int hg_warp_l1_bwd(const double *H, const float *img, const float *tgt, const float *grad_loss,
                   int32_t B, int32_t h, int32_t w, double *grad_H, void *stream);

/* Fused offsets -> loss and offsets -> gradient for h x w patches (h, w >= 2)
 * whose source rectangle has its corners at the pixel centres: the same
 * arithmetic as hg_aca_rect_fwd(offsets, 0, 0, w - 1, (w - 1) / (h - 1))
 * followed by hg_warp_l1_fwd, resp. hg_warp_l1_bwd and hg_aca_rect_bwd, in
 * one launch each (one workgroup per patch; ACA and its reverse mode run in
 * the workgroup's first lane, H stays on chip).
 *   hg_photometric_fwd: loss (B floats).
 *   hg_photometric_bwd: grad_offsets (B x 4 x 2 floats) = grad_loss[b] *
 *     dloss[b]/d offsets_b (recomputes the forward quantities).
 *   hg_photometric_fwd_grad: loss and grad_unit (B x 4 x 2 floats) =
 *     dloss[b]/d offsets_b in one pass over img and tgt (the loss is linear
 *     in grad_loss, so a later backward only scales grad_unit:
 *     hg_scale_grad(grad_unit, grad_loss, B, grad_offsets) writes
 *     grad_offsets[b] = grad_loss[b] * grad_unit[b], 8 floats per patch).
 * Errors: B outside [0, 2^27], h or w outside [2, 32768], h w > 2^29, NULL
 * pointer with B > 0 -> HG_EINVAL; B == 0 is a no-op.                                            */
int hg_photometric_fwd(const float *offsets, const float *img, const float *tgt, int32_t B,
                       int32_t h, int32_t w, float *loss, void *stream);
int hg_photometric_bwd(const float *offsets, const float *img, const float *tgt,
                       const float *grad_loss, int32_t B, int32_t h, int32_t w,
                       float *grad_offsets, void *stream);
int hg_photometric_fwd_grad(const float *offsets, const float *img, const float *tgt,
                            int32_t B, int32_t h, int32_t w, float *loss, float *grad_unit,
                            void *stream);
int hg_scale_grad(const float *grad_unit, const float *grad_loss, int32_t B,
                  float *grad_offsets, void *stream);

/* Iterative refinement of 4-point offsets: the structure of iterative deep
 * homography networks (six solver calls per forward pass in the deep-pipeline
 * experiments), with the network's predicted update replaced by a gradient
 * step on the photometric loss. Each of `iters` iterations is one launch of
 * hg_photometric_bwd's kernel with grad_loss = 1 that also applies
 *   offsets -= step * dL_b/d offsets_b      (float, per patch)
 * in place. offsets: B x 4 x 2 floats, TL TR BR BL; loss (B floats, may be
 * NULL) receives the loss at the final offsets (one more launch).
 * hg_refine launches on the stream; hg_refine_graph_create captures the same
 * sequence (with these pointers and scalars) for hg_graph_launch (allocates,
 * synchronises; needs B > 0).
 * Errors: B outside [0, 2^27], h or w outside [2, 32768], h w > 2^29, iters
 * outside [0, 1000], non-finite step, NULL img/tgt/offsets with B > 0 ->
 * HG_EINVAL. B == 0 is a no-op.                                                                   */
int hg_refine(const float *img, const float *tgt, int32_t B, int32_t h, int32_t w, int32_t iters,
              float step, float *offsets, float *loss, void *stream);
int hg_refine_graph_create(const float *img, const float *tgt, int32_t B, int32_t h, int32_t w,
                           int32_t iters, float step, float *offsets, float *loss, void *stream,
                           hg_graph **out);

/* Plain stored-intermediate form of the same pipeline (for comparison):
 * warp -> warped (B x h x w floats) ; L1 -> loss ; its backward ->
 * grad_warped (floats) ; warp backward from grad_warped -> grad_H (doubles).
 * Same conventions as above; the stored warp is rounded to float.           */
int hg_warp_store_fwd(const double *H, const float *img, int32_t B, int32_t h, int32_t w,
                      float *warped, void *stream);
int hg_l1_fwd(const float *warped, const float *tgt, int32_t B, int32_t h, int32_t w,
              float *loss, void *stream);
int hg_l1_bwd(const float *warped, const float *tgt, const float *grad_loss, int32_t B,
              int32_t h, int32_t w, float *grad_warped, void *stream);
int hg_warp_bwd_from_grad(const double *H, const float *img, const float *grad_warped, int32_t B,
                          int32_t h, int32_t w, double *grad_H, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HOMOG_H */
