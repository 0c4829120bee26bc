/*
 * vrsplat -- C-ABI of an MI355X (gfx950) foveated hybrid radiance-field
 * renderer after VR-Splatting (Franke, Fink & Stamminger, PACMCGIT 8(1),
 * 2025): a peripheral 3D Gaussian splatting pass over the full image
 * (Sec. 3.2, Eq. 1), a foveal neural-point splat into an image pyramid with
 * depth-occlusion culling (Sec. 3.3, Sec. 4 "Inference"), a small gated
 * convolutional decoder with the periphery crop injected (Sec. 3.3), and the
 * edge-aware combination (Sec. 3.4, Eqs. 2-5), each with a backward entry
 * for end-to-end fitting (Sec. 3.5).
 *
 * Conventions shared by every entry point
 *  - Every array argument is a DEVICE pointer owned by the caller; the
 *    library never allocates or frees device memory.  Scratch memory is a
 *    caller-provided workspace whose size a *_workspace_size query returns.
 *  - Small descriptors (vrs_view, vrs_crop, option structs) are HOST
 *    pointers, read during the call; they are copied into kernel arguments.
 *  - All work is enqueued asynchronously on `stream` (a hipStream_t; NULL is
 *    the default stream).  Nothing synchronises the host, so a sequence of
 *    calls can be captured into a HIP graph.
 *  - Argument errors are detected on the host and returned as VRS_EINVAL
 *    before anything is launched.  Launch failures return VRS_EHIP.
 *  - Data-dependent overflow (more tile pairs or point fragments than the
 *    workspace was sized for) is detected on the device: the kernels write
 *    VRS_ECAPACITY into *dev_status (an int32 in device memory that the
 *    caller zeroes) and the outputs of that call are undefined.
 *  - Backward entries ACCUMULATE (+=) into gradient arrays; the caller zeroes
 *    them.  A backward call needs the workspace of its forward call intact.
 *  - Layouts: primitives are structure-of-arrays planes ([attr][n]); full
 *    frames are planar [view][channel][H][W]; pyramids are NHWC float32
 *    packed [crop][layer][y][x][C]; foveal images are planar
 *    [crop][3][S][S] packed back to back.  Pixel (i, j) has its centre at
 *    (i + 0.5, j + 0.5).  All views of one call share width and height.
 *  - Numerics: rasterisation runs in float32.  The integer decisions
 *    (culling, pixel and tile rectangles, depth keys, pyramid layer and
 *    target pixels) follow the single-precision operation order documented
 *    at each entry, with IEEE-rounded + - * / sqrt and no contraction.
 */
#ifndef VRSPLAT_H
#define VRSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VRS_OK = 0,
  VRS_EINVAL = 1,        /* bad argument (host-side check, nothing launched) */
  VRS_ECAPACITY = 2,     /* workspace capacity exceeded (device-side, in dev_status) */
  VRS_EHIP = 3,          /* HIP runtime error */
  VRS_EUNSUPPORTED = 4,  /* valid but unsupported configuration */
  VRS_ETIMEOUT = 5       /* a device-side bounded wait expired (dev_status) */
} vrs_status;

enum { VRS_MAX_VIEWS = 8, VRS_MAX_CROPS = 32, VRS_MAX_LEVELS = 8 };
enum { VRS_F32 = 0, VRS_BF16 = 1 };                   /* decoder arithmetic */
enum { VRS_BLEND_LINEAR = 0, VRS_BLEND_PAPER = 1 };   /* combination mask   */

/* Pinhole view.  rot is the world-to-camera rotation (row-major), trans the
 * world-to-camera translation: x_cam = rot * x_world + trans.  The camera
 * looks along +z; pixel = (fx x/z + cx, fy y/z + cy).  Geometry closer than
 * znear is culled. */
typedef struct {
  float fx, fy, cx, cy;
  float rot[9];
  float trans[3];
  float znear;
  int32_t width, height;
} vrs_view;

/* Foveal crop: the sub-frustum of view `view` (Sec. 3.3, Fig. 5) covering
 * pixels [x0, x0+size) x [y0, y0+size) of that view, i.e. the same focal
 * lengths with the principal point shifted by (-x0, -y0).  (gaze_x, gaze_y)
 * is the fixation point e in view pixels, the centre of the blend (Eq. 2).
 * size must be a multiple of 2^(levels-1). */
typedef struct {
  int32_t view, x0, y0, size;
  float gaze_x, gaze_y;
} vrs_crop;

/* Run-time placement of crop k, in DEVICE memory (an array [n_crops] of
 * these, 16 bytes each): origin (x0, y0) and fixation point (gaze_x,
 * gaze_y) in view pixels.  Entry points that take a `place` argument read
 * the crops' origins and gazes from it when it is not NULL (the host
 * vrs_crop then supplies only view and size, and its origin is not
 * checked), so a captured frame takes a new fixation by rewriting this
 * table -- the paper queries the eye tracker only after the periphery is
 * rendered (Sec. 4 "Inference").  Origins read from the table are clamped
 * into the view, [0, W - size] x [0, H - size]. */
typedef struct {
  int32_t x0, y0;
  float gaze_x, gaze_y;
} vrs_crop_place;

/* Blend order of the periphery.  PRIMITIVE: every pixel of a tile blends
 * its Gaussians in (float32 bits of the mean's view depth t.z, index) order.
 * PIXEL (Sec. 3.2, the per-pixel sorting that removes popping): pixel p
 * blends them in (key, index) order, the key being the camera depth z* of
 * the maximum of the Gaussian's 3D density along the ray through p's centre,
 *   z* = (d^T M mu) / (d^T M d),  d = ((p_x + 0.5 - cx)/fx, (p_y + 0.5 - cy)/fy, 1),
 * mu = rot*mean + trans, M = (rot Sigma rot^T)^-1, computed in float32 in
 * this order: Sigma^-1 by cofactors over ((s00 c00 + s01 c01) + s02 c02);
 * Q = rot Sigma^-1 and M_ij = Q_i . rot_j, b = M mu, each dot product as
 * ((a0 b0 + a1 b1) + a2 b2); u = ((x + 0.5) - cx)/fx, v likewise;
 * num = (b0 u + b1 v) + b2, den = ((m00 u + 2m01 v + 2m02) u + (m11 v +
 * 2m12) v) + m22 with 2m01 = 2*m01 etc.; key = num / den, compared by its
 * order-preserving bits (a non-positive or non-finite det(Sigma) gives the
 * key t.z).  Eq. 1 then accumulates that per-pixel depth; everything else
 * is as in PRIMITIVE order.  The backward entry supports PRIMITIVE only, and
 * the per-pixel work counts and replay positions are not kept in PIXEL
 * order; PIXEL order takes tiles of 8 or 16 (VRS_EUNSUPPORTED for 32). */
enum { VRS_ORDER_PRIMITIVE = 0, VRS_ORDER_PIXEL = 1 };

/* Rasteriser options.  Defaults: tile 16, radix_bits 8, alpha_clamp 0.99,
 * alpha_min 1/255, t_min 1e-4, lowpass 0.3, extent 3, bg 0.  tile and
 * radix_bits change only the work's organisation, never a result: they are
 * the autotuner's choices. */
typedef struct {
  int32_t tile;          /* screen tile edge: 8, 16 or 32 */
  int32_t radix_bits;    /* digit width of the radix sorts: 4, 6, 8 or 11 (0 = 8) */
  int32_t order;         /* VRS_ORDER_PRIMITIVE or VRS_ORDER_PIXEL, see below */
  float alpha_clamp;     /* alpha = min(alpha_clamp, opacity e^q) */
  float alpha_min;       /* contributions with alpha < alpha_min are skipped */
  float t_min;           /* a pixel stops before T would fall below t_min */
  float lowpass;         /* dilation added to the 2D covariance diagonal (px^2) */
  float extent;          /* splat half-extent in standard deviations */
  float bg[3];           /* background colour added as T_final * bg */
} vrs_raster_opts;

/* Decoder description: n_levels gated 3x3 conv levels, level 0 finest;
 * width[l] output channels of level l; in_ch pyramid channels (4).
 * dtype: VRS_F32 (float32 arithmetic) or VRS_BF16 (bfloat16 MFMA operands,
 * float32 accumulation).  The packed float32 weight buffer holds, for
 * l = 0..n_levels-1, W_l [2*width[l]][3][3][Cin_l] then b_l [2*width[l]],
 * then the RGB head W_o [3][width[0]] and b_o [3], with
 * Cin_l = in_ch + (l+1 < n_levels ? width[l+1] : 0) + (l == 0 ? 3 : 0).
 * Output channels 0..width-1 are the feature half f, width..2width-1 the
 * gate half g. */
typedef struct {
  int32_t n_levels;
  int32_t width[VRS_MAX_LEVELS];
  int32_t in_ch;
  int32_t dtype;
} vrs_decoder_desc;

const char* vrs_status_string(vrs_status s);
/* Library version string. */
const char* vrs_version(void);

/* ---------------------------------------------------------------- bake
 * Attribute baking (Sec. 4 "Inference": opacities and covariances are baked
 * into the primitives before rendering).  logscale [3][n], quat [4][n]
 * (w, x, y, z; normalised inside), logit [n] -> cov [6][n] =
 * (xx, xy, xz, yy, yz, zz) of R(q) diag(exp(2 logscale)) R(q)^T and
 * opacity [n] = sigmoid(logit). */
vrs_status vrs_bake_gaussians(const float* logscale, const float* quat, const float* logit,
                              int64_t n, float* cov, float* opacity, void* stream);
/* Adjoint of vrs_bake_gaussians: accumulates d_logscale [3][n], d_quat [4][n]
 * (with respect to the unnormalised input quaternion), d_logit [n] from
 * d_cov [6][n] and d_opacity [n] (d_opacity may be NULL). */
vrs_status vrs_bake_gaussians_backward(const float* logscale, const float* quat,
                                       const float* logit, int64_t n, const float* d_cov,
                                       const float* d_opacity, float* d_logscale, float* d_quat,
                                       float* d_logit, void* stream);

/* ------------------------------------------------------------ periphery
 * Peripheral 3D Gaussian splatting of n_views full images (Sec. 3.2).
 * Inputs: mean [3][n], cov [6][n] (baked), opacity [n], sh [K][3][n] with
 * K = (sh_degree+1)^2, sh_degree in 0..3.
 * Per view and Gaussian, in float32 (EWA projection):
 *   t = rot*mean + trans, evaluated ((r0 x + r1 y) + r2 z) + t; cull unless
 *   t.z > znear; Jacobian J of the pixel projection with x/z, y/z clamped
 *   to +-1.3 (W/2)/fx, +-1.3 (H/2)/fy; Sigma2D = (J R) Sigma (J R)^T +
 *   lowpass*I; cull unless det > 0; conic = Sigma2D^-1;
 *   r = ceil(extent * sqrt(lambda_max)); pixel rectangle
 *   [ceil(px - r - 0.5), floor(px + r - 0.5)] clipped to the image (cull if
 *   empty); colour = max(0, 0.5 + sum_k Y_k(dir) sh_k) with dir the unit
 *   vector from the camera centre to the mean (real SH, degree <= 3).
 * Binning: every Gaussian is listed in each tile its rectangle touches;
 * each tile list is ordered by (float32 bits of t.z, Gaussian index).
 * Blending per pixel (front to back, Eq. 1 for depth): a Gaussian
 * contributes only if the pixel lies in its rectangle;
 *   alpha = min(alpha_clamp, opacity exp(-0.5 d^T conic d)), skipped below
 *   alpha_min; the pixel stops before T(1 - alpha) < t_min;
 *   C += rgb alpha T, D += t.z alpha T, T *= 1 - alpha.
 * Outputs: rgb [V][3][H][W] = C + T bg, depth [V][H][W] = D (Eq. 1),
 * t_final [V][H][W] = T, n_contrib [V][H][W] = number of Gaussians blended.
 * Workspace: vrs_render_workspace_size(); max_pairs bounds the number of
 * (Gaussian, tile) pairs.  The workspace keeps the projected records, the
 * sorted tile lists and per-pixel stop positions for the backward call. */
size_t vrs_render_workspace_size(int64_t n, int n_views, const vrs_view* views,
                                 const vrs_raster_opts* opts, int64_t max_pairs);
vrs_status vrs_render_gaussians(const float* mean, const float* cov, const float* opacity,
                                const float* sh, int sh_degree, int64_t n,
                                const vrs_view* views, int n_views, const vrs_raster_opts* opts,
                                float* rgb, float* depth, float* t_final, int32_t* n_contrib,
                                void* ws, size_t ws_bytes, int64_t max_pairs,
                                int32_t* dev_status, void* stream);
/* Offsets (bytes into the workspace) of the render's intermediate results:
 * pair_count (uint32, device), tile lists as sorted Gaussian indices
 * (uint32 [max_pairs]), tile ranges (uint32 pairs [tiles][2] = begin, end
 * for tile index v*tiles_per_view + ty*tiles_x + tx), and per pixel the
 * number of Gaussians whose rectangle held the pixel and that the pixel
 * evaluated before it stopped (uint32 [V][H][W]: the blend's work count);
 * super_pair_count (uint32, device): the number of (super-tile, Gaussian)
 * pairs the binning sorted, a super-tile being 8 x 8 tiles;
 * exact_pass_count (uint32, device; PIXEL order only, else 0): the number of
 * pixels whose per-pixel order was resolved by the exact pass;
 * tile_words (uint64 [max_pairs]; PIXEL order only, else 0): at the first
 * min(length, 4096) positions of each tile range, the blend's reordering of
 * those records as (order-preserving bits of beta) << 32 | Gaussian index,
 * beta non-decreasing and at most every single-precision per-pixel key, at
 * the tile's pixels in its rectangle, of every record at that position or
 * later (later positions keep sorted_ids' order; other words unused).
 * For inspection, tests and throughput accounting. */
typedef struct {
  size_t pair_count, sorted_ids, tile_ranges, pixel_evals;
  int64_t tiles_x, tiles_y, tiles_total;
  size_t super_pair_count, exact_pass_count, tile_words;
} vrs_render_layout;
vrs_status vrs_render_workspace_layout(int64_t n, int n_views, const vrs_view* views,
                                       const vrs_raster_opts* opts, int64_t max_pairs,
                                       vrs_render_layout* out);
/* Adjoint of vrs_render_gaussians, replaying each pixel back to front from
 * its stored final transmittance.  d_rgb [V][3][H][W]; d_depth [V][H][W] or
 * NULL.  Accumulates d_mean [3][n], d_cov [6][n], d_opacity [n],
 * d_sh [K][3][n].  Forward inputs and outputs and the workspace must be
 * those of the matching forward call. */
vrs_status vrs_render_gaussians_backward(const float* mean, const float* cov,
                                         const float* opacity, const float* sh, int sh_degree,
                                         int64_t n, const vrs_view* views, int n_views,
                                         const vrs_raster_opts* opts, const float* t_final,
                                         const float* d_rgb, const float* d_depth, float* d_mean,
                                         float* d_cov, float* d_opacity, float* d_sh, void* ws,
                                         size_t ws_bytes, int64_t max_pairs, void* stream);

/* ------------------------------------------------------- tone mapping
 * The combined image mapped to a displayable range by a differentiable
 * camera model (Sec. 3.4, last paragraph, following ADOP; the paper does not
 * restate the model, so this is the library's reading).  Per view v, channel
 * c and pixel (x, y):
 *   t = ((x_in * e) * wb[c]) * vig,  e = 2^-ev (double precision, rounded),
 *   vig = ((k3 r2 + k2) r2 + k1) r2 + 1,  r2 = (dy dy + dx dx) inv_d2,
 *   dx = (x + 0.5) - cx, dy = (y + 0.5) - cy (the view's principal point),
 *   inv_d2 = 1 / ((W/2)^2 + (H/2)^2) rounded from double precision,
 *   s = clamp(t, 0, 1) (n - 1), i = min(floor(s), n - 2), f = s - i,
 *   out = R_i + f (R_{i+1} - R_i)
 * (single precision, in that order: t decides the segment and the clamp).
 * in, out: DEVICE float32 [V][3][H][W] (out may be in; every view of one
 * size).  params: DEVICE float32 [V][7 + n_resp] = ev, wb_r, wb_g, wb_b, k1,
 * k2, k3, R_0 .. R_{n_resp-1}.  2 <= n_resp <= 256.  VRS_EINVAL on null
 * pointers, mismatched view sizes or a bad n_resp. */
vrs_status vrs_tonemap(const float* in, const vrs_view* views, int n_views, const float* params,
                       int n_resp, float* out, void* stream);
/* Adjoint of vrs_tonemap for d_out [V][3][H][W]: d_in (may be NULL) is
 * WRITTEN; d_params [V][7 + n_resp] (may be NULL) is ACCUMULATED (sums over
 * the pixels reduced in a fixed order per parameter; the response samples'
 * sums are accumulated per block with LDS atomics, whose order may vary).
 * The clamp has zero derivative outside (0, 1).  ws: DEVICE workspace of
 * vrs_tonemap_workspace_size bytes, needed when d_params is given. */
size_t vrs_tonemap_workspace_size(const vrs_view* views, int n_views, int n_resp);
vrs_status vrs_tonemap_backward(const float* in, const vrs_view* views, int n_views,
                                const float* params, int n_resp, const float* d_out, float* d_in,
                                float* d_params, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------- training loss
 * D-SSIM of Eq. 6 (as in 3DGS): 1 - mean over every element of the SSIM
 * map of x against y, planes of [planes][H][W] float32 (DEVICE; e.g.
 * images x channels), with the 11 x 11 window of the 11-tap Gaussian of
 * sigma 1.5 normalised to sum 1 (outer product), zero padding outside each
 * plane, C1 = 0.01^2, C2 = 0.03^2.  Evaluated (single precision) in terms of
 * the difference e = x - y, whose blurred mean D and variance v_e make the
 * map's complement (b1 v_e + D^2 a2) / (b1 b2) free of cancellation where x
 * and y agree (a1, a2, b1, b2 the usual numerator and denominator factors,
 * b1 = a1 + D^2, b2 = a2 + v_e); the adjoint likewise.  loss: DEVICE
 * float32 [1] written.  ws: DEVICE workspace of
 * vrs_dssim_workspace_size bytes (the same size serves the adjoint). */
size_t vrs_dssim_workspace_size(int planes, int width, int height);
vrs_status vrs_dssim(const float* x, const float* y, int planes, int width, int height,
                     float* loss, void* ws, size_t ws_bytes, void* stream);
/* Adjoint with respect to x: d_x += d_loss * d(D-SSIM)/dx, d_loss a DEVICE
 * float32 scalar (NULL: 1). */
vrs_status vrs_dssim_backward(const float* x, const float* y, int planes, int width, int height,
                              const float* d_loss, float* d_x, void* ws, size_t ws_bytes,
                              void* stream);

/* The regulariser of Eq. 7: R = |mean F - mean crop(P)|, the means over
 * every pixel and channel of all crops together: F the decoder output
 * (DEVICE, packed [crop][3][S][S] as vrs_decode_fovea writes it), P the
 * periphery [V][3][H][W] (DEVICE), crop k covering view pixels
 * [x0, x0 + S) x [y0, y0 + S) (from `place` when not NULL, as for
 * vrs_composite_frame).  r: DEVICE float32 [2] = R, mean F - mean crop(P)
 * (sums in double precision, fixed order).  ws: DEVICE workspace of
 * vrs_regulariser_workspace_size() bytes. */
size_t vrs_regulariser_workspace_size(void);
vrs_status vrs_regulariser(const float* fovea_rgb, const float* rgb, int n_views, int width,
                           int height, const vrs_crop* crops, int n_crops,
                           const vrs_crop_place* place, float* r, void* ws, size_t ws_bytes,
                           void* stream);
/* Adjoint: with g = d_r sign(r[1]) / (3 sum S^2) (d_r a DEVICE scalar, NULL:
 * 1; sign(0) = 0), d_fovea += g and d_rgb -= g over every crop pixel (either
 * may be NULL; overlapping crops add up). */
vrs_status vrs_regulariser_backward(int n_views, int width, int height, const vrs_crop* crops,
                                    int n_crops, const vrs_crop_place* place, const float* r,
                                    const float* d_r, float* d_fovea, float* d_rgb,
                                    void* stream);

/* One Adam step (Kingma and Ba; the optimiser of Sec. 3.5) over n float32
 * parameters in DEVICE memory, in place: m = b1 m + (1 - b1) g,
 * v = b2 v + (1 - b2) g^2, p -= lr (m / (1 - b1^step)) /
 * (sqrt(v / (1 - b2^step)) + eps), step >= 1 (bias corrections from double
 * precision).  All four arrays 16-byte aligned; VRS_EINVAL otherwise. */
vrs_status vrs_adam_step(float* param, const float* grad, float* m, float* v, int64_t n,
                         int step, float lr, float beta1, float beta2, float eps, void* stream);

/* ------------------------------------------------------- scene layout
 * Spatial (Morton, Z-order) permutation of a point set, for storing a static
 * scene so that points adjacent in memory are adjacent in space (a load-time
 * storage step, not part of the per-frame path, whose results do not depend
 * on point order except for the order of exactly equal depths).  pos [3][n]
 * float32 (device); each coordinate is mapped to 10 bits over the set's
 * finite bounding box (non-finite coordinates to the last cell) and the
 * 30-bit interleaved x, y, z codes are sorted stably.  perm [n] (device,
 * caller-owned) receives point indices in that order.  ws: device workspace
 * of vrs_spatial_order_workspace_size(n) bytes (0 if n < 1 or n >= 2^31).
 * VRS_EINVAL on null pointers, a bad n or a short workspace. */
size_t vrs_spatial_order_workspace_size(int64_t n);
vrs_status vrs_spatial_order(const float* pos, int64_t n, uint32_t* perm, void* ws,
                             size_t ws_bytes, void* stream);
/* Allocation-free form of vrs_spatial_order, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same permutation, with the scratch
 * memory taken from a fixed device array inside the library (12.5 MB per
 * device, held until the process ends) instead of a workspace.  At most
 * VRS_NOALLOC_MAX_POINTS points per call (VRS_EINVAL beyond, or on null
 * pointers or n < 1).  Every call on one device shares that array, so calls
 * that overlap on a device (concurrent streams or threads) race; calls on one
 * stream are ordered and safe.  Allocates nothing, not even on its first call
 * on a device (which only looks up the array's device address). */
enum { VRS_NOALLOC_MAX_POINTS = 1 << 20 };
vrs_status vrs_spatial_order_noalloc(const float* pos, int64_t n, uint32_t* perm, void* stream);

/* ---------------------------------------------------------------- fovea
 * Neural-point splat into a multi-resolution pyramid for every crop
 * (Sec. 3.3 sub-frustum and depth culling; Sec. 4 "Inference": one count,
 * one scan and one fill over all layers and crops).  Inputs: pos [3][np],
 * radius [np] (world units), feat [np][channels] IEEE half bits, opacity
 * [np] or NULL (all ones).  Per point and view, in float32:
 *   t = rot*pos + trans; cull unless t.z > znear;
 *   p = (fx (t.x/t.z) + cx, fy (t.y/t.z) + cy);
 *   depth cull when depth/t_final are given ([V][H][W], the periphery's
 *   Eq. 1 depth and final transmittance): at pixel floor(p) inside the view,
 *   A = 1 - T_final; cull if A >= cov_min and t.z > slack * (D / A);
 *   s = ((2 fx) radius)/t.z; s <= 1: layer 0 only; else s = m 2^e (frexp),
 *   l0 = e - 1 (clamped to levels-1, single layer), second layer l0+1
 *   unless m == 0.5; layer weights 1 - f and f with f = log2(s) - l0;
 *   per crop and layer l: xl = ((p.x - x0) * 2^-l) - 0.5 (y likewise),
 *   bilinear weights to the four pixels around (xl, yl) inside the layer.
 * Per layer pixel the fragments are blended front to back in (float32 bits
 * of t.z, point id) order: alpha = w * opacity, F += feat alpha T,
 * T *= 1 - alpha.  The point id is point_ids[i] for stored point i when
 * point_ids (device, uint32 [np], distinct values) is given -- the caller's
 * own numbering, for a point set stored permuted (e.g. in spatial order) --
 * else i.  Output pyramid: packed [crop][layer][y][x][channels] float32.
 * channels must be 4; levels 1..8. */
size_t vrs_splat_workspace_size(int64_t np, int n_views, const vrs_view* views,
                                const vrs_crop* crops, int n_crops, int levels,
                                int64_t max_frags);
vrs_status vrs_splat_points(const float* pos, const float* radius, const uint16_t* feat,
                            const float* opacity, int64_t np, int channels, int levels,
                            const vrs_view* views, int n_views, const vrs_crop* crops,
                            int n_crops, const vrs_crop_place* place, const float* depth,
                            const float* t_final,
                            float cov_min, float slack, const uint32_t* point_ids,
                            float* pyramid, void* ws, size_t ws_bytes, int64_t max_frags,
                            int32_t* dev_status, void* stream);
/* Offsets of the splat's intermediate results: frag_count (uint32),
 * sorted layer-pixel keys (uint32 [max_frags]) and sorted point indices
 * (uint32 [max_frags]); layer pixel index = position in the packed pyramid. */
typedef struct {
  size_t frag_count, sorted_keys, sorted_ids;
  int64_t pyramid_pixels;
} vrs_splat_layout;
vrs_status vrs_splat_workspace_layout(int64_t np, int n_views, const vrs_view* views,
                                      const vrs_crop* crops, int n_crops, int levels,
                                      int64_t max_frags, vrs_splat_layout* out);
/* Adjoint of vrs_splat_points given d_pyramid (same layout as pyramid).
 * Accumulates d_feat [np][channels] (float32), d_pos [3][np], d_radius [np]
 * and d_opacity [np] (each may be NULL).  Culling is a non-differentiable
 * mask. */
vrs_status vrs_splat_points_backward(const float* pos, const float* radius,
                                     const uint16_t* feat, const float* opacity, int64_t np,
                                     int channels, int levels, const vrs_view* views,
                                     int n_views, const vrs_crop* crops, int n_crops,
                                     const vrs_crop_place* place, const float* d_pyramid,
                                     float* d_feat, float* d_pos, float* d_radius,
                                     float* d_opacity, void* ws, size_t ws_bytes,
                                     int64_t max_frags, void* stream);

/* Crop placement from fixation points (Sec. 3.3 sub-frustum around the
 * gaze; Sec. 4 "Inference"): gaze [n_crops][2] float32 (DEVICE, view pixels)
 * -> place [n_crops] (DEVICE), each crop of its host size centred on its
 * gaze with the integer origin x0 = clamp(rint(gaze_x - size/2), 0,
 * W - size) (rint rounds ties to even; y0 likewise), the gaze stored beside
 * it.  One small kernel on `stream`, capturable; view and size come from the
 * host crops (their origins are ignored).  VRS_EINVAL on null pointers, no
 * crops, a bad view or a crop larger than its view. */
vrs_status vrs_place_crops(const float* gaze, const vrs_view* views, int n_views,
                           const vrs_crop* crops, int n_crops, vrs_crop_place* place,
                           void* stream);

/* -------------------------------------------------------------- decoder
 * Small gated CNN turning each crop's pyramid into its foveal image F
 * (Sec. 3.3): h_top = G(X_top); h_l = G_l([X_l, up2(h_{l+1}), Pcrop if l=0]);
 * F = W_o h_0 + b_o, with G(x) = ELU(W_f*x + b_f) * sigmoid(W_g*x + b_g),
 * 3x3 kernels with zero padding, up2 = bilinear x2 (half-pixel centres,
 * edge clamp), Pcrop = the periphery rgb under the crop.  pyramid as written
 * by vrs_splat_points with `levels` layers (levels >= n_levels);
 * rgb_periphery [V][3][H][W]; weights packed float32 as described at
 * vrs_decoder_desc.  Output fovea_rgb packed [crop][3][S][S] float32.
 * The workspace holds the activations the backward call needs. */
size_t vrs_decoder_workspace_size(const vrs_decoder_desc* dd, const vrs_crop* crops,
                                  int n_crops);
vrs_status vrs_decode_fovea(const float* pyramid, int levels, const float* rgb_periphery,
                            const vrs_view* views, int n_views, const vrs_crop* crops,
                            int n_crops, const vrs_crop_place* place, const float* weights,
                            const vrs_decoder_desc* dd, float* fovea_rgb, void* ws,
                            size_t ws_bytes, void* stream);
/* Adjoint of vrs_decode_fovea: from d_fovea accumulates d_pyramid (may be
 * NULL), d_rgb_periphery (may be NULL) and d_weights (packed like weights,
 * may be NULL). */
vrs_status vrs_decode_fovea_backward(const float* pyramid, int levels,
                                     const float* rgb_periphery, const vrs_view* views,
                                     int n_views, const vrs_crop* crops, int n_crops,
                                     const vrs_crop_place* place, const float* weights,
                                     const vrs_decoder_desc* dd,
                                     const float* d_fovea, float* d_pyramid,
                                     float* d_rgb_periphery, float* d_weights, void* ws,
                                     size_t ws_bytes, void* stream);

/* ------------------------------------------------------------ combine
 * Combination of periphery P [V][3][H][W] and foveal crops F (Sec. 3.4).
 * For each crop in index order and each of its pixels, with r the distance
 * of the pixel centre to the crop's gaze point and d_f = size/2:
 *   VRS_BLEND_LINEAR: c = clamp((d_f - r)/ring, 0, 1);
 *   VRS_BLEND_PAPER:  r_n = clamp(r/d_f, 0, 1) (Eq. 2),
 *     f_p = (r_n - m)/(1 - m) (Eq. 3), f_e = |Sobel(mean_rgb(F))|/4 with
 *     replicated crop borders (Eq. 4), c = 1 - S2(clamp(f_p + gamma f_e, 0,
 *     1)), S2(x) = 6x^5 - 15x^4 + 10x^3 (Eq. 5);
 *   out = (1 - c) out + c F.  Elsewhere out = P.
 * out may be rgb_periphery itself (in place): then only the pixels under
 * the crops are read and written (the rest already hold P). */
vrs_status vrs_composite_frame(const float* rgb_periphery, int n_views, int width, int height,
                               const float* fovea_rgb, const vrs_crop* crops, int n_crops,
                               const vrs_crop_place* place, int mode, float ring, float m,
                               float gamma, float* out, void* stream);
/* Adjoint: from d_out accumulates d_rgb_periphery and d_fovea (either may be
 * NULL).  In VRS_BLEND_PAPER mode the edge term's dependence on F is
 * differentiated too. */
vrs_status vrs_composite_frame_backward(const float* rgb_periphery, int n_views, int width,
                                        int height, const float* fovea_rgb,
                                        const vrs_crop* crops, int n_crops,
                                        const vrs_crop_place* place, int mode,
                                        float ring, float m, float gamma, const float* d_out,
                                        float* d_rgb_periphery, float* d_fovea, void* stream);

/* --------------------------------------------------------------- loss
 * L1 photometric term of the fitting loss (Sec. 3.5, Eq. 6):
 * loss[0] = sum |pred - target| / n (written, float32 device scalar);
 * d_pred (may be NULL) accumulates scale * sign(pred - target) / n. */
vrs_status vrs_l1_loss(const float* pred, const float* target, int64_t n, float* loss,
                       float* d_pred, float scale, void* stream);

/* ---------------------------------------------------------- frame plan
 * Everything fixed across the frames of one scene and rig: views, crop
 * views and sizes, the pyramid depth, the rasteriser options with the
 * autotuned tile size and sort radix, the capacities (tile pairs, point
 * fragments) sized by counting passes, the decoder shape, the depth cull and
 * the combination.  The plan is host memory only (a copy of the descriptor
 * and of the views and crops arrays); it owns no device memory: the
 * workspaces are the caller's, of vrs_workspace_size bytes each.  It may be
 * shared by streams that each have their own workspaces and buffers. */
typedef struct {
  int32_t n_views;
  const vrs_view* views;        /* [n_views], all of one width and height */
  int64_t n_gaussians;
  int32_t sh_degree;
  int64_t n_points;
  int32_t point_channels;       /* 4 */
  int32_t levels;               /* pyramid layers */
  int32_t n_crops;              /* 0: the frame is the periphery alone */
  const vrs_crop* crops;        /* [n_crops]: view and size (origins are the
                                   frame's gaze placement, or these) */
  vrs_raster_opts raster;
  vrs_decoder_desc decoder;
  int32_t depth_cull;           /* cull points against the periphery (Sec. 3.3) */
  float cov_min, slack;         /* depth-cull rule, see vrs_splat_points */
  int32_t blend_mode;           /* VRS_BLEND_LINEAR or VRS_BLEND_PAPER */
  float ring, m, gamma;         /* combination (Sec. 3.4) */
  int64_t max_pairs, max_frags; /* capacities */
} vrs_plan_desc;
typedef struct vrs_plan vrs_plan;   /* opaque */
enum { VRS_WS_RENDER = 0, VRS_WS_SPLAT = 1, VRS_WS_DECODER = 2 };
/* VRS_EINVAL for any bad field (each stage's own checks), VRS_EUNSUPPORTED
 * for point_channels other than 4; *plan is NULL then. */
vrs_status vrs_plan_create(const vrs_plan_desc* desc, vrs_plan** plan);
void vrs_plan_destroy(vrs_plan* plan);
/* Workspace bytes of the frame's stage `which` (VRS_WS_*); 0 if invalid,
 * and for the foveal stages of a plan without crops. */
size_t vrs_workspace_size(const vrs_plan* plan, int which);
/* Copy of the plan's descriptor (its pointers refer to the plan's copies). */
vrs_status vrs_plan_describe(const vrs_plan* plan, vrs_plan_desc* out);

/* Stage timing on a plan: while set, vrs_render_frame records the caller's
 * HIP event start_event on its stream right before stage `stage`'s first
 * kernel and stop_event right after its last one (the caller reads the last
 * pair).  VRS_TRACE_OFF clears every stage.  Not to be changed while a
 * frame of this plan is being enqueued by another thread. */
enum {
  VRS_TRACE_OFF = 0, VRS_TRACE_GS_BLEND = 1, VRS_TRACE_GS_SORT = 2, VRS_TRACE_GS_PREPROCESS = 3,
  VRS_TRACE_GS_EMIT = 4, VRS_TRACE_SPLAT = 5, VRS_TRACE_DECODER = 6, VRS_TRACE_COMPOSITE = 7,
  VRS_TRACE_GS_DEPTH_SORT = 8
};
vrs_status vrs_plan_trace(vrs_plan* plan, int stage, void* start_event, void* stop_event);

/* Scene of a frame (DEVICE pointers, caller-owned): baked Gaussians as for
 * vrs_render_gaussians, points as for vrs_splat_points (point_opacity and
 * point_ids may be NULL), decoder weights packed as for vrs_decode_fovea. */
typedef struct {
  const float *mean, *cov, *opacity, *sh;
  const float *pos, *radius;
  const uint16_t* feat;
  const float* point_opacity;
  const uint32_t* point_ids;
  const float* decoder_weights;
} vrs_scene;

/* Per-frame buffers (DEVICE, caller-owned).  rgb receives the periphery and
 * then, in place, the combined frame; depth, t_final and n_contrib the
 * periphery's; pyramid and fovea_rgb the foveal stages' (packed as for
 * vrs_splat_points and vrs_decode_fovea); place the crops' placement when a
 * gaze is given; the three workspaces of vrs_workspace_size bytes; the
 * capacity status words (zeroed by the caller). */
typedef struct {
  float *rgb, *depth, *t_final;
  int32_t* n_contrib;
  float *pyramid, *fovea_rgb;
  vrs_crop_place* place;
  void *ws_render, *ws_splat, *ws_decoder;
  int32_t *status_render, *status_splat;
} vrs_frame_buffers;

/* One stereo foveated frame (Fig. 5): periphery of every view
 * (vrs_render_gaussians), then -- when gaze (DEVICE, float32 [n_crops][2],
 * view pixels) is given -- the crops placed on the device from the gaze read
 * at that point (vrs_place_crops; else the plan's crop origins), the point
 * splat culled against the periphery's depth (vrs_splat_points), the decoder
 * (vrs_decode_fovea) and the combination written into rgb
 * (vrs_composite_frame in place).  Results equal those of the stage entry
 * points called in that order.  flags: VRS_FRAME_STATS also keeps in the
 * render workspace the per-pixel last contributing positions and evaluation
 * counts (the adjoint's replay start and the blend's work count, see
 * vrs_render_workspace_layout); an inference frame leaves them out.
 * Asynchronous on `stream`, capturable into a HIP graph; a captured frame
 * follows new gaze-buffer contents without being captured again. */
enum { VRS_FRAME_STATS = 1 };
vrs_status vrs_render_frame(const vrs_plan* plan, const vrs_scene* scene, const float* gaze,
                            const vrs_frame_buffers* buffers, int32_t flags, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* VRSPLAT_H */
