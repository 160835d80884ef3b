/*
 * bf_gpa.h -- C ABI of the MI355X (gfx950) implementation of the
 * Gaussian-Polynomial Approximation (GPA) of the bilateral filter
 * (Chaudhury & Dabhade, "Fast and Provably Accurate Bilateral Filtering",
 * arXiv 1603.08109).
 *
 * What is computed
 * ----------------
 * The bilateral filter of Sec. 1, eq. (BF), with Gaussian range kernel
 * g(t) = exp(-t^2 / 2 sigma_r^2) (eq. range_kernel) and a box or Gaussian
 * spatial kernel on Omega = [-W, W]^2 (eqs. spatial_kernel1/2), is replaced
 * by eq. (GPA): the range kernel becomes the order-N Gaussian-polynomial of
 * eq. (GaussPolynomial) on intensities centred at `center` (Sec. 3,
 * eq. shift and Prop. centering).  Algorithm 2 (Sec. 3) evaluates it with
 * N+1 spatial filterings of the auxiliary images of eq. (intImg) and the
 * per-pixel ratio of eqs. (P), (Q), (PbyQ).  N is chosen from the requested
 * accuracy delta via Cor. (eps) and Prop. (LambW) unless given explicitly.
 *
 * Conventions
 * -----------
 * - Images are single-channel float32, row-major, `height` x `width`, with a
 *   row pitch given in ELEMENTS (>= width).  All image pointers are DEVICE
 *   pointers owned by the caller.  Input values are expected in
 *   [center - T, center + T] (by default [0, 255]); they are not range
 *   checked on the device.
 * - Pixels outside the image contribute nothing (the sums of eq. BF / GPA
 *   run over the part of Omega inside the image).
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   Every device call is asynchronous on that stream.
 * - Return codes: BF_OK (0) on success, a negative BF_E* code on error,
 *   a positive BF_W* code for a warning (the call still succeeded).
 *   bf_last_error_message() gives a thread-local description of the last
 *   non-zero code.  No C++ exception crosses this interface.
 * - Plans are immutable after bf_plan; a plan owns its device tables and
 *   its workspace, all allocated inside bf_plan.  bf_forward/bf_backward
 *   never allocate.  Calls that share one plan must not overlap in time
 *   (they share the plan's workspace).
 */
#ifndef BF_GPA_H
#define BF_GPA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BF_OK               0
#define BF_EINVAL          -1  /* bad argument */
#define BF_ENOMEM          -2  /* device or host allocation failed */
#define BF_EHIP            -3  /* a HIP runtime call failed */
#define BF_EUNSUPPORTED    -4  /* valid request outside what the build supports */
#define BF_WNOGUARANTEE     1  /* N below the order that guarantees +-delta */

/* spatial kernel (Sec. 1) */
#define BF_BOX    0   /* w = 1/|Omega| on [-W, W]^2, eq. spatial_kernel2 */
#define BF_GAUSS  1   /* w(i) = exp(-|i|^2 / 2 sigma_s^2), eq. spatial_kernel1 */
#define BF_GAUSS_REC 2 /* the recursive Gaussian Sec. 1 and Sec. 3 cite (Deriche's fit
                          of exp(-x^2/2) by two damped oscillations), unbounded support,
                          O(1) per pixel and order whatever sigma_s; W is ignored */

/* rule that turns delta into N */
#define BF_NRULE_LAMBERTW  0  /* Cor. eps + Prop. LambW, exact W0 (default) */
#define BF_NRULE_ALG1      1  /* Algorithm 1 as printed (sigma_r >= 70 -> N = 10) */
#define BF_NRULE_POISSON   2  /* smallest N whose Poisson tail (Prop. upperBound) <= eps */

/* flags */
#define BF_FLAG_FP32_ACCUM   1  /* accumulate P and Q in float32 instead of float64 */
#define BF_FLAG_GRAD         2  /* reserve the workspace bf_backward needs */
#define BF_FLAG_STREAMED     4  /* run the orders in blocks through device memory (the
                                   path taken automatically when W is too wide for the
                                   fused on-chip tiles); allocates about 64 bytes per pixel */
#define BF_FLAG_JOINT        8  /* cross (joint) filter: the range kernel acts on a guide
                                   image (bf_forward_joint); fused tiles only, no adjoint */
#define BF_FLAG_MIRROR      16  /* reflecting border (edge samples repeated) instead of zero
                                   extension; on the streamed path only for box W <= 96 and
                                   Gaussian W <= 124; with BF_FLAG_GRAD the adjoint runs on
                                   the image extended by W on each side (see bf_backward) */
#define BF_FLAG_TILE_VALU   32  /* force the fused tile on the vector ALUs (the planner's
                                   choice otherwise); BF_EUNSUPPORTED if W does not fit; not
                                   together with BF_FLAG_STREAMED (BF_EINVAL).  Other flag bits
                                   than the BF_FLAG_* here return BF_EINVAL. */
#define BF_FLAG_MFMA_FP32  128  /* streamed Gaussian passes: plain float32 matrix-core products
                                   instead of float32 emulated by three-way bfloat16 splits
                                   (six bf16 products per float32 product, about 2.3x fewer
                                   matrix-core cycles, same rounding level) */

/* forward engines (bf_plan_info.path) */
#define BF_PATH_TILE       0  /* one fused launch, tile on the vector ALUs */
#define BF_PATH_STREAMED   1  /* blocks of orders through device memory */
#define BF_PATH_RECURSIVE  3  /* BF_GAUSS_REC: row and column recursions per block of orders */
#define BF_PATH_VOLUME     4  /* bf_plan_volume: row, column and depth passes per block of orders */
#define BF_PATH_WIDE       5  /* T/sigma_r in (13, 37.4]: the streamed Gaussian with float64
                                 per-pixel states (forward only, zero or mirror border, W <= 120) */

typedef struct bf_params {
  int32_t kernel;    /* BF_BOX, BF_GAUSS or BF_GAUSS_REC */
  double  sigma_s;   /* Gaussian spatial scale (ignored for box) */
  int32_t W;         /* half-width of Omega; 0 with BF_GAUSS means ceil(3 sigma_s) */
  double  sigma_r;   /* range scale, eq. range_kernel */
  double  T;         /* half dynamic range: inputs in [center-T, center+T]; 0 -> 127.5 */
  double  center;    /* centring value t_c of eq. shift; NaN -> T */
  int32_t N;         /* > 0: explicit order; 0: derive from delta */
  double  delta;     /* requested max |f_BF - f_GPA|; 0 -> 1e-3 */
  int32_t n_rule;    /* BF_NRULE_* */
  int32_t height;    /* image size the plan serves */
  int32_t width;
  int32_t flags;     /* BF_FLAG_* */
} bf_params;

typedef struct bf_plan_info {
  int32_t N;                 /* order: N+1 spatial filterings */
  int32_t W;                 /* support half-width */
  double  w0;                /* normalised centre weight w(0) = 1 / sum_Omega w */
  double  eps;               /* kernel tolerance of Cor. eps */
  double  lambda;            /* T^2 / sigma_r^2 */
  double  kernel_bound;      /* Poisson tail at N, Prop. upperBound */
  double  guaranteed_delta;  /* 2 T bound / (w0 - bound), Prop. accuracy (inf if none) */
  int32_t tile_rows;         /* tile height the fused forward kernel uses; for the
                                box column strips of the streamed engine (bf_plan
                                only), the row-segment length of the plain forward */
  int32_t tile_cols;         /* tile width; for the box strips, output columns per strip */
  int64_t workspace_bytes;   /* device bytes owned by the plan */
  int32_t path;              /* BF_PATH_* the forward runs (bf_order: the one it would run) */
} bf_plan_info;

typedef struct bf_plan bf_plan_t;
typedef struct bf_batch bf_batch_t;

/* Host-only planning: fills `out` from `p` (N, W, w0, eps, bounds) without
 * touching the device.  Same rules as bf_plan.  Returns BF_OK,
 * BF_WNOGUARANTEE (explicit N below the bound, or the Algorithm-1 rule
 * sigma_r >= 70 -> N = 10), or BF_EINVAL / BF_EUNSUPPORTED. */
int bf_order(const bf_params* p, bf_plan_info* out);

/* Build a plan for one image size and parameter set: validates `p`,
 * derives W (Sec. 1: W = ceil(3 sigma_s) for the Gaussian), w0, eps
 * (Cor. eps) and N (Prop. LambW, or as chosen by n_rule), builds the
 * float64 recursion tables and uploads them, allocates the workspace
 * (the backward's when BF_FLAG_GRAD is set).  *out receives the plan
 * (owned by the caller; free with bf_destroy).  Uses the current HIP device.
 * Range: with lambda = (T / sigma_r)^2, every path serves lambda <= 170
 * (e^{-x^2/2} a normal float32 for |x| <= T / sigma_r).  For 170 < lambda
 * <= 1400 (e.g. sigma_r >= 3.41 on [0, 255]) only the forward Gaussian
 * (W <= 120, zero or mirror border, no GRAD / JOINT / TILE_* / MFMA_FP32)
 * runs, on BF_PATH_WIDE; other requests there return BF_EUNSUPPORTED, as
 * does every lambda above 1400. */
int bf_plan(const bf_params* p, bf_plan_t** out);
int bf_plan_get_info(const bf_plan_t* plan, bf_plan_info* out);
int bf_destroy(bf_plan_t* plan);

/* A second plan with the same parameters and its own device workspace.  A
 * plan's parameters never change after bf_plan, but bf_forward and
 * bf_backward use its workspace (the adjoint's recompute buffer and
 * partial sums, the streamed paths' state), so calls that may overlap, e.g.
 * on two streams, need one plan each.  *out is owned by the caller (free
 * with bf_destroy); the clone lives on the current HIP device.  Errors as
 * for bf_plan. */
int bf_plan_clone_workspace(const bf_plan_t* plan, bf_plan_t** out);

/* Forward filter, Algorithm 2 (Sec. 3): one fused kernel launch, or, for
 * supports too wide for a tile's region to stay on chip (and with
 * BF_FLAG_STREAMED), the streamed sequence that filters blocks of orders
 * through the plan's device workspace.
 *   in      device, height x width float32, row pitch in_pitch (elements)
 *   out     device, height x width float32, row pitch out_pitch; must not
 *           alias `in`
 *   saved   NULL, or device buffer of 3*height*width float32 that receives
 *           per-pixel state for bf_backward (layout: three planes of
 *           height*width, dense pitch = width); must be NULL with
 *           BF_FLAG_MIRROR (BF_EUNSUPPORTED)
 * Errors: BF_EINVAL for NULL pointers or pitches < width; BF_EHIP if the
 * launch fails. */
int bf_forward(const bf_plan_t* plan, const float* in, int64_t in_pitch,
               float* out, int64_t out_pitch, float* saved, void* stream);

/* Allocation-free forward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same filter and the same fused-tile kernel as bf_plan +
 * bf_forward, without a plan: the parameters are normalised and N, W and the
 * engine chosen exactly as bf_plan does, and the constant tables that a plan
 * keeps in its own workspace go to one static device array of the library
 * instead (64 KiB per device, held until the process ends), written by small
 * kernels on `stream` whose arguments carry the values.  The call makes no
 * device allocation and frees nothing.
 *   p       as for bf_plan; BF_FLAG_GRAD, JOINT and STREAMED are
 *           refused (BF_EUNSUPPORTED); BF_FLAG_MIRROR, FP32_ACCUM and
 *           TILE_VALU are honoured
 *   in      device, height x width float32, row pitch in_pitch (elements)
 *   out     device, height x width float32, row pitch out_pitch; must not
 *           alias `in`
 * Limits: only parameters for which bf_plan picks the fused tile
 * (BF_PATH_TILE: small supports, or any support on small images) run here;
 * others return BF_EUNSUPPORTED.  Tables beyond the static array (16384
 * floats, an order N of about 2000) return BF_EINVAL.
 * Every call on one device shares the static array and leaves its tables
 * there: calls that overlap on one device (other streams or threads) race;
 * calls in order on one stream do not.
 * Returns BF_OK, BF_WNOGUARANTEE as bf_plan does, or BF_EINVAL / BF_EUNSUPPORTED
 * / BF_EHIP. */
int bf_forward_noalloc(const bf_params* p, const float* in, int64_t in_pitch, float* out,
                       int64_t out_pitch, void* stream);

/* Video and volume data, the extension named in Sec. 1 and Sec. 5: D slices
 * of height x width (p->height, p->width), the kernel w1 x w1 x w1 on the cube
 * [-W, W]^3 (box or truncated Gaussian, W <= 32), zero extension or, with
 * BF_FLAG_MIRROR, reflection about every face (edge samples repeated), Algorithm
 * 2 with three-axis filtering; N from the rule of bf_plan with the centre weight
 * (w1(0) / sum w1)^3.  Forward filter only: BF_FLAG_GRAD, JOINT and TILE_VALU
 * return BF_EUNSUPPORTED, as does BF_GAUSS_REC.  T/sigma_r above 13
 * (lambda in (170, 1400]) takes the Gaussian only, on the float64-state passes
 * of BF_PATH_WIDE (not with BF_FLAG_MFMA_FP32).
 * Allocates about 80 bytes per voxel.  *out is owned by the caller
 * (bf_destroy). */
int bf_plan_volume(const bf_params* p, int32_t depth, bf_plan_t** out);

/* Filter a volume planned by bf_plan_volume.
 *   in   device, depth slices of height x width float32, rows of pitch in_pitch
 *        elements, slice d starting at in + d * height * in_pitch (slices stacked)
 *   out  device, same layout with pitch out_pitch; must not alias `in`
 * Errors: BF_EINVAL for NULL pointers, pitches < width, aliasing, or a plan
 * not from bf_plan_volume; BF_EHIP if a launch fails. */
int bf_forward_volume(const bf_plan_t* plan, const float* in, int64_t in_pitch, float* out, int64_t out_pitch,
                      void* stream);

/* Cross (joint) bilateral filter, the extension named in Sec. 1 and Sec. 5:
 * out(i) = sum_j w(j) g(h(i-j) - h(i)) f(i-j) / sum_j w(j) g(h(i-j) - h(i)),
 * with the range kernel g replaced by phi_N on the centred guide h (T, center
 * and N refer to the guide's range).  The plan must have been built with
 * BF_FLAG_JOINT; it runs in one fused launch with two spatial filterings per
 * order (F_n of the guide, and F_n f), N orders.
 *   in      device, height x width float32 (f), pitch in_pitch
 *   guide   device, height x width float32 (h), pitch guide_pitch
 *   out     device, height x width float32, pitch out_pitch; aliases neither
 * Errors: BF_EINVAL for NULL pointers, pitches < width, aliasing, or a plan
 * without BF_FLAG_JOINT; BF_EHIP if the launch fails. */
int bf_forward_joint(const bf_plan_t* plan, const float* in, int64_t in_pitch, const float* guide,
                     int64_t guide_pitch, float* out, int64_t out_pitch, void* stream);

/* Data range of an image, for planning with the centre and half-range taken
 * from the data: writes {min, max} of the
 * height x width float32 image `in` (device, row pitch `pitch`) to the DEVICE
 * array minmax[2], skipping NaNs ({+inf, -inf} if there is no number).  Plan
 * with center = (min + max)/2 and T = (max - min)/2: every |f - center| <= T,
 * so the accuracy guarantee of Prop. (accuracy) still holds, and a range
 * narrower than [0, 255] lowers lambda = T^2/sigma_r^2 and with it N (and
 * admits a smaller sigma_r in float32).  Two kernel launches on `stream`, no
 * allocation.  Errors: BF_EINVAL for NULL pointers, sizes < 0 or a pitch <
 * width; BF_EHIP if a launch fails. */
int bf_image_range(const float* in, int64_t pitch, int32_t height, int32_t width, float* minmax,
                   void* stream);

/* Vector-Jacobian product of the forward filter (an extension: the paper
 * does not differentiate the filter).  With gbar = dL/d(out):
 *   grad_in     NULL or device float32 image (pitch gin_pitch): dL/d(in)
 *   grad_sigma  NULL or device double[2]: {dL/d sigma_r, dL/d sigma_s};
 *               dL/d sigma_s is NaN for the box kernel (W is discrete), and
 *               W and N are held fixed for the Gaussian one.
 *   saved       the buffer filled by bf_forward on the same input, or NULL:
 *               then the forward state is recomputed into the plan's
 *               workspace (requires BF_FLAG_GRAD at plan time).
 * The auxiliary images are recomputed, never stored (supports wider than the
 * fused adjoint tiles stream blocks of filtered adjoint images through the
 * plan's workspace).  Deterministic: the sigma gradients are reduced in a
 * fixed order.
 * With BF_FLAG_MIRROR the reflected filter equals the zero-border filter of
 * the image extended by W on each side by reflection, cropped back; the call
 * pads the image (and the output gradient, with zeros) into the plan's
 * workspace, runs the zero-border adjoint there (recomputing its state:
 * `saved` must be NULL, else BF_EUNSUPPORTED) and adds the gradient of every
 * extended sample onto the pixel it reflects.  Errors of the inner adjoint
 * are returned as they are. */
int bf_backward(const bf_plan_t* plan, const float* in, int64_t in_pitch,
                const float* grad_out, int64_t gout_pitch, const float* saved,
                float* grad_in, int64_t gin_pitch, double* grad_sigma, void* stream);

/* Batched forward over many images of uneven size, each with its own
 * parameters (an extension beyond the paper).  bf_batch_plan builds one plan
 * per image and a work list of tiles ordered by decreasing cost; the images
 * that fit the fused tiles run as ONE persistent kernel launch whose
 * workgroups claim tiles from a device counter.  Images that a single-image
 * plan would run on the streamed passes (Gaussian W >= 16, wide box supports
 * on large images) get such a plan of their own instead; their launches run
 * on four side streams of the batch, forked from the persistent launch's
 * stream and joined back, concurrently with it, and read their image
 * pointers from the batch's device copy of the call's parameters.  The whole
 * sequence (parameter copy, fork, persistent launch, side-stream launches,
 * join) is captured in a hipGraph on the first bf_batch_forward of each of two
 * staging slots, and every call is then ONE hipGraphLaunch on `stream`
 * (bf_batch_get_info counts them).  Image pointer arrays are host arrays of
 * `count` DEVICE pointers, copied at call time into pinned staging that the
 * graph copies to the device.  Per-image plan problems are reported by
 * bf_batch_status. */
int bf_batch_plan(int32_t count, const bf_params* per_image, bf_batch_t** out);
int bf_batch_forward(bf_batch_t* batch, const float* const* in, const int64_t* in_pitch,
                     float* const* out, const int64_t* out_pitch, void* stream);
/* Per-image N and status codes (host arrays of `count`, either may be NULL). */
int bf_batch_status(const bf_batch_t* batch, int32_t* per_image_status, int32_t* per_image_N);

/* How a batch runs (an extension beyond the paper; a pure query). */
typedef struct bf_batch_info {
  int32_t images_persistent;       /* images whose tiles the persistent launch claims */
  int32_t images_streamed;         /* images on a streamed plan of their own (side streams) */
  int64_t persistent_lds_bytes;    /* dynamic LDS per workgroup of the chosen persistent shape,
                                      sized for the persistent images only */
  int64_t workspace_bytes;         /* device bytes held by the batch and its images' plans */
  int64_t forward_graph_launches;  /* hipGraphLaunch calls bf_batch_forward has made */
  int64_t forward_direct_launches; /* launch sequences bf_batch_forward issued outside its graph */
  int64_t backward_graph_launches; /* hipGraphLaunch calls bf_batch_backward(_saved) has made */
  int64_t backward_direct_launches;/* adjoint calls issued launch by launch (images with BF_FLAG_MIRROR) */
} bf_batch_info;
int bf_batch_get_info(const bf_batch_t* batch, bf_batch_info* out);
/* Time the candidate launch shapes for this batch on `stream` (inputs as
 * for bf_batch_forward) and keep the fastest; the choice is cached in the
 * file named by BF_TUNE_CACHE (if set), keyed by the batch's shape summary.
 * *chosen receives the index of the chosen candidate (may be NULL). */
int bf_batch_tune(bf_batch_t* batch, const float* const* in, const int64_t* in_pitch,
                  float* const* out, const int64_t* out_pitch, void* stream, int32_t* chosen);
/* Batched vector-Jacobian product (an extension beyond the paper), for a
 * batch planned with BF_FLAG_GRAD on at least one image.  Per image i, as
 * bf_backward with saved = NULL: the forward state is recomputed by one
 * persistent batch launch; the adjoint tiles of all images whose support
 * fits the fused adjoint run as one more persistent launch over a
 * cost-ordered work list, and wider supports run the streamed adjoint image
 * by image.  Images on a streamed plan of their own (see bf_batch_plan) run
 * that plan's adjoint on the batch's side streams, concurrently, reading
 * their pointers from the batch's device copy of the call's parameters.
 * The whole sequence is captured in a hipGraph on the first call of each
 * combination of (saved given, grad_sigma given), and every call is then ONE
 * hipGraphLaunch on `stream` (bf_batch_get_info counts them).  Images with
 * BF_FLAG_MIRROR run bf_backward of a plan of their own (built at
 * bf_batch_plan, on the image extended by reflection), image by image,
 * recomputing their state; a batch holding one issues its adjoint launch by
 * launch.  Arguments are host arrays of `count` entries:
 *   in, in_pitch          the images and row pitches (device pointers)
 *   grad_out, gout_pitch  dL/d(out_i)
 *   grad_in, gin_pitch    NULL, or receives dL/d(in_i) (an entry may be NULL)
 *   grad_sigma            NULL or DEVICE double[2 * count]: per image
 *                         {dL/d sigma_r, dL/d sigma_s}, NaN for the box
 *                         kernel's sigma_s; entries of images whose plan
 *                         failed (bf_batch_status < 0) are left untouched.
 * Returns BF_EINVAL for NULL arrays, pitches < width, or a batch planned
 * without BF_FLAG_GRAD; BF_EHIP if a launch fails.  The batch's device
 * workspace is shared by its calls: calls on one batch are serialised
 * (each waits for the previous call's host-side staging). */
int bf_batch_backward(bf_batch_t* batch, const float* const* in, const int64_t* in_pitch,
                      const float* const* grad_out, const int64_t* gout_pitch, float* const* grad_in,
                      const int64_t* gin_pitch, double* grad_sigma, void* stream);
/* The batch pair with the forward state kept by the caller (as bf_forward /
 * bf_backward with `saved`), so the adjoint skips its recompute launch.
 * bf_batch_forward_saved runs the persistent forward directly (not from the
 * captured graph; images on their own streamed plans run those on the side
 * streams) and also writes, for image i, three planes of
 * height*width float32 (dense pitch = width) to the DEVICE buffer saved[i];
 * bf_batch_backward_saved takes the same arrays and reads them.  `saved` is
 * a host array of `count` device pointers; entries of images whose plan
 * failed are ignored, every other one must be non-NULL (images with
 * BF_FLAG_MIRROR recompute their state and leave theirs unread).  The planes belong to
 * the inputs the forward saw: passing other inputs gives the gradient at the
 * saved state.  Errors as for bf_batch_forward / bf_batch_backward, plus
 * BF_EINVAL for a NULL `saved` array or entry, or a batch planned without
 * BF_FLAG_GRAD. */
int bf_batch_forward_saved(bf_batch_t* batch, const float* const* in, const int64_t* in_pitch,
                           float* const* out, const int64_t* out_pitch, float* const* saved, void* stream);
int bf_batch_backward_saved(bf_batch_t* batch, const float* const* in, const int64_t* in_pitch,
                            const float* const* grad_out, const int64_t* gout_pitch, const float* const* saved,
                            float* const* grad_in, const int64_t* gin_pitch, double* grad_sigma, void* stream);
int bf_batch_destroy(bf_batch_t* batch);

const char* bf_status_string(int status);
const char* bf_last_error_message(void);
/* Library version string. */
const char* bf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BF_GPA_H */
