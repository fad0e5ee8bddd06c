/*
 * dfr — per-pixel astronomical image reprojection on AMD Instinct MI355X
 * (gfx950).  C ABI of libdfr.so.
 *
 * The operation (paper "dfreproject: A Python package for astronomical
 * reprojection", section 3): every output pixel is taken through the target
 * WCS to the sky (shift, SIP A/B distortion, CD matrix, gnomonic
 * deprojection and spherical rotation, section 3.2.1), then through the
 * source WCS back to a source-pixel position (inverse rotation and gnomonic
 * projection, inverse CD, inverse SIP AP/BP, shift, section 3.2.2); the
 * source image is interpolated there (nearest, bilinear or bicubic,
 * section 3.1 step 3) together with a footprint (the interpolation of a
 * ones image), and the output is normalised by that footprint (section
 * 3.1, last paragraph).  The calls mirror the paper's single-call API
 * (source image + WCS, target WCS, output shape, interpolation order;
 * section 2).
 *
 * Conventions used by every call
 *   - x is the 0-based column (FITS NAXIS1, contiguous in memory), y the
 *     0-based row; integer coordinates are pixel centres.  Images are
 *     row-major float32, [rows][pitch] for sources and dense [out_h][out_w]
 *     for outputs.
 *   - CRPIX is FITS 1-based; CRVAL (RA, Dec) and CD are in degrees.
 *   - SIP polynomials (Shupe et al. 2005) are added: u' = u + A(u, v),
 *     v' = v + B(u, v), both evaluated at the undistorted (u, v); the
 *     inverse likewise with AP/BP.  The longitude of the pole is 180 deg
 *     (the TAN default that the paper's equations imply).
 *   - Interpolation reads zero outside the source: the value S and the
 *     footprint F sum only in-bounds taps.  Where F > 0 the output is S/F
 *     and the footprint is F; elsewhere (including directions on or behind
 *     the source tangent plane) the output is 0 (NaN with nan_outside) and
 *     the footprint 0.  Nearest rounds half to even.  Bicubic is Keys cubic
 *     convolution with parameter cubic_a (default -0.5).
 *   - Image pointers are DEVICE memory owned by the caller; WCS structs,
 *     coefficient arrays and option structs are HOST memory, read during
 *     the call only.  Work is enqueued on `stream` (a hipStream_t; NULL is
 *     the default stream) and is complete once that stream is synchronised.
 *   - Argument errors are detected on the host before any device work is
 *     enqueued; outputs are then left untouched.  On DFR_OK every output
 *     pixel is written, so outputs need no clearing by the caller.
 *   - The library keeps per-device workspaces (released by dfr_release) and
 *     a tile-shape cache; calls may come from several host threads.
 */
#ifndef DFR_H
#define DFR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DFR_MAX_SIP_ORDER 9
#define DFR_ABI_VERSION 3

typedef struct dfr_wcs {
  double crpix[2];       /* CRPIX1, CRPIX2 (1-based)                              */
  double crval[2];       /* CRVAL1 = RA, CRVAL2 = Dec, degrees; |Dec| <= 90       */
  double cd[4];          /* CD1_1, CD1_2, CD2_1, CD2_2, degrees per pixel         */
  int32_t a_order, b_order, ap_order, bp_order; /* 0 = polynomial absent       */
  /* (order+1)^2 doubles each, element [p*(order+1)+q] = coefficient of
   * u^p v^q; entries with p+q > order must be 0.  NULL when order is 0. */
  const double *a, *b, *ap, *bp;
} dfr_wcs;

typedef enum { DFR_NEAREST = 0, DFR_BILINEAR = 1, DFR_BICUBIC = 2 } dfr_interp;

typedef enum {
  DFR_OK = 0,
  DFR_E_NULL = 1,        /* a required pointer is NULL                              */
  DFR_E_SHAPE = 2,       /* negative size, pitch < width, or size overflow           */
  DFR_E_WCS = 3,         /* non-finite value, singular CD, |Dec| > 90, SIP term with
                            p+q > order, or SIP order outside [0, DFR_MAX_SIP_ORDER] */
  DFR_E_UNSUPPORTED = 4, /* unknown interpolation/precision, or a source WCS with
                            forward SIP A/B but no inverse AP/BP                     */
  DFR_E_DEVICE = 5,      /* a HIP runtime call or kernel launch failed               */
  DFR_E_NOMEM = 6,       /* device or host allocation failed                          */
  DFR_E_ARG = 7,         /* other invalid argument (option struct size, count, ...)  */
  DFR_E_LIMIT = 8        /* size beyond a fixed limit of the call (the static
                            scratch of dfr_reproject_noalloc)                        */
} dfr_status;

typedef enum {
  DFR_PREC_F32 = 0,      /* FP64 set-up per 32x32 cell, FP32 per pixel (default): a
                            certified cubic model of the cell's position map where
                            its bound holds (target without SIP), else the full
                            chain as FP32 offsets from an FP64 anchor              */
  DFR_PREC_F64 = 1,      /* every pixel in FP64 through the composed rotation        */
  DFR_PREC_TRIG_F64 = 2, /* every pixel in FP64 through explicit (RA, Dec) and the
                            trigonometric two-stage form of section 3.2              */
  DFR_PREC_F32_ANCHOR = 3 /* FP32 per pixel, always the full chain from anchors    */
} dfr_precision;

typedef struct dfr_options {
  uint32_t size;          /* sizeof(dfr_options); checked for ABI compatibility    */
  int32_t precision;      /* dfr_precision                                           */
  double cubic_a;         /* Keys parameter for bicubic; -0.5 by default             */
  int32_t nan_outside;    /* nonzero: uncovered output pixels are NaN, not 0          */
  int32_t tile;           /* 0 = choose (tuned cache or heuristic); else a tile id    */
  /* Nullable DEVICE buffer [out_h][out_w][2] of doubles: receives the source
   * position each pixel was interpolated at (exactly the value the kernel
   * used; NaN where the direction has no source position).  For tests.     */
  double *debug_positions;
  /* dfr_reproject_backward: request a grad_src that is bitwise reproducible
   * across runs and tile shapes.  Both 0 and 1 give that result: the source
   * adjoint is always summed exactly.  Every contribution g w / F is
   * rounded to a multiple of 2^-Q, 2^-Q = 2^-30 max|g| rounded down to a
   * power of two (a rounding of at most 2^-31 max|g| per contribution), and
   * the multiples are summed in 64-bit integers, so no order or grouping of
   * the additions matters; |g w / F| beyond 2^32 max|g| saturates.  The WCS gradient is reduced in a fixed order for a given
   * tile shape. */
  int32_t deterministic;
  int32_t reserved_;      /* must be 0 */
} dfr_options;

/* Fill `opt` with the defaults (FP32 path, a = -0.5, zeros outside, auto tile). */
void dfr_options_init(dfr_options *opt);

/* Reproject one source image onto the target grid (section 3; the paper's
 * single-call API of section 2).
 *   src        device, [src_h][src_pitch] float32 (may be NULL if src_h or
 *              src_w is 0: then every output pixel is uncovered)
 *   out        device, [out_h][out_w] float32 (may be NULL when out_h*out_w=0)
 *   footprint  device, [out_h][out_w] float32, nullable
 *   opt        host, nullable (defaults)                                      */
dfr_status dfr_reproject(const float *src, int32_t src_h, int32_t src_w, int64_t src_pitch,
                         const dfr_wcs *src_wcs, const dfr_wcs *tgt_wcs,
                         int32_t out_h, int32_t out_w, dfr_interp interp,
                         float *out, float *footprint, const dfr_options *opt,
                         void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as dfr_reproject, same arguments, same kernels and bit-identical
 * results, but it allocates nothing.  The per-cell model table that
 * dfr_reproject keeps in a per-stream workspace lives instead in a fixed
 * device array of DFR_NOALLOC_SCRATCH_BYTES (8 MiB) that every GPU the
 * library runs on holds until the process ends.
 *   Limit: with the default precision (DFR_PREC_F32) and a target without
 *   SIP the table takes 112 B per 32x32 output cell, so at most 74,898 cells
 *   (e.g. 8192 x 8192); a larger output returns DFR_E_LIMIT before any
 *   device work.  The other precisions use no scratch and have no limit.
 *   Sharing: every call on one GPU uses that GPU's one array.  Calls whose
 *   device work can overlap (different streams without ordering, several
 *   host threads) race on it and give wrong results; calls ordered on one
 *   stream are safe.  The array keeps the last call's table; nothing in it
 *   needs clearing (the model prepass writes every cell it reads).
 *   Errors: as dfr_reproject, DFR_E_LIMIT as above, DFR_E_DEVICE if the
 *   array's device address cannot be obtained. */
#define DFR_NOALLOC_SCRATCH_BYTES (8u << 20)
dfr_status dfr_reproject_noalloc(const float *src, int32_t src_h, int32_t src_w,
                                 int64_t src_pitch, const dfr_wcs *src_wcs,
                                 const dfr_wcs *tgt_wcs, int32_t out_h, int32_t out_w,
                                 dfr_interp interp, float *out, float *footprint,
                                 const dfr_options *opt, void *stream);

/* A reprojection geometry prepared once for many images of the same shape
 * and WCS pair (a time series on fixed pointing, repeated reprojection of
 * model images): the FP64 set-up of section 3.2 and the per-cell position
 * models are computed once, into device memory the plan owns (about 112 B
 * per 32x32 output cell), and each execute runs only the per-pixel kernel.
 * Opaque; not thread-safe to destroy while another thread executes it. */
typedef struct dfr_plan dfr_plan;

/* Create a plan on the current device; the model prepass is enqueued on
 * `stream` (execute on the same stream, or synchronise first).  The source
 * pointer is not needed yet: src_h and src_w fix the shape.  Errors as for
 * dfr_reproject; only the FP32 forms (DFR_PREC_F32, DFR_PREC_F32_ANCHOR)
 * have plans (DFR_E_UNSUPPORTED otherwise), debug positions are refused
 * (DFR_E_ARG), DFR_E_NOMEM when the model table cannot be allocated.
 *   plan  host, out: the new plan (NULL on error)                         */
dfr_status dfr_plan_create(int32_t src_h, int32_t src_w, const dfr_wcs *src_wcs,
                           const dfr_wcs *tgt_wcs, int32_t out_h, int32_t out_w,
                           dfr_interp interp, const dfr_options *opt, void *stream,
                           dfr_plan **plan);

/* Reproject one image with a plan: out and footprint exactly as
 * dfr_reproject with the plan's geometry and options gives them (bit for
 * bit).  src is device [src_h][src_pitch] float32 with the plan's shape;
 * out device [out_h][out_w]; footprint nullable.  DFR_E_ARG when called on
 * another device than the plan's. */
dfr_status dfr_plan_execute(const dfr_plan *plan, const float *src, int64_t src_pitch, float *out,
                            float *footprint, void *stream);

/* Free a plan (NULL is a no-op).  Call it once the work enqueued with the
 * plan has completed. */
dfr_status dfr_plan_destroy(dfr_plan *plan);

/* One sub-exposure of a batch (the paper's use case: many exposures stacked
 * onto one target grid, section 1). */
typedef struct dfr_frame {
  const float *src;       /* device, [h][pitch] float32                          */
  int32_t h, w;
  int64_t pitch;
  dfr_wcs wcs;
} dfr_frame;

/* Reproject n frames of uneven sizes onto one target grid in a single
 * persistent launch replayed from a captured HIP graph.  outs[i] and
 * footprints[i] are device [out_h][out_w] float32 (footprints or any entry
 * of it nullable).  The result of every frame is bit-identical to
 * dfr_reproject of that frame with the same options.  The graph is cached
 * per (n, out shape, interp, orders, tile) and replayed when they repeat. */
dfr_status dfr_reproject_batch(int32_t n, const dfr_frame *frames, const dfr_wcs *tgt_wcs,
                               int32_t out_h, int32_t out_w, dfr_interp interp,
                               float *const *outs, float *const *footprints,
                               const dfr_options *opt, void *stream);

/* The window of the target grid each frame of a batch can cover: boxes is
 * host [n][4] = {x0, y0, w, h} in target pixels (whole 32-pixel cells,
 * clipped to the output; w = h = 0 when no pixel can reach the frame).
 * Every pixel outside frame i's box is uncovered in dfr_reproject_batch
 * (the boxes come from the rigorous bounds of the model prepass, which this
 * runs on `stream` and waits for; with a target SIP there are no models and
 * every box is the whole grid).  Errors as for dfr_reproject_batch. */
dfr_status dfr_batch_boxes(int32_t n, const dfr_frame *frames, const dfr_wcs *tgt_wcs,
                           int32_t out_h, int32_t out_w, dfr_interp interp,
                           const dfr_options *opt, void *stream, int32_t *boxes);

/* dfr_reproject_batch into a window per frame: boxes is host [n][4] =
 * {x0, y0, w, h} inside the output (DFR_E_SHAPE otherwise); outs[i] and
 * footprints[i] (footprints or any entry nullable) are device [h][w]
 * float32 holding target pixels x0 .. x0+w-1, y0 .. y0+h-1 of frame i,
 * bit-identical to those pixels of dfr_reproject_batch; outs[i] may be NULL
 * when w * h = 0.  With the boxes of dfr_batch_boxes the dense per-frame
 * traffic of a stack shrinks to the pixels each frame can cover. */
dfr_status dfr_reproject_batch_cropped(int32_t n, const dfr_frame *frames,
                                       const dfr_wcs *tgt_wcs, int32_t out_h, int32_t out_w,
                                       dfr_interp interp, const int32_t *boxes,
                                       float *const *outs, float *const *footprints,
                                       const dfr_options *opt, void *stream);

/* Coadd (stack) n frames onto one target grid: the paper's motivating use of
 * reprojection, combining sub-exposures on a common grid (section 1), with
 * each frame weighted by its footprint (the per-pixel normalisation of
 * section 3.1).  With out_i and F_i what dfr_reproject gives for frame i,
 * per target pixel, over the frames with F_i > 0 there:
 *   sum_wf  device [out_h][out_w] float32: sum of out_i * F_i
 *   sum_f   device [out_h][out_w] float32: sum of F_i
 *   coadd   device [out_h][out_w] float32, nullable: sum_wf / sum_f where
 *           sum_f > 0, else 0 (NaN with opt->nan_outside)
 * The sums are FP32, accumulated in frame order (fused multiply-add), so
 * the result is deterministic and independent of the tile shape.  With
 * accumulate != 0 the sums start from the values already in sum_wf and
 * sum_f (a stack too large for one call is built by several; the result is
 * then bit-identical to one call over all frames in the same order).  The
 * three outputs must not overlap each other or any source.  n = 0 is an
 * empty stack.  opt->tile chooses the tile (0: a default); no per-frame
 * output is written, so the per-frame image traffic of the batch is gone:
 * each source is read about once and each target pixel written once. */
dfr_status dfr_coadd_batch(int32_t n, const dfr_frame *frames, const dfr_wcs *tgt_wcs,
                           int32_t out_h, int32_t out_w, dfr_interp interp, float *sum_wf,
                           float *sum_f, float *coadd, int32_t accumulate,
                           const dfr_options *opt, void *stream);

/* Number of source-WCS gradient entries dfr_reproject_backward writes:
 * crval(2), crpix(2), cd(4), ap[(ap_order+1)^2], bp[(bp_order+1)^2]. */
int64_t dfr_wcs_grad_size(const dfr_wcs *src_wcs);

/* Backward pass of dfr_reproject (FP32 path) for a loss L with
 * grad_out = dL/dout ([out_h][out_w] float32, device):
 *   grad_src  device [src_h][src_w] float32, nullable, overwritten:
 *             dL/dsrc = adjoint of the interpolation (scatter-add of w*g/F);
 *   grad_wcs  device float64 [dfr_wcs_grad_size(src_wcs)], nullable,
 *             overwritten: dL/d(source CRVAL, CRPIX, CD, AP, BP) in degrees
 *             and pixels; AP/BP entries with p+q > order are 0.
 * Pixels with F <= 0 contribute nothing.  Nearest gives zero WCS gradient. */
dfr_status dfr_reproject_backward(const float *src, int32_t src_h, int32_t src_w,
                                  int64_t src_pitch, const dfr_wcs *src_wcs,
                                  const dfr_wcs *tgt_wcs, int32_t out_h, int32_t out_w,
                                  dfr_interp interp, const float *grad_out, float *grad_src,
                                  double *grad_wcs, const dfr_options *opt, void *stream);

/* Squared-residual loss for WCS alignment: over n pixels,
 *   loss = sum_i m_i (out_i - ref_i)^2  and  grad_out_i = 2 m_i (out_i - ref_i),
 * with m_i = mask[i] (device float32, nullable = all ones).  loss is a device
 * double (overwritten), grad_out device float32 [n] (nullable). */
dfr_status dfr_sq_residual(const float *out, const float *ref, const float *mask, int64_t n,
                           double *loss, float *grad_out, void *stream);

/* Time the candidate tile shapes for this reprojection on `stream` (the
 * outputs are written, with identical values, by every candidate), store the
 * fastest in the tile cache (and in the JSON file named by the environment
 * variable DFR_TUNE_CACHE, if set) and return its id in *tile.  Tile shape
 * never changes results. */
dfr_status dfr_autotune(const float *src, int32_t src_h, int32_t src_w, int64_t src_pitch,
                        const dfr_wcs *src_wcs, const dfr_wcs *tgt_wcs, int32_t out_h,
                        int32_t out_w, dfr_interp interp, float *out, float *footprint,
                        const dfr_options *opt, void *stream, int32_t *tile);

/* As dfr_autotune, for a batch (times whole persistent launches). */
dfr_status dfr_autotune_batch(int32_t n, const dfr_frame *frames, const dfr_wcs *tgt_wcs,
                              int32_t out_h, int32_t out_w, dfr_interp interp,
                              float *const *outs, float *const *footprints,
                              const dfr_options *opt, void *stream, int32_t *tile);

/* Number of tile shapes and the (width, height) in output pixels of tile
 * id 1..dfr_tile_count(); returns DFR_E_ARG for an unknown id. */
int32_t dfr_tile_count(void);
dfr_status dfr_tile_shape(int32_t tile, int32_t *width, int32_t *height);

/* CD matrix from PC and CDELT (section 3.1): CD_ij = CDELT_i * PC_ij. */
void dfr_cd_from_pc_cdelt(const double pc[4], const double cdelt[2], double cd[4]);

/* Validate a WCS the way every entry point does (host only, no device). */
dfr_status dfr_check_wcs(const dfr_wcs *wcs, int32_t as_source);

/* The local position model of one 32x32 cell of output pixels that the
 * default FP32 path evaluates (section 3.2's two stages composed; host only,
 * no device work).  Cell (cx, cy) holds output pixels x in [32 cx, 32 cx+32),
 * y in [32 cy, 32 cy+32); a pixel's offsets from the cell centre are
 * a = x - (32 cx + 15.5), b = y - (32 cy + 15.5), and the model is
 *   x_src = base[0] + sum_k coef_x[k] a^i b^j   (y_src likewise)
 * with (i, j) for k = 0..9: (0,0) (0,1) (0,2) (0,3) (1,0) (1,1) (1,2) (2,0)
 * (2,1) (3,0); the coefficients are the FP32 values the kernels use.
 * `bound` receives a rigorous bound (px) on |model - exact position| over the
 * whole cell (1e30 where no model exists: a target with SIP, a projective
 * denominator that may vanish in the cell), `certified` 1 when the kernels
 * use the model: the part of the bound the cubic leaves out of the map is
 * <= 1e-6 px (the rest is the FP32 rounding of the coefficients, about
 * 6e-8 of their contributions, which the FP32 chain shares).  `tie` receives
 * the distance from a rounding tie within which nearest decides a pixel of
 * the cell from an FP64 position: twice the bound on |FP32 evaluation of the
 * model - exact position| (`bound` plus the FP32 rounding of Horner's rule,
 * gamma_6 sum_k |coef_k| 15.5^(i+j)), at least 1e-6 (0.5 where no model
 * exists).  All outputs are host pointers and may be NULL.  Errors: DFR_E_NULL (a WCS is NULL), DFR_E_WCS /
 * DFR_E_UNSUPPORTED as dfr_reproject, DFR_E_ARG (cx or cy negative). */
dfr_status dfr_cell_model(const dfr_wcs *src_wcs, const dfr_wcs *tgt_wcs, int32_t cx, int32_t cy,
                          double coef_x[10], double coef_y[10], int32_t base[2], double *bound,
                          int32_t *certified, double *tie);

/* Free cached per-device workspaces and graphs (the calling thread's device). */
dfr_status dfr_release(void);

/* A static, human-readable description of a status ("unknown status" for a
 * value outside dfr_status); never NULL, owned by the library. */
const char *dfr_strerror(dfr_status status);

/* DFR_ABI_VERSION of the built library (compare with the header's). */
int32_t dfr_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
