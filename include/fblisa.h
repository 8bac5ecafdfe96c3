/*
 * fblisa.h -- C ABI of the MI355X (gfx950) FB-LISA hot-path library, libfblisa.so.
 *
 * The library computes, on one GPU, the three operations FB-LISA (arXiv 2605.12085)
 * spends its time in, for 3D circular cone-beam CT with data split into whole views:
 *
 *   fb_lisa_forward      A_N x over a mini-batch N of views, optionally fused with the
 *                        residual A_N x - b_N and the mini-batch objective
 *                        f_N(x) = n_theta/(2|N|) ||A_N x - b_N||^2      (eq. 2.5, Alg. 1 Step 2b)
 *   fb_lisa_backproject  the matched adjoint: grad f_N = n_theta/|N| A_N^T r  (eq. 2.5, Step 2b)
 *   fb_lisa_step         the prox-gradient trial xbar = prox_{alpha R}(x - alpha g) with
 *                        R = mu ||.||_1 + indicator[lo, hi], and the two inner products
 *                        of the sufficient-decrease test (2.3)           (Alg. 1 Step 2c)
 *
 * The discretised operator A (the paper uses an unspecified third-party projector)
 * is Joseph's ray-driven method with bilinear interpolation:
 *   - voxel (i,j,k) centre ((i-(nx-1)/2)hx, (j-(ny-1)/2)hy, (k-(nz-1)/2)hz) mm,
 *     volumes are C arrays [nz][ny][nx] (x fastest);
 *   - view v at angle theta_v: source SOD(cos, sin, 0), detector centre
 *     (SOD-SDD)(cos, sin, 0), detector axes e_u = (-sin, cos, 0), e_v = (0, 0, 1);
 *   - pixel (iu, iv) centre at detector centre + (iu-(nu-1)/2)du e_u + (iv-(nv-1)/2)dv e_v,
 *     projections are C arrays [view][nv][nu] (u fastest); one ray per pixel;
 *   - a ray marches the slices of its dominant index axis (largest |q-s|/h, ties to the
 *     lower axis x < y < z), samples each slice bilinearly (taps outside the volume are
 *     zero) and is scaled by the slice-to-slice path length h_a |q-s| / |q_a - s_a|.
 * Rays whose dominant axis would be z (cone angles beyond 45 degrees) are not supported:
 * plan creation rejects such geometries.
 *
 * Conventions for every call:
 *   - Device pointers are plain HIP device addresses owned by the caller; array buffers
 *     are contiguous in the layouts above and 16-byte aligned, scalar outputs (loss_dev,
 *     red_dev) 8-byte aligned.  Host pointers (geometry,
 *     angles, view lists) are read during the call only.
 *   - `stream` is a hipStream_t (NULL = default stream).  Compute calls only enqueue
 *     work: they never synchronise the device.  A plan serves one stream at a time.
 *   - Every function returns FBL_OK (0) or an FBL_E_* code and then sets a thread-local
 *     message readable with fbl_last_error().  Argument checks happen on the host before
 *     anything is enqueued: a call that fails a check launches nothing.  Faults inside
 *     kernels surface at the caller's next synchronisation.
 */
#ifndef FBLISA_H
#define FBLISA_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define FBL_API __attribute__((visibility("default")))
#else
#define FBL_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    FBL_OK = 0,
    FBL_E_INVALID = 1,   /* null pointer, bad size, misaligned buffer, bad scalar */
    FBL_E_GEOMETRY = 2,  /* geometry fails a precondition (see fbl_geometry_check) */
    FBL_E_RANGE = 3,     /* view id or batch size out of range */
    FBL_E_DTYPE = 4,     /* unsupported storage type */
    FBL_E_HIP = 5,       /* a HIP runtime call failed; the message holds its error string */
    FBL_E_NOMEM = 6      /* device or host allocation failed */
};

/* Storage types of the volume (x, xbar) and of the measured data b. */
enum {
    FBL_F32 = 0,
    FBL_BF16 = 1,
    FBL_F16 = 2
};

/* Scan geometry (millimetres, radians).  `angles` is a host array of n_views angles, or
 * NULL for the uniform set 2*pi*v/n_views (the paper's acquisitions are uniform over
 * [0, 2*pi)). */
typedef struct {
    int64_t nx, ny, nz;
    double hx, hy, hz;
    int64_t nu, nv;
    double du, dv;
    double sod, sdd;
    int64_t n_views;
    const double *angles;
} fbl_geometry;

typedef struct fbl_plan fbl_plan;

/* Host-only geometry validation; touches no device.  Checks: every count >= 1 (each at
 * most 2^24) and nx*ny*nz < 2^31, nu*nv <= 2^28; positive finite spacings; SOD > 0;
 * SDD > SOD; SOD and SDD - SOD both exceed the half-diagonal of the volume grown by two
 * voxels on every side (the volume lies strictly between source and detector); finite
 * angles; no ray with z as its dominant axis.  Returns FBL_OK or FBL_E_GEOMETRY
 * (FBL_E_INVALID for NULL). */
FBL_API int fbl_geometry_check(const fbl_geometry *g);

/* Create a plan on the current HIP device: validates the geometry, computes the per-view,
 * per-column ray parameters in FP64 on the host, and allocates the plan's device memory:
 * its tables (about 64 bytes per view and detector column), its FP64 reduction partials,
 * a [max_batch][nv][nu] FP32 scratch for the backprojection's weighted residual, and a
 * y-fastest copy [nz][nx][ny] of the volume in vol_dtype that the forward projection
 * refreshes for views marching x = const slices.  Nothing is allocated after this call,
 * so the three compute calls keep the argument lists of the method's operations.
 * max_batch in [1, n_views].  vol_dtype is FBL_F32, FBL_BF16 or
 * FBL_F16 (x and xbar); proj_dtype is FBL_F32, FBL_BF16 or FBL_F16 (b).  Storage types
 * only change what is read and written: every ray sum and the residual are formed in
 * FP32 and every reduction in FP64.  On failure *out is NULL.
 * The plan is released with fbl_plan_destroy (NULL is accepted). */
FBL_API int fbl_plan_create(const fbl_geometry *g, int32_t vol_dtype, int32_t proj_dtype, int32_t max_batch,
                    fbl_plan **out);
FBL_API void fbl_plan_destroy(fbl_plan *plan);

/* Forward projection of a mini-batch of views (eq. 2.5; Alg. 1 Steps 2b and 2c).
 *   x         device, [nz][ny][nx] in the plan's vol_dtype
 *   views     host, B view ids in [0, n_views) (duplicates allowed); B in [1, max_batch]
 *   b         device, full data [n_views][nv][nu] in proj_dtype, or NULL
 *   y         device FP32 [B][nv][nu]: y = A_views x, or the residual A_views x - b[views]
 *             when b is given (row k of y belongs to views[k])
 *   loss_dev  device, one double, or NULL: *loss_dev = loss_scale * sum(y^2), summed in
 *             FP64 in a fixed order (deterministic); pass loss_scale = n_theta/(2B) for
 *             f_N of (2.5).  Overwritten, not accumulated. */
FBL_API int fb_lisa_forward(fbl_plan *plan, const void *x, const int32_t *views, int32_t B, const void *b, float *y,
                    double *loss_dev, double loss_scale, void *stream);

/* Matched backprojection (eq. 2.5: grad f_N = n_theta/|N| A_N^T (A_N x - b_N)).
 *   r           device FP32 [B][nv][nu] (row k belongs to views[k])
 *   views, B    as for fb_lisa_forward
 *   grad_scale  scalar applied to the result (n_theta/B for the gradient of (2.5))
 *   g           device FP32 [nz][ny][nx], overwritten with grad_scale * A_views^T r.
 * Voxel-driven and free of atomics: the result does not depend on launch order. */
FBL_API int fb_lisa_backproject(fbl_plan *plan, const float *r, const int32_t *views, int32_t B, double grad_scale,
                        float *g, void *stream);

/* Prox-gradient trial of Alg. 1 Step 2c and the inner products of (2.3).
 *   x, g      device, [nz][ny][nx]; x in vol_dtype, g FP32
 *   alpha > 0, mu >= 0, 0 <= lo <= hi (hi may be +infinity)
 *   xbar      device, vol_dtype: xbar = min(max(x - alpha g - alpha mu, lo), hi), formed
 *             in FP64 and rounded once to the storage type (may not alias x or g)
 *   red_dev   device, three doubles: red[0] = <g, xbar - x>, red[1] = ||xbar - x||^2 with
 *             xbar the stored (rounded) value, red[2] = ||g||^2; FP64 sums in a fixed
 *             order (deterministic). */
FBL_API int fb_lisa_step(fbl_plan *plan, const void *x, const float *g, double alpha, double mu, double lo, double hi,
                 void *xbar, double *red_dev, void *stream);

/* fb_lisa_step on an FP32 master iterate with a 16-bit copy for the projector (the
 * precision form in which the volume the projector reads is stored in 16 bits while the
 * iterate itself keeps FP32): the plan's vol_dtype must be FBL_BF16 or FBL_F16.
 *   x, xbar   device FP32 [nz][ny][nx]: xbar = min(max(x - alpha g - alpha mu, lo), hi),
 *             formed in FP64 and rounded once to FP32
 *   xbar16    device, vol_dtype [nz][ny][nx]: xbar rounded to nearest (ties to even), the
 *             input of the next fb_lisa_forward of the trial point
 *   red_dev   as fb_lisa_step, on the FP32 values of x and xbar.
 * None of x, g, xbar, xbar16 may alias another.  FBL_E_DTYPE for an FP32 plan. */
FBL_API int fb_lisa_step_mixed(fbl_plan *plan, const float *x, const float *g, double alpha, double mu, double lo,
                               double hi, float *xbar, void *xbar16, double *red_dev, void *stream);

/* FP64 instantiation of the projector pair, for checks (finite differences, adjoint
 * identity, comparison with an FP64 reference): the same operator A as fb_lisa_forward and
 * fb_lisa_backproject with every position, weight and sum in FP64.  Plain kernels (one
 * thread per ray, the transpose scattered with FP64 atomic additions), far slower than
 * the FP32 path; not part of the method's loop.
 *   fb_lisa_forward_f64:     x device FP64 [nz][ny][nx]; y device FP64 [B][nv][nu] = A_views x
 *   fb_lisa_backproject_f64: r device FP64 [B][nv][nu]; g device FP64 [nz][ny][nx],
 *                            overwritten with grad_scale * A_views^T r (eq. 2.5)
 * views, B and errors as fb_lisa_forward. */
FBL_API int fb_lisa_forward_f64(fbl_plan *plan, const double *x, const int32_t *views, int32_t B, double *y,
                                void *stream);
FBL_API int fb_lisa_backproject_f64(fbl_plan *plan, const double *r, const int32_t *views, int32_t B,
                                    double grad_scale, double *g, void *stream);

/* Learned initial step of the line search (Alg. 1 Step 2c starts from a proposed step;
 * the backtracking on (2.3) still accepts or rejects every proposal).  The proposer is a
 * perceptron with FBL_MLP_IN inputs, two ReLU hidden layers of FBL_MLP_HIDDEN units and one
 * linear output, FP32.  Its parameters are one device FP32 vector of FBL_MLP_NPARAMS
 * values in the order W1[64][5], b1[64], W2[64][64], b2[64], w3[64], b3 (row-major,
 * y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3).  These calls need no plan; they are
 * stream-ordered and never synchronise.  Device arrays are 16-byte aligned. */
enum { FBL_MLP_IN = 5, FBL_MLP_HIDDEN = 64, FBL_MLP_NPARAMS = 64 * 5 + 64 + 64 * 64 + 64 + 64 + 1 };

/* Bytes of the caller-owned device workspace fbl_mlp_loss_grad needs for n samples. */
FBL_API size_t fbl_mlp_workspace_bytes(int64_t n);

/* out[i] = MLP(X[i]) for X device FP32 [n][FBL_MLP_IN], out device FP32 [n]; n >= 1. */
FBL_API int fbl_mlp_forward(const float *params, const float *X, int64_t n, float *out, void *stream);

/* Mean-squared training loss L = 1/(2n) sum_i (MLP(X[i]) - t[i])^2 and its gradient.
 *   t         device FP32 [n] targets
 *   grad      device FP32 [FBL_MLP_NPARAMS], overwritten with dL/dparams (FP64 sums over
 *             samples in a fixed order, rounded once)
 *   loss_dev  device double, or NULL: overwritten with 2 n L = sum_i e_i^2 (FP64)
 *   work      device, fbl_mlp_workspace_bytes(n) bytes, 256-byte aligned */
FBL_API int fbl_mlp_loss_grad(const float *params, const float *X, const float *t, int64_t n, float *grad,
                              double *loss_dev, void *work, void *stream);

/* One Adam step (Kingma and Ba) in FP32 on every parameter: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, params -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * step >= 1 counts the updates made so far including this one; m, v device FP32 state of
 * FBL_MLP_NPARAMS values (zero before the first step). */
FBL_API int fbl_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step, double lr, double beta1,
                         double beta2, double eps, void *stream);

/* Launch timing, for measurement.  While enabled, every kernel launch a compute call
 * makes is bracketed by a pair of HIP events on the call's stream; fbl_timing_read waits
 * for the recorded events, returns per kernel the summed duration (ms) and the number of
 * launches since timing was enabled or last read, and clears the record.  Disabled by
 * default; enabling clears any earlier record, disabling keeps it for a later read.  Event creation may allocate driver
 * resources, so a timing plan is not for callers that cannot allocate. */
enum {
    FBL_K_FORWARD = 0,      /* forward projection with residual and loss partials */
    FBL_K_TRANSPOSE = 1,    /* y-fastest copy of the volume for x = const slices */
    FBL_K_FINALIZE = 2,     /* FP64 reduction of per-block partials */
    FBL_K_PRESCALE = 3,     /* path-length weighting of the residual */
    FBL_K_BACKPROJECT = 4,  /* matched backprojection */
    FBL_K_STEP = 5,         /* prox trial with its partial inner products */
    FBL_K_COUNT = 6
};
FBL_API int fbl_timing_enable(fbl_plan *plan, int on);
/* Which kernels are bracketed while timing is enabled: bit k of mask selects FBL_K_k
 * (default: all).  Every bracketed launch adds two event records to its stream, so a
 * caller that times a whole run selects only the kernels it needs.  Bits at or above
 * FBL_K_COUNT are FBL_E_INVALID. */
FBL_API int fbl_timing_select(fbl_plan *plan, uint32_t mask);
FBL_API int fbl_timing_read(fbl_plan *plan, double ms[FBL_K_COUNT], int64_t launches[FBL_K_COUNT]);

/* fb_lisa_step with stochastic rounding of the trial point to the storage type (for 16-bit
 * iterates, so that updates below half a unit in the last place are not lost on average).
 * A value v between adjacent representable numbers a < v < a + q becomes a + q with
 * probability (v - a) / q: it goes up iff u < (v - a) / q, where u = (z >> 11) * 2^-53 and
 * z is output number i+1 of SplitMix64 (Steele, Lea and Flood, 2014) seeded with `key`,
 * i the voxel's linear index.  Representable values are unchanged.  The result depends
 * only on (x, g, alpha, mu, lo, hi, key): a caller replays it with the same key and
 * decorrelates trials with different keys.  Arguments and errors as fb_lisa_step. */
FBL_API int fb_lisa_step_sr(fbl_plan *plan, const void *x, const float *g, double alpha, double mu, double lo,
                            double hi, uint64_t key, void *xbar, double *red_dev, void *stream);

/* fb_lisa_step without a plan and without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same operation, rounding to nearest and outputs as fb_lisa_step on
 * a volume of n_voxels values in vol_dtype (x, xbar; g FP32), n_voxels in [1, 2^31).
 * Its scratch (FP64 partial sums, at most 2048 blocks x 3) is a 48 KiB array in the
 * library's device code, one per GPU, held until the process ends; its address is taken
 * on the first call on each device.  Calls on the same GPU share that array: calls that
 * overlap in time on one GPU (different streams, or other threads) race and must be
 * ordered by the caller.  Errors as fb_lisa_step; FBL_E_RANGE for n_voxels out of range. */
FBL_API int fb_lisa_step_noalloc(int64_t n_voxels, int32_t vol_dtype, const void *x, const float *g, double alpha,
                                 double mu, double lo, double hi, void *xbar, double *red_dev, void *stream);

/* Message of the last failed call on this thread ("" if none); valid until the next
 * call on the same thread. */
FBL_API const char *fbl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FBLISA_H */
