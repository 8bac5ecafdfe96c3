// Shared declarations of the gfx950 FB-LISA library: device-side parameter tables,
// the plan, and the launch functions each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <vector>

#include "../../include/fblisa.h"

namespace fbl {

// Views per kernel launch: the list travels by value in the kernel arguments, so a
// call needs no host-to-device copy.  Larger batches are split into several launches.
constexpr int kViewsPerLaunch = 256;

struct ViewList {
    int32_t v[kViewsPerLaunch];
};

// Per-(view, detector column) ray parameters, computed on the host in FP64.
// All rays of a column share their dominant axis a (x or y), their in-slice horizontal
// index coordinate xi(m) = xi0 + m*xi1 and their ray parameter tau(m) = t0 + m*t1 at
// slice m; the vertical index coordinate of row iv is eta = cz + tau*V[iv].  The ray
// length per slice is w = wa * sqrt(l2 + v2[iv]).
//
// Index coordinates reach a few thousand, where an FP32 value resolves only ~1e-4 of a
// voxel; the kernels therefore form positions in FP64 once per chunk of slices, split
// them into an integer voxel index and an FP32 offset, and step the offset in FP32
// inside the chunk (offsets stay below the chunk length, resolved to ~1e-6 voxel).
struct ColParam {
    double xi0, xi1;  // horizontal index coordinate on slice m (xi0 + m*xi1)
    double t0, t1;    // ray parameter on slice m (t0 + m*t1), 0 at source, 1 at pixel
    float wa;         // h_a / |q_a - s_a|
    float l2;         // (q_x - s_x)^2 + (q_y - s_y)^2, mm^2
    int32_t axis;     // 0: slices are x = const (xi is y), 1: slices are y = const (xi is x)
    int32_t pad;
};

// FP64 path-length factors of a column for the FP64 check kernels: w = wa * sqrt(l2 + v^2).
struct ColParam64 {
    double wa, l2;
};

// Per-view quantities used by the voxel-driven backprojection to find the detector
// columns near a voxel: the projection u(p) = sdd (p.e_u)/(sod - p.n) of a point p.
struct ViewParam {
    float c, s;         // cos, sin of the view angle
    int32_t axis_first; // dominant axis of column 0
    int32_t split;      // first column with the other axis (nu if none); at most one change
};

struct Geo {
    int nx, ny, nz;
    int nu, nv;
    float hx, hy, hz;
    float du, dv;
    float sod, sdd;
    double cz;       // (nz-1)/2: the vertical index coordinate of the source plane
    float cu, cv;    // (nu-1)/2, (nv-1)/2
    float dvz;       // dv / hz
    int64_t np;      // nu*nv
};

struct DeviceTables {
    const ColParam *col;    // [n_views][nu]
    const double *rowV;     // [nv] vertical index slope (iv-(nv-1)/2)*dv/hz
    const float *rowV2;     // [nv] (iv-(nv-1)/2)^2 dv^2, mm^2
    const ViewParam *view;  // [n_views]
};

}  // namespace fbl

struct fbl_plan {
    fbl_geometry geom;            // host copy; geom.angles points into angles_host
    double *angles_host;
    int device;
    int32_t vol_dtype, proj_dtype, max_batch;
    fbl::Geo geo;
    fbl::ColParam *d_col;
    fbl::ColParam64 *d_col64;     // FP64 path-length factors (FP64 check kernels only)
    double *d_rowV;
    float *d_rowV2;
    fbl::ViewParam *d_view;
    int *d_bp_order;              // backprojection tiles in launch order (most work first)
    double *d_partials;           // FP64 per-block partial sums
    int64_t n_partials;
    float *d_rw;                  // [max_batch][nv][nu] weighted residual for the backprojection
    void *d_xt;                   // [nz][nx][ny] y-fastest copy of the forward's input volume
    unsigned char *view_axis0;    // host, per view: 1 if some column marches x = const slices
    int fp_blocks_max;            // forward blocks per view at the finest split (partials sizing)
    int fp_line;                  // per-thread LDS line length of the forward
    int bp_pairs;                 // detector columns per slice the backprojection tile holds
    int bp_cand;                  // detector rows that can reach one voxel on a slice (the fallback tap loop)
    // launch timing (off unless fbl_timing_enable): event pairs around each launch
    struct TimedLaunch {
        int kernel;
        hipEvent_t start, stop;
    };
    bool timing_on;
    uint32_t timing_mask;         // bit k: launches of kernel FBL_K_k are bracketed
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
};

namespace fbl {

// Thread-local error message read by fbl_last_error: set_error stores a printf-style
// message and returns `code`; clear_error empties it and returns FBL_OK.
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int clear_error();
// Checks of the prox trial's buffers and scalars shared by its entry points: non-NULL,
// 16-byte aligned arrays (red_dev 8), xbar not aliasing x or g, alpha > 0, mu >= 0,
// 0 <= lo <= hi.  Returns FBL_OK or FBL_E_INVALID with the message set.
int check_step_buffers(const void *x, const float *g, double alpha, double mu, double lo, double hi, const void *xbar,
                       const double *red_dev);

// Launch functions (stream-ordered, no synchronisation).  Each returns hipSuccess or the
// launch error.
hipError_t launch_transpose(const fbl_plan *p, const void *x, hipStream_t st);
// parts: the slice march of each ray split over 1, 2 or 4 waves (forward_parts).
hipError_t launch_forward(const fbl_plan *p, const void *x, const ViewList &vl, int nb, int first,
                          const void *b, float *y, bool want_loss, int parts, hipStream_t st);
int forward_blocks_per_view(const Geo &g, int parts);
int forward_parts(const Geo &g, int B);   // parts for a call of B views (fills the chip)
int forward_rows_per_thread();
hipError_t launch_finalize_sum(double *partials, int64_t n, int ncomp, double scale, double *out,
                               hipStream_t st);
hipError_t launch_prescale(const fbl_plan *p, const float *r, const ViewList &vl, int nb, int first,
                           double grad_scale, float *rw, hipStream_t st);
hipError_t launch_backproject(const fbl_plan *p, const float *rw, const ViewList &vl, int nb, int first,
                              bool accumulate, float *g, hipStream_t st);
// The prox trial's launches (the one-pass kernel and, for many blocks, a second reduction
// level) fill the plan's partials; the final sum is taken over final_partials[0, 3 n_final).
hipError_t launch_step(const fbl_plan *p, const void *x, const float *g, double alpha, double mu, double lo,
                       double hi, bool stochastic, uint64_t key, void *xbar, double **final_partials,
                       int64_t *n_final, hipStream_t st);

// FP64 check instantiation of the projector pair (y and r point at the chunk's rows).
hipError_t launch_forward64(const fbl_plan *p, const double *x, const ViewList &vl, int nb, double *y,
                            hipStream_t st);
hipError_t launch_backproject64(const fbl_plan *p, const double *r, const ViewList &vl, int nb, double scale,
                                bool accumulate, double *g, hipStream_t st);

size_t mlp_workspace_bytes(int64_t n);
hipError_t launch_mlp_forward(const float *prm, const float *X, int64_t n, float *out, hipStream_t st);
hipError_t launch_mlp_loss_grad(const float *prm, const float *X, const float *t, int64_t n, float *grad,
                                double *loss, void *work, hipStream_t st);
hipError_t launch_mlp_adam(float *prm, const float *grad, float *m, float *v, int64_t step, double lr, double b1,
                           double b2, double eps, hipStream_t st);

// Prox trial on an FP32 master iterate that also writes the 16-bit copy (plan's vol_dtype).
hipError_t launch_step_mixed(const fbl_plan *p, const float *x, const float *g, double alpha, double mu, double lo,
                             double hi, float *xbar, void *xbar16, double **final_partials, int64_t *n_final,
                             hipStream_t st);

int64_t step_partials_needed(int64_t d);   // FP64 partials the prox trial of d voxels writes
int backproject_tile();   // in-slice tile extent of the backprojection (voxels)
int backproject_tile_z(); // its extent along z (voxels)

}  // namespace fbl
