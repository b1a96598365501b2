/*
 * patop -- matrix-free photoacoustic forward operator A and its exact adjoint A^T
 * on MI355X (gfx950).  C ABI.
 *
 * The operator maps radial-basis-function voxel coefficients p0 (Sec. 2.4,
 * Eq. continuous_discretized_field) to the sampled signals s_hat of K finite
 * planar or cylindrically focused transducers (Eq. def_operatorS,
 * Eq. measurement_discrete):
 *
 *     s_hat_k = D_U( h * f_k )                 (Eq. discrete_conv, Alg. 1)
 *
 * where h is the discrete system kernel (Eq. def_bh) and f_k are geometric
 * coefficients on the fine time grid tau_m = t0 + m/(U fs), evaluated either
 *   - in closed form from the area of transducer surface swept by the shell
 *     [c tau_{m-1}, c tau_m) around each voxel (Eq. ui_area, Alg. 3, Alg. 4,
 *     Sec. 4.1 planar, Sec. 4.2 cylindrical), or
 *   - by a midpoint quadrature over surface points (Eq. def_f_point, Alg. 2).
 * The adjoint is the exact transpose (appendix on adjoint operators, Alg. 5-7).
 *
 * Conventions shared by every call:
 *   - Host-side geometry is SI (metres, seconds, hertz, metres/second), FP64.
 *   - Voxel i = ix + n[0]*(iy + n[1]*iz) sits at origin + (ix, iy, iz)*spacing.
 *   - Fine bin m (m in Z) is [tau_{m-1}, tau_m); output sample l = 1..L is
 *     stored at index l-1.  The signal is the untruncated sum over all bins;
 *     bins that cannot reach one of the L samples are skipped.
 *   - Device buffers are owned by the caller and passed as plain device
 *     pointers; coefficients are [batch][N] and signals [batch][K][L],
 *     contiguous, of type float (PAT_FP32) or double (PAT_FP64).
 *   - forward and adjoint OVERWRITE their output, run asynchronously on the
 *     given HIP stream (NULL = default stream) and never synchronise.
 *   - A context is not thread-safe; calls that overlap on one context race on
 *     its workspace.  Several contexts may coexist.
 *   - No exception crosses the ABI: every call returns a pat_status; the text
 *     of the last failure is available from pat_last_error.
 */
#ifndef PATOP_H
#define PATOP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PATOP_ABI_VERSION 4

typedef enum {
    PAT_OK = 0,
    PAT_E_ARG = 1,         /* NULL pointer, bad size, bad enum value            */
    PAT_E_FRAME = 2,       /* e1, e2 not orthonormal to 1e-9                    */
    PAT_E_SHAPE = 3,       /* non-positive size, theta_max outside (0, pi/2)    */
    PAT_E_SEPARATION = 4,  /* grid closer than kappa to a transducer (Assumption 1(iii)) */
    PAT_E_KERNEL = 5,      /* non-finite or empty system kernel                 */
    PAT_E_STATE = 6,       /* forward/adjoint before set_geometry               */
    PAT_E_DEVICE = 7,      /* a HIP call failed (text in pat_last_error)        */
    PAT_E_OOM = 8,         /* device allocation failed                          */
    PAT_E_UNSUPPORTED = 9  /* valid request the library does not support      */
} pat_status;

enum { PAT_PLANAR = 0, PAT_CYLINDER = 1 };
/* PAT_AREA_CLOSED: exact shell areas (Alg. 3 with Alg. 4).
 * PAT_AREA_QUADRATURE: surface points (Alg. 2, Eq. def_f_point).
 * PAT_AREA_TRAPEZOID: as PAT_AREA_CLOSED, but the cylinder's I_l by the chord of
 *   the level curve (Eq. trapezoid_Il, no elliptic integral); planar unchanged.
 * PAT_AREA_LUT: as PAT_AREA_CLOSED, but the cylinder's elliptic integrals read
 *   from tables of E(arcsin s, nu) and F(arcsin s, nu) on the 1000 x 1000
 *   power-law grid of Eq. LUT_sampling, interpolated bilinearly (Sec. 4.2, LUT
 *   paragraph; nu > 1 by Eq. reciprocal_modulus).  The context keeps the 16 MB
 *   FP64 table in device memory, built on the device by pat_set_geometry. */
enum { PAT_AREA_CLOSED = 0, PAT_AREA_QUADRATURE = 1, PAT_AREA_TRAPEZOID = 2, PAT_AREA_LUT = 3 };
enum { PAT_FP32 = 0, PAT_FP64 = 1 };
enum { PAT_PHI_CONE = 0, PAT_PHI_WENDLAND2 = 1 };
enum { PAT_EIR_GAUSS_COS = 0, PAT_EIR_SAMPLED = 1 };

/* One transducer.
 * planar (Sec. 4.1, Eq. plane_param): rectangle centred at c0 spanned by the
 *   orthonormal e1 (half-size half_w, the paper's L1) and e2 (half_h, L2).
 * cylinder (Sec. 4.2, Eq. cylinder_param): c0 is the centre of the focal
 *   line, e1 the cylinder axis (half-length half_len, L_z), the surface point at
 *   angle 0 is c0 + radius*e2, angular half-aperture theta_max in (0, pi/2).
 * The orientation sign of e1 x e2 does not matter. */
typedef struct {
    int32_t shape;         /* PAT_PLANAR or PAT_CYLINDER */
    int32_t reserved;
    double c0[3], e1[3], e2[3];
    double half_w, half_h;                 /* planar   */
    double radius, theta_max, half_len;    /* cylinder */
    double unused;
} pat_transducer;

typedef struct {
    int64_t n[3];
    double origin[3];      /* centre of voxel (0, 0, 0) */
    double spacing;
} pat_grid;

/* Discrete system kernel h[n], n = n_first .. n_first + len - 1, on the fine
 * grid of step 1/(U fs) (Eq. def_bh); kappa is the support radius of the radial
 * function, used for the separation check.  The array is copied. */
typedef struct {
    const double* h;
    int64_t n_first;
    int64_t len;
    double kappa;
} pat_kernel;

/* Electrical impulse response, support [0, T_e] (Assumption 1(ii)).
 * PAT_EIR_GAUSS_COS: e(t) = cos(2 pi fc (t - t_c)) exp(-(t - t_c)^2/(2 sigma_t^2))
 *   for 0 <= t <= t_e, 0 elsewhere.
 * PAT_EIR_SAMPLED: piecewise-linear interpolant of samples[j] at t = j*dt,
 *   j = 0 .. n_samples-1, 0 outside. */
typedef struct {
    int32_t kind;
    int32_t reserved;
    double fc, sigma_t, t_c, t_e;
    const double* samples;
    int64_t n_samples;
    double dt;
} pat_eir;

typedef struct {
    double sound_speed;    /* c, m/s                                   */
    double fs;             /* sampling rate F_s, Hz                    */
    double t0;             /* recording origin t_0 >= 0, s (Eq. def_operatorS) */
    int32_t L;             /* samples per transducer                   */
    int32_t U;             /* up-sampling factor of the fine grid      */
    int32_t area_mode;     /* PAT_AREA_CLOSED, _QUADRATURE, _TRAPEZOID or _LUT        */
    int32_t quad_n1;       /* quadrature cells along the first surface coordinate  */
    int32_t quad_n2;       /* quadrature cells along the second surface coordinate */
    int32_t precision;     /* PAT_FP32 or PAT_FP64 (element type of device buffers) */
    int32_t max_batch;     /* workspace is sized for this many volumes (>= 1)      */
    int32_t flags;         /* 0, or PAT_FLAG_TIME_TILES with bits 8-11 = log2 of the
                              tile width in area shells (5..9; 0 = automatic)      */
    int32_t area_step;     /* coarse area grid of Remark 1: the area of each shell of
                              area_step fine bins (bins (j-1) area_step + 1 .. j area_step)
                              is evaluated once and split evenly over its bins;
                              1 = every fine bin (exact); 1..U for the closed,
                              trapezoid and table modes, 1 for quadrature          */
    int32_t reserved;      /* must be 0                                            */
} pat_params;

/* pat_params.flags: the closed-form forward (area modes closed, trapezoid and
 * table; not quadrature, where it is refused with PAT_E_ARG) runs one
 * work-group per (transducer, tile of consecutive area shells) that owns its
 * tile of the fine-bin vector f_k (Eq. ui_area), instead of one per (4 x 4 x
 * 4 voxel cube, transducer chunk) adding into f with atomics.  Same result to
 * rounding (the order of the FP64 sums differs).  The work items are sorted by
 * an estimated cost at pat_set_geometry; pat_forward_sparse and the adjoint
 * are unchanged.  pat_query(9) returns the tile width (0 when off). */
#define PAT_FLAG_TIME_TILES 1

typedef struct pat_ctx pat_ctx;

/* Create a context on HIP device `device` (the device is made current during
 * the call).  *out receives the handle; PAT_E_DEVICE if the device is absent. */
pat_status pat_create(pat_ctx** out, int32_t device);

/* Validate the geometry, build the device tables (transducer frames in units of
 * the fine radial step c/(U fs), kernel polyphase table, per-bin scale
 * UF_s/(c tau_{m-1/2}) of Eq. ui_area, quadrature points) and upload them.
 * Allocates the context's workspace for params->max_batch volumes.
 * Synchronises the device once.  tr[K], grid, kernel and params are read only
 * during the call.  Errors: PAT_E_ARG, PAT_E_FRAME, PAT_E_SHAPE,
 * PAT_E_SEPARATION, PAT_E_KERNEL, PAT_E_DEVICE, PAT_E_OOM, and
 * PAT_E_UNSUPPORTED beyond the limits: 2^31 voxels or more, U > 65536, a fine
 * time axis (bins that can reach a sample) reaching beyond +-2^30; on error the
 * previous geometry, if any, is dropped (the context returns to PAT_E_STATE). */
pat_status pat_set_geometry(pat_ctx* ctx, const pat_transducer* tr, int32_t K,
                            const pat_grid* grid, const pat_kernel* kernel,
                            const pat_params* params);

/* signal = A coef (Alg. 1).  coef: device [batch][N], signal: device
 * [batch][K][L], element type per params.precision, each aligned to its element
 * size.  1 <= batch <= max_batch.  Asynchronous on hip_stream (NULL: the
 * default stream).  Errors (nothing is launched): PAT_E_ARG for a NULL or
 * misaligned buffer or a batch out of range, PAT_E_STATE before a successful
 * pat_set_geometry; PAT_E_DEVICE if a launch fails. */
pat_status pat_forward(pat_ctx* ctx, const void* coef, void* signal, int32_t batch,
                       void* hip_stream);

/* A restricted to the support of the coefficients (Alg. 3 with its sum over voxels
 * limited to the voxels where some volume's coefficient is nonzero; the paper
 * computes its reference signals this way on sparse phantoms).  Same arguments and
 * result as pat_forward up to summation order; the support is rebuilt on the device
 * from `coef` at every call (no host synchronisation).  Surface methods only:
 * PAT_E_UNSUPPORTED for PAT_AREA_QUADRATURE. */
pat_status pat_forward_sparse(pat_ctx* ctx, const void* coef, void* signal, int32_t batch,
                              void* hip_stream);

/* coef = A^T signal (Alg. 5 with Alg. 6 or Alg. 7).  Same layouts as forward. */
pat_status pat_adjoint(pat_ctx* ctx, const void* signal, void* coef, int32_t batch,
                       void* hip_stream);

/* signal = A coef like pat_forward, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid it): the call allocates nothing and frees nothing.  Its only scratch,
 * the FP64 fine-bin coefficients ([batch][K][fine bins kept] doubles), lives
 * in a static device array of 64 MiB per GPU that the library holds until the
 * process ends, cleared by a kernel at every call (the context's own
 * workspace is not used).  Every call on one GPU shares that array: calls that
 * overlap on one GPU (other streams, other contexts, other threads) race and
 * must be serialised by the caller.  Same arguments, layouts and result as
 * pat_forward; PAT_E_UNSUPPORTED when batch * K * (fine bins kept) * 8 bytes
 * exceeds 64 MiB (pat_query(2) gives the fine bins kept), PAT_E_DEVICE if the
 * array's address could not be looked up when the context was created. */
pat_status pat_forward_noalloc(pat_ctx* ctx, const void* coef, void* signal, int32_t batch,
                               void* hip_stream);

/* Host-only, FP64: discrete system kernel h[n] of Eq. def_bh for
 * g(t) = -1/2 c t phi(c|t|) (Prop. 1) with phi = cone or Wendland
 * (1 - r/kappa)^2_+, h = e * g (Eq. def_h), on the fine grid of step
 * 1/(U fs).  Writes up to `cap` taps to h_out and returns their range.
 * PAT_E_ARG if cap is too small (len still reports the size needed). */
pat_status pat_build_kernel(int32_t phi_type, double kappa, const pat_eir* eir,
                            double sound_speed, double fs, int32_t U,
                            double* h_out, int64_t cap, int64_t* n_first, int64_t* len);

/* Host-only validation of a geometry (the checks pat_set_geometry makes),
 * usable without a GPU.  *dist_lower receives the lower bound of the voxel to
 * surface distance used for the separation check (may be NULL). */
pat_status pat_check_geometry(const pat_transducer* tr, int32_t K, const pat_grid* grid,
                              double kappa, double* dist_lower);

/* Queries (what):
 *   0 number of transducers K        1 number of voxels N
 *   2 fine bins kept per transducer  3 index of the first kept bin (M_lo)
 *   4 1 if some arrival may fall after the last sample (window truncation)
 *   5 workspace bytes                6 ABI version
 *   7 area evaluations per volume and application (closed form: one per
 *     quadrant and fine bin; quadrature: one per surface point), counted on
 *     the device at the first request (synchronous)
 *   8 voxel-transducer pairs per volume
 *   9 area shells per time tile of the (transducer, time tile) forward, 0 if off */
pat_status pat_query(const pat_ctx* ctx, int32_t what, double* out);

/* Vector-ALU peak of HIP device `device` as this library's kernels are built
 * (FP32 not packed): an FMA-only kernel, sixteen independent chains per lane
 * and no memory access in its loop, over eight work-groups per compute unit,
 * timed with HIP events.  out[0] FP64 FLOP/s, out[1] FP32 FLOP/s (an FMA counts
 * 2), out[2] compute units, out[3] peak engine clock in GHz (device
 * properties).  Synchronous; allocates and frees a few MB of device memory.
 * Measurement aid for placing the published peaks; PAT_E_DEVICE without a GPU. */
pat_status pat_probe_peak(int32_t device, double* out);

const char* pat_status_string(int32_t status);
const char* pat_last_error(const pat_ctx* ctx);

/* Frees the context's device memory (after synchronising its device). */
void pat_destroy(pat_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* PATOP_H */
