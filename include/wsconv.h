/*
 * wsconv -- FFT-based convolution with radially symmetric weakly singular
 * kernels on the unit square, for AMD Instinct MI355X (gfx950).
 *
 * Method: Tiwari, Pandey, Paul, Anand, "Fast accurate approximation of
 * convolutions with weakly singular kernel and its applications".
 *
 *   (A u)(x)   = int_D g(x - y) u(y) dy,  D = [0,1]^2            (Section 1, eq. conv)
 *   (A_n u)(x) = sum_{k in F_n} ghat(k) uhat_{e,n}(k) e^{2 pi i k.x/b}    (Section 2.1, eq. An)
 *
 * evaluated at the grid points x_j = j/n, j in [0,n)^2.  The density is
 * zero-extended to the b-periodic square [0,b]^2 (eq. fc_discrete), its
 * trapezoidal Fourier coefficients are taken on the nb x nb grid, multiplied
 * by the kernel moments ghat(k) (Section 2.2, eq. ghat) and transformed back.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Arrays of grid samples are row-major [n][n] with the FIRST index the x1
 *    coordinate (sample [j1][j2] = u(j1/n, j2/n)); batches are [batch][n][n].
 *  - Real arrays are float64 (WS_FP64 plans) or float32 (WS_FP32 plans);
 *    complex arrays are interleaved (re, im) pairs of the same width.
 *  - Every device pointer must be device memory of the current HIP device,
 *    aligned to 16 bytes, and is owned by the caller.  The library never
 *    allocates device memory; the caller sizes buffers with the *_query calls.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *    enqueued asynchronously on it; calls return without waiting unless the
 *    description says otherwise.
 *  - Return value: 0 (WS_OK) on success, a negative WS_E* code on failure;
 *    nothing is enqueued when a call fails its argument checks.
 *    conv_last_error() then returns a message (per host thread).
 *  - A plan may be used from one host thread at a time.
 */
#ifndef WSCONV_H
#define WSCONV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define WS_OK            0
#define WS_EINVAL       -1   /* invalid argument (sizes, kernel parameters, NULL pointers) */
#define WS_EUNSUPPORTED -2   /* valid but not supported (FFT length, plan/precision combination) */
#define WS_EDEVICE      -3   /* a HIP runtime call failed */

/* Kernel families (Section 2.2). */
#define WS_LOG       0   /* g(x) = scale * log|x|                               */
#define WS_POWER     1   /* g(x) = scale * |x|^gamma,  -2 < gamma < 0           */
#define WS_HELMHOLTZ 2   /* g(x) = scale * (i/4) H0^(1)(kappa |x|), kappa > 0   */
#define WS_YUKAWA    3   /* g(x) = scale * K0(kappa |x|), kappa > 0 (Table yukawa: scale = 1/(2 pi)) */

/* Arithmetic of the apply. */
#define WS_FP64 0
#define WS_FP32 1        /* FFT passes and spectral multiply in float32; twiddles formed in float64 and rounded once to float32 */

/* Fourier-smoothing shapes (Section 2.4). */
#define WS_FS_NONE   0
#define WS_FS_DISC   1   /* indicator of the disc |x - c| < size                 */
#define WS_FS_SQUARE 2   /* indicator of the square |x - c|_inf < size           */

/* Lippmann-Schwinger solver status (ws_ls_info.status). */
#define WS_LS_CONVERGED 0
#define WS_LS_MAXIT     1
#define WS_LS_BREAKDOWN 2

typedef struct {
    int    family;   /* WS_LOG, WS_POWER, WS_HELMHOLTZ or WS_YUKAWA */
    double scale;    /* multiplies g */
    double gamma;    /* WS_POWER: exponent, -2 < gamma < 0 */
    double kappa;    /* WS_HELMHOLTZ: wavenumber > 0; WS_YUKAWA: decay rate > 0 */
    double beta;     /* real kernels: 0 for the global moments (closed forms of Section 2.2; for
                        WS_YUKAWA the truncated moment int_0^a rho K0(kappa rho) J0(xi rho) d rho
                        in closed form), or the localisation radius 0 < beta <= a of Section 2.3:
                        the table is then ghat_eta(k) + Khat(k), the moments of g eta_beta by the
                        trapezoidal rule after rho = beta tau^4, plus the DFT of the trapezoid
                        samples of the smooth part g (1 - eta_beta) (see conv_plan) */
} ws_kernel;

typedef struct {
    int    n;               /* grid points per side on D; power of two, 16 <= n <= 2048 */
    int    b;               /* period of the extension D_e = [0,b]^2 (Section 2.1): 2, or 3 for
                               densities supported on all of D (b >= 1 + sqrt 2, Section 2.1).
                               b = 3 is not taken by Fourier smoothing (WS_EUNSUPPORTED) */
    double a;               /* truncation radius of the kernel ball B_a(0) (eq. io); <= 0 selects
                               the default (b + sqrt(2)/2 - 1/2)/2, the midpoint of the disc window
                               below.  The scheme computes the convolution only when a is at least
                               the largest distance |x - y| between a target x in D and a point y
                               of the density's support, and smaller than the distance from x to
                               every periodic image of that support (Section 2.1, eq. io): for a
                               density supported in the disc |y - (1/2, 1/2)| <= rho
                               (support_radius = rho > 0) the window is
                               [rho + sqrt(2)/2, b - 1/2 - rho]; for support anywhere in D
                               (support_radius <= 0) it is [sqrt(2), b - 1], which is empty at
                               b = 2.  A radius outside its window is WS_EINVAL unless force_a is
                               set; any a must satisfy 0 < a < b */
    double support_radius;  /* rho: the densities (and LS contrasts, and Fourier-smoothed
                               densities out to their window radius psi_r2) vanish outside
                               |y - (1/2, 1/2)| <= rho; <= 0: supported anywhere in D */
    int    force_a;         /* nonzero: skip the window check of a (the operator is then the
                               truncated kernel's, which differs from A where the window fails) */
} ws_grid;

/* Fourier smoothing descriptor for one density (Section 2.4, eqs. ls1, tfs).
 * The density passed to conv_apply is then u_tilde, a smooth extension, and
 * the operator is applied to u_tilde * chi^n * psi, where chi^n is the
 * truncated b-periodic Fourier series of the shape's indicator on F_n and
 * psi(r) = 1 for r <= psi_r1, step((r - psi_r1)/(psi_r2 - psi_r1)) between,
 * 0 for r >= psi_r2, with r = |x - c| and step(t) = exp(2 e^{-1/t}/(t - 1)).
 * The centre must be a grid point (n*c1 and n*c2 integers) so chi^n is real.
 * The smoothed density vanishes beyond psi_r2 from the centre: with a plan
 * built for support_radius rho > 0 and without force_a, |c - (1/2, 1/2)| +
 * psi_r2 must not exceed rho (WS_EINVAL), so the a-window of the plan holds. */
typedef struct {
    int    shape;          /* WS_FS_NONE, WS_FS_DISC or WS_FS_SQUARE */
    double c1, c2;         /* centre */
    double size;           /* disc radius or square half-width */
    double psi_r1, psi_r2; /* window radii, 0 < psi_r1 < psi_r2 */
} ws_fs_desc;

typedef struct {
    int    status;        /* WS_LS_CONVERGED, WS_LS_MAXIT or WS_LS_BREAKDOWN */
    int    iterations;    /* Arnoldi columns built (all cycles, all refinements) */
    int    matvecs;       /* operator applications, including true-residual checks */
    int    refinements;   /* outer refinement steps (mixed precision), else 0 */
    double rel_residual;  /* final true relative residual ||u_inc - K u|| / ||u_inc||, in FP64 */
} ws_ls_info;

typedef struct ws_plan* ws_plan_t;

/* Sizes of the caller-owned buffers for a plan.
 * plan_bytes: device buffer holding the kernel moments ghat(k) (Section 2.2)
 *   and the twiddle tables (with beta > 0 also the localised scheme's
 *   construction scratch: the quadrature nodes and the n x n smooth-kernel
 *   samples and their half-transformed copy); work_bytes_per_density: device
 *   scratch for one density in conv_apply (the half-spectrum intermediate).
 * Returns WS_EINVAL / WS_EUNSUPPORTED for parameters conv_plan would reject. */
int conv_plan_query(const ws_kernel* kernel, const ws_grid* grid, int precision,
                    size_t* plan_bytes, size_t* work_bytes_per_density);

/* Build a plan (Section 2.1 discretisation + Section 2.2 moments).
 * Computes, on the device and in FP64, the moments ghat(k) for every k in
 * F_n scaled by (nb)^-2, in the layout the apply kernels read, plus the
 * twiddle tables; all of it is written into plan_buf (plan_bytes, device).
 * With kernel->beta > 0 (real kernels) the table is that of the localised
 * scheme (Section 2.3, eq. io_split): ghat_eta(k) = 2 pi int_0^beta g eta J0
 * rho d rho by the trapezoidal rule in tau after rho = beta tau^4 (M + 1 nodes,
 * M = max(768, ceil(4 beta pi sqrt(2) n))), plus Khat(k), the DFT over
 * (-n, n)^2 of h^2 g(|m| h)(1 - eta_beta(|m| h)), h = 1/n; eta_beta is 1 on
 * [0, beta/2] and the smooth step exp(2 e^(-1/t) / (t - 1)) of
 * t = (rho - beta/2)/(beta/2) beyond.  Localised plans copy their quadrature
 * nodes from the host and synchronise `stream` before returning.
 * The host-side plan object keeps raw pointers into plan_buf: the caller must
 * keep plan_buf alive until conv_destroy.  Enqueued on `stream`. */
int conv_plan(const ws_kernel* kernel, const ws_grid* grid, int precision,
              void* plan_buf, void* stream, ws_plan_t* out_plan);

/* Effective truncation radius a of a plan (after defaulting). */
double conv_plan_radius(ws_plan_t plan);

/* Apply A_n (Section 2.1, eq. An) to `batch` densities.
 *  density: [batch][n][n] samples u_j; real for WS_LOG / WS_POWER plans,
 *           complex for WS_HELMHOLTZ plans; element type per the plan precision.
 *  out:     [batch][n][n] results (A_n u)(x_j), same type as density.  May equal
 *           density (in place).
 *  work:    batch * work_bytes_per_density bytes of device scratch.
 *  fs:      NULL, or a host array of `batch` descriptors; entries with shape
 *           WS_FS_NONE are applied plainly (Section 2.4 otherwise).
 * batch = 0 is a no-op. */
int conv_apply(ws_plan_t plan, int batch, const void* density, void* out, void* work,
               const ws_fs_desc* fs, void* stream);

/* conv_apply for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  Same operation, arguments and results as conv_apply, without the
 * `work` argument: the intermediate lives in a fixed 64 MiB device array of
 * the library (one per device, held from the first call on that device until
 * the process ends), so a plan qualifies when its work_bytes_per_density is
 * at most 64 MiB (at period 2 every real-kernel plan up to n = 2048 in FP64,
 * Helmholtz plans up to n = 1024 in FP64, 2048 in FP32; at period 3 every plan
 * up to n = 1024, and FP32 real-kernel plans at 2048); larger ones return
 * WS_EUNSUPPORTED.  Densities go through the passes
 * min(conv_apply_chunk(plan), 64 MiB / work_bytes_per_density) at a time, with
 * results bitwise equal to conv_apply's.  The call allocates nothing; its
 * first call on a device resolves the array's device address once.  Every
 * call on a device shares the one array: calls that overlap in time on one
 * device (other streams, other host threads) race and must be serialised by
 * the caller. */
int conv_apply_noalloc(ws_plan_t plan, int batch, const void* density, void* out, const ws_fs_desc* fs,
                       void* stream);

/* One of the three passes of conv_apply without Fourier smoothing, for callers
 * that time or interleave them: pass 0 = row transforms of the density into
 * `work`, pass 1 = column transforms with the multiply by ghat (in `work`),
 * pass 2 = inverse row transforms from `work` into `out` (Section 2.1, eq. An).
 * conv_apply(plan, batch, u, out, work, NULL, s) enqueues exactly pass 0, 1, 2.
 * Arguments as for conv_apply; `density` is read by pass 0 only and `out`
 * written by pass 2 only. */
int conv_apply_pass(ws_plan_t plan, int pass, int batch, const void* density, void* out, void* work,
                    void* stream);

/* Apply several plans' operators at once: item i applies plans[i] to batch[i]
 * densities at density[i] (layout and element type as conv_apply) into out[i]
 * (may equal density[i]), with work[i] holding
 * min(batch[i], conv_apply_chunk(plans[i])) * work_bytes_per_density of plan i.
 * Every pass of the apply is one launch shared by all items of one period (up
 * to 8 items per launch; plans of period 2 and of period 3 take separate
 * launches), so densities of different grid sizes and kernels run together;
 * each result equals what conv_apply gives for that item alone, to rounding.
 * All plans must have the same precision and be all real-kernel (WS_LOG /
 * WS_POWER) or all WS_HELMHOLTZ (else WS_EUNSUPPORTED); no Fourier smoothing.  Items must
 * not share work buffers.  count = 0 is a no-op. */
int conv_apply_multi(int count, const ws_plan_t* plans, const int* batch, const void* const* density,
                     void* const* out, void* const* work, void* stream);

/* Number of densities conv_apply takes through all three passes at a time:
 * a chunk's intermediate is sized to stay in the GPU's last-level cache
 * between passes.  Callers driving conv_apply_pass over a large batch should
 * group densities the same way.  work_bytes_per_density times this count is
 * the scratch conv_apply actually touches. */
int conv_apply_chunk(ws_plan_t plan);

/* Device scratch needed by ls_solve for a given restart length. */
int ls_solve_query(ws_plan_t plan, int restart, int mixed_precision, size_t* work_bytes);

/* Solve the Nystrom discretisation of the Lippmann-Schwinger equation
 * (Section 3.3, eq. descretls):  u_j + kappa^2 (A_n(m u))_j = u_inc_j,  j in G_n,
 * by restarted GMRES(restart) from u = 0 with Gram-Schmidt and one
 * reorthogonalisation (delayed into the next Arnoldi step's single reduction)
 * and Givens rotations, all in FP64 on the device; the stop test is the
 * true relative residual ||u_inc - K u||_2 / ||u_inc||_2 <= tol (K = I + kappa^2 A_n M).
 *  plan:      a WS_HELMHOLTZ plan (kappa from the kernel).
 *  contrast:  [n][n] float64, m = 1 - mu (device).
 *  u_inc:     [n][n] complex128 incident field (device).
 *  u_out:     [n][n] complex128 solution (device).
 *  mixed_precision: 0 -> FP64 operator throughout; 1 -> iterative refinement: FP64 residual
 *             and correction, inner GMRES with the FP32 operator (plan precision WS_FP32).
 *  max_matvecs: bound on operator applications (all cycles).
 *  work:      ls_solve_query bytes of device scratch.
 *  info:      host struct, filled on return.
 * Arnoldi steps are enqueued in chunks of four, replayed from graphs captured
 * on first use and cached in the plan per (work, contrast, restart) buffers;
 * with the environment variable WSCONV_LS_GRAPHS=0 set when the plan is built
 * they are launched directly.  On the null stream the solve runs on a
 * library-owned stream ordered after and before the caller's work.
 * Synchronises the stream a few times per restart cycle to read the convergence state.
 * Returns WS_OK when it converged, 1 (positive) when it stopped at max_matvecs
 * (u_out holds the last iterate) and WS_LS_BREAKDOWN status with return 2 on a
 * non-finite residual. */
int ls_solve(ws_plan_t plan, const void* contrast, const void* u_inc, double tol,
             int restart, int max_matvecs, int mixed_precision, void* u_out, void* work,
             ws_ls_info* info, void* stream);

/* Device scratch needed by ls_solve_batch for `count` solves (1 <= count <= 64). */
int ls_solve_batch_query(ws_plan_t plan, int count, int restart, int mixed_precision, size_t* work_bytes);

/* `count` solves of eq. descretls (Section 3.3) with one plan, run together:
 * u_s + kappa^2 (A_n(m_s u_s))_j = u_inc_s,j for s < count, each with its own
 * contrast and incident field.
 *  contrast: device [count][n][n] float64; u_inc, u_out: device [count][n][n]
 *            complex128 (16-byte aligned); work: ls_solve_batch_query bytes,
 *            256-byte aligned; info: host array of `count` entries.
 * The solves run as `count` GMRES instances in lockstep: every Arnoldi step is
 * one set of launches for all of them (the operator over `count` densities,
 * the Gram-Schmidt and Givens kernels over `count` instances), and each
 * instance keeps its own Hessenberg matrix, rotations, stop test and
 * max_matvecs budget, so solve s returns what ls_solve returns for it alone.
 * Arguments otherwise as for ls_solve.  Returns WS_OK when every solve
 * converged, else the largest status among them (1: some solve stopped at
 * max_matvecs, 2: some solve broke down on a non-finite value; info[s] says
 * which), or a negative WS_E* code. */
int ls_solve_batch(ws_plan_t plan, int count, const void* contrast, const void* u_inc, double tol, int restart,
                   int max_matvecs, int mixed_precision, void* u_out, void* work, ws_ls_info* info, void* stream);

/* Device scratch needed by ls_solve_fs (the smoothed contrast and its
 * pre-pass intermediate, then ls_solve's scratch).  WS_EUNSUPPORTED for
 * plans of period b != 2; fs is checked as in conv_apply and must name a
 * disc or a square. */
int ls_solve_fs_query(ws_plan_t plan, const ws_fs_desc* fs, int restart, int mixed_precision,
                      size_t* work_bytes);

/* ls_solve for a contrast with a jump across the boundary of a disc or square
 * Omega (Section 2.4 applied to the Lippmann-Schwinger density m u of
 * Section 3.3; Example 9 with m = -1 in a disc).  The caller passes a smooth
 * extension m_tilde of the contrast on Omega (device [n][n] float64,
 * 16-byte aligned) and the descriptor of Omega and of the window psi; the
 * operator uses the smoothed contrast m_s = m_tilde chi^n_Omega psi (eqs. ls1,
 * tfs), computed on the device into `work` (256-byte aligned,
 * ls_solve_fs_query bytes), and the solve proceeds as ls_solve with
 * contrast m_s.  Every other argument, the return value and the stream
 * behaviour are as for ls_solve. */
int ls_solve_fs(ws_plan_t plan, const void* contrast_tilde, const ws_fs_desc* fs, const void* u_inc,
                double tol, int restart, int max_matvecs, int mixed_precision, void* u_out, void* work,
                ws_ls_info* info, void* stream);

/* Device scratch for conv_eval: the spectrum of one density (nb x nb
 * complex128) and its three real planes (3 nb x nb float64), the row-pass
 * intermediate (n x nb complex128), two groups of three nb x T float64 planes
 * for a tile of T targets (T = 64 .. 4096, 96 MiB per group at most) and, for
 * real-kernel plans, the density widened to complex.  WS_EUNSUPPORTED for
 * WS_FP32 plans. */
int conv_eval_query(ws_plan_t plan, size_t* work_bytes);

/* (A_n u)(x) at `count` arbitrary points x of the plane (Section 2.1: the
 * series of eq. An, sum_{k in F_n} ghat(k) uhat_{e,n}(k) e^{2 pi i k.x/b},
 * read at x; the quadrature form of eqs. quad / quad_wts gives the same sum).
 *  density: [n][n] samples of one density, as for conv_apply (FP64 plans).
 *  targets: device [count][2] float64, (x1, x2) of each point (any real
 *           values; the series is b-periodic).
 *  out:     device [count] complex128.  F_n = [-nb/2, nb/2)^2 is not
 *           symmetric, so off the grid the value is complex even for a real
 *           density and kernel; at grid points it equals conv_apply's.
 *  work:    conv_eval_query bytes, 256-byte aligned.
 * Cost: one forward transform of the density, then |F_n| = (nb)^2 complex
 * multiply-adds per target (for modest target counts), the sum over k2 as a
 * complex matrix product per tile of targets (three real products, rocBLAS
 * DGEMM, in the three-multiplication form; the library
 * keeps one rocBLAS handle per device, made on the first call there, which
 * may allocate rocBLAS's own device workspace). */
int conv_eval(ws_plan_t plan, const void* density, int count, const double* targets, void* out,
              void* work, void* stream);

/* Read back `count` moments ghat(k) (Section 2.2, eq. ghat) of a built plan,
 * for the integer frequencies (k1[i], k2[i]) in F_n, as computed on the device
 * (FP64, without the (nb)^-2 factor).  out: host array of 2*count doubles
 * (real, imaginary).  Synchronises `stream`. */
int conv_plan_moments(ws_plan_t plan, int count, const int* k1, const int* k2, double* out, void* stream);

/* Release the host-side plan object (the caller frees plan_buf). */
void conv_destroy(ws_plan_t plan);

/* Message for the last failing call on this host thread ("" if none). */
const char* conv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WSCONV_H */
