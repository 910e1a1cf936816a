/*
 * tfsc -- semi-coherent time-frequency detection statistic for LISA
 * stellar-mass binary searches (arXiv 2510.19047), on AMD MI355X (gfx950).
 *
 * C ABI of libtfsc.so.  Every array argument is a DEVICE pointer owned by the
 * caller (the library never allocates or frees device memory).  Every call is
 * asynchronous and stream-ordered on `stream` (a hipStream_t; NULL = the
 * default stream).  Errors are reported as tfsc_status codes; no exception
 * crosses the ABI.  Argument checks that need device data (none today) would
 * be reported through per-template flags, never through a fault.
 *
 * Notation (paper Sec. "Methods"): the data are cut into Nt tranches of
 * M samples (duration dT = M dt, bin spacing delta f = 1/dT); each tranche is
 * Fourier transformed once; a template's frequency track visits one
 * tranche-bin pixel per bin of its N_F = 21 bin window per tranche; tranches
 * are grouped into N_seg equal segments (coherence length T_seg).
 */
#ifndef TFSC_H
#define TFSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TFSC_ABI_VERSION 4

typedef enum {
    TFSC_OK = 0,
    TFSC_ERR_ARG = 1,          /* NULL pointer or out-of-range scalar       */
    TFSC_ERR_SHAPE = 2,        /* inconsistent sizes                        */
    TFSC_ERR_DTYPE = 3,        /* unsupported element type / combination    */
    TFSC_ERR_WORKSPACE = 4,    /* workspace missing or too small            */
    TFSC_ERR_UNSUPPORTED = 5,  /* valid request the library does not handle */
    TFSC_ERR_HIP = 6,          /* a HIP runtime call failed                 */
    TFSC_ERR_SCRATCH = 7       /* larger than the static device scratch     */
} tfsc_status;

/* TFSC_I16: complex 16-bit two's-complement fixed point, value =
 * layer_scale * stored with |stored| <= 32767 (see tfsc_pixels). */
typedef enum { TFSC_F64 = 0, TFSC_F32 = 1, TFSC_BF16 = 2, TFSC_F16 = 3, TFSC_I16 = 4 } tfsc_dtype;

/* Pixel store layouts (complex values stored as interleaved (re, im)):
 *   LAYER_MAJOR    [C][K][Nt]  -- tranches contiguous within one frequency layer
 *   TRANCHE_MAJOR  [C][Nt][K]  -- bins contiguous within one tranche
 *   LAYER_MAJOR_CI [K][Nt][C]  -- as LAYER_MAJOR with the C channels of a pixel
 *                                 adjacent, so one load fetches all channels   */
typedef enum { TFSC_LAYER_MAJOR = 0, TFSC_TRANCHE_MAJOR = 1, TFSC_LAYER_MAJOR_CI = 2 } tfsc_layout;

/* Sampling grid.  C = 1 (TDI A), 2 (A, E; the paper's channels, Eq. (tdi2))
 * or 3 (A, E and T = (X + Y + Z)/sqrt3, the null channel;
 * tfsc_bank_statistic_multi returns TFSC_ERR_UNSUPPORTED for C = 3); M even,
 * 64 <= M <= 4096 and a
 * power of two (the transform's FFT); K = M/2 + 1 bins per tranche;
 * n_fresnel must be 21 (paper: N_F = 21 bins centred on the bin just above
 * the track frequency).  tukey_alpha is the data window's shape (paper: 0.1;
 * 0 = rectangular); it only enters tfsc_transform.                          */
typedef struct {
    int32_t n_channels;
    int32_t tranche_len;
    int32_t n_tranches;
    int32_t n_fresnel;
    double dt;
    double tukey_alpha;
} tfsc_grid;

/* Whitened TF pixels D[c][k][m] plus the template weights.  pix holds
 * complex values of `dtype` in `layout`; for the 16-bit types (BF16, F16,
 * I16) the true value is layer_scale[c*K + k] * stored (layer_scale is
 * [C][K] FP32, NULL otherwise).  The 16-bit stores are the paper's reduced
 * precision form (Sec. "Hardware acceleration and computational cost":
 * 16-bit storage with a per-layer scale); I16 spends all 16 bits on one
 * fixed-point grid per layer (step = layer max / 32767), about seven times
 * finer than F16's 11-bit significand for unit-variance whitened pixels.
 * inv_asd[K] = u_k = 1/sqrt(S0(f_k)) and tranche_w[Nt] = w_m = 1/sqrt(mu_m)
 * (0 = tranche excluded, e.g. it overlaps a data gap).  The template pixel of
 * channel c is T_c(t_m, f_m) h_m(f_k) u_k w_m (paper Eqs. (tdi2),
 * (inner-tranche-tf)).  tfsc_transform writes these five arrays.
 *
 * rho: NULL for a PSD separable as S_m(f_k) = mu_m S0(f_k).  For a PSD that
 * varies between tranches in a general way (paper Sec. "Search extension to
 * data with gaps": a time-frequency PSD per tranche, for locally stationary
 * noise), rho[K][Nt] FP32 (bin-major, tranches contiguous; device memory,
 * owned by the caller) holds rho_mk = sqrt(mu_m S0(f_k) / S_m(f_k)) and the
 * template pixel becomes T_c h_m(f_k) u_k w_m rho_mk; tfsc_transform_tf
 * writes it.  Read by tfsc_bank_statistic (THREAD schedule: every pixel
 * type; WAVE schedule: F64 or F32 pixels with the same arithmetic, or F32
 * pixels with F64 arithmetic), by tfsc_statistic_vjp (every pixel type) and
 * by tfsc_bank_statistic_multi (one rho for all realisations).
 *
 * orbit: NULL for the rigid analytic orbit (first order in the eccentricity
 * L / (2 sqrt3 R), paper Sec. "Implementation details").  Else the
 * spacecraft positions of the caller's orbit (paper Sec. "Outlook": numerical
 * or generic orbits at no extra cost), orbit[(3 i + x) Nt + m] = coordinate x
 * of spacecraft i at t_m = m dT in light-seconds, FP64 [3][3][Nt], device
 * memory owned by the caller.  The arm directions come from these positions;
 * the link transfer and the TDI-1.5 combination keep the equal arm length
 * L = 2.5e9 m.  tfsc_orbit_positions writes the analytic orbit in this
 * layout (a table equal to it gives the same results bit for bit).  Read by
 * every statistic call and the VJP.
 *
 * links: NULL for equal arms.  Else the light times of the six links at the
 * tranche starts (paper Sec. "Outlook": varying arm lengths and point-ahead
 * corrections of numerical orbits), links[l Nt + m] in seconds, FP64 [6][Nt],
 * device memory owned by the caller, positive and finite; rows 0, 1, 2 are
 * the links 0->1, 1->2, 2->0 and rows 3, 4, 5 the reverse links 1->0, 2->1,
 * 0->2 (sender->receiver).  Each tranche's geometry is frozen: link s->r is
 * received at p_r after its light time along the arm direction n_sr, and
 * the TDI combinations take every path's own delay,
 *   G_sr = -i pi f L_sr sinc(pi f L_sr (1 - k.n_sr))
 *          exp(-i pi f (L_sr (1 - k.n_sr) + 2 k.p_r)) (polarisation factor),
 *   X = (1 - D01 D10)(G20 + D20 G02) - (1 - D02 D20)(G10 + D10 G01), Y, Z
 *   cyclic, D_sr = exp(-2 pi i f L_sr), A, E, T from X, Y, Z as for equal
 *   arms (paper Sec. "Implementation details", Eq. (tdi2)).
 * Six equal times L on a table whose sides are exactly L give the
 * equal-arm response.  tfsc_link_lengths writes |p_r - p_s| of an orbit.
 *
 * tdi_generation: 0 or 1 for the first-generation combinations above (the
 * paper's rescaled TDI-1.5), 2 for the second generation on the same
 * frozen geometry (the data the paper analyses are TDI-2; Sec.
 * "Implementation details"): each combination minus itself delayed by the
 * round trips of its two arms, X2 = (1 - D01 D10 D02 D20) X, Y and Z
 * cyclic.  2 needs the links table (else TFSC_ERR_UNSUPPORTED); other
 * values give TFSC_ERR_ARG.
 * Read by tfsc_bank_statistic (both schedules; F64 pixels with F64
 * arithmetic or F32 with F32; no rho; the paper's Fresnel forms); the VJP,
 * the several-realisation and the harmonics calls return
 * TFSC_ERR_UNSUPPORTED when it is set.                                     */
typedef struct {
    tfsc_dtype dtype;
    tfsc_layout layout;
    void *pix;
    float *layer_scale;
    double *inv_asd;
    double *tranche_w;
    float *rho;
    const double *orbit;
    const double *links;
    int32_t tdi_generation;
} tfsc_pixels;

/* Template bank, structure of arrays, n templates, FP64:
 * mc [Msun] chirp mass; eta symmetric mass ratio (0.01..0.25); f0 [Hz] GW
 * frequency at t = 0; cos_theta, phi source direction (polar, azimuth);
 * psi polarisation angle; cos_iota inclination.  Track: 2PN TaylorT3.
 * The chirp mass is given either as mc or as ln_mc = ln(Mc / Msun) (the
 * differentiable parameter of tfsc_statistic_vjp); exactly one of the two
 * pointers is non-NULL (else TFSC_ERR_ARG).  With ln_mc the device forms
 * Mc = exp(ln_mc) in FP64 (within an ulp of the host's exp), and
 * tfsc_follow_up_step steps ln_mc in place.                                 */
typedef struct {
    int64_t n;
    const double *mc, *eta, *f0, *cos_theta, *phi, *psi, *cos_iota;
    const double *ln_mc;
} tfsc_bank;

/* Segment layout.  nseg_fixed > 0 gives every template that many segments;
 * 0 selects the per-template rule N_seg = 16 * 2^n, n = #{i=1..4 :
 * fdot0 >= 1.34e-12 Hz/s * 2^(3i - 3/2)} (16..256).  Segment s of a template
 * holds tranches m with floor(m N_seg / Nt) = s.  nseg[n] and
 * seg_offset[n+1] (exclusive prefix sum of nseg) are written by
 * tfsc_segment_layout and read by the statistic calls.                     */
typedef struct {
    int32_t nseg_fixed;
    int32_t *nseg;
    int64_t *seg_offset;
} tfsc_segments;

/* Arithmetic and schedule of the statistic kernels.
 * precision: TFSC_F64 -- response, Fresnel kernel and sums in FP64;
 *            TFSC_F32 -- FP32 response, Fresnel kernel and tranche sums
 *                        (segment sums stay FP64).  The track (phase,
 *                        frequency, chirp, bin index, track end) is always
 *                        FP64.
 * schedule:  TFSC_SCHED_THREAD -- one thread per template walking its
 *                        tranches (the paper's mapping); any layout.
 *            TFSC_SCHED_WAVE   -- one 64-lane wavefront per template, lanes
 *                        over consecutive tranches, persistent grid pulling
 *                        templates from a device work counter; LAYER_MAJOR
 *                        or LAYER_MAJOR_CI.
 * block_waves / groups_per_cu: launch shape of the WAVE schedule, waves per
 * block (1..4) and resident blocks per compute unit (1..64); 0 = default
 * (4, 4); larger values return TFSC_ERR_ARG.  order: optional [n] permutation of template indices giving the
 * processing order (NULL = bank order); results are written at the
 * template's own index whatever the order.
 * fresnel: TFSC_FRESNEL_PAPER -- the paper's Fresnel approximations (its
 *            rational forms for |z| <= 6, one-term asymptotic forms above;
 *            paper Sec. "Time-frequency waveform representation");
 *          TFSC_FRESNEL_ACCURATE -- the Fresnel integrals themselves to
 *            FP64 rounding in Eq. (fresnel-ft) (series, continued fraction
 *            and asymptotic series of the auxiliary functions), every bin in
 *            the general form: tfsc_bank_statistic with F64 pixels and F64
 *            precision or F32 pixels and F32 precision, no rho (else
 *            TFSC_ERR_UNSUPPORTED); the other calls accept only the paper's
 *            forms.
 * tune_key: NULL, or a key given to tfsc_tune_statistic earlier in this
 *            process; with block_waves and groups_per_cu both 0 the WAVE
 *            schedule then takes the launch shape tuned under that key
 *            (the defaults if the key was never tuned).                    */
enum { TFSC_SCHED_THREAD = 0, TFSC_SCHED_WAVE = 1 };
enum { TFSC_FRESNEL_PAPER = 0, TFSC_FRESNEL_ACCURATE = 1 };
typedef struct {
    int32_t precision;
    int32_t schedule;
    int32_t block_waves;
    int32_t groups_per_cu;
    const int32_t *order;
    int32_t fresnel;
    const char *tune_key;
} tfsc_options;

/* Per-template flag bits written by tfsc_bank_statistic. */
enum {
    TFSC_FLAG_INVALID = 1,      /* parameters out of range: statistic 0      */
    TFSC_FLAG_EMPTY = 2,        /* no active tranche                         */
    TFSC_FLAG_BAND_END = 4,     /* track ended by the band or compactness    */
    TFSC_FLAG_MERGE_END = 8,    /* track ended by the merger condition       */
    TFSC_FLAG_ALL_EXCLUDED = 16 /* every active tranche excluded (w_m = 0)   */
};

enum { TFSC_WS_LAYOUT = 0, TFSC_WS_STATISTIC = 1, TFSC_WS_VJP = 2, TFSC_WS_TRANSFORM = 3, TFSC_WS_ORDER = 4 };

int tfsc_abi_version(void);
const char *tfsc_status_string(int status);

/* Bytes of device workspace call `which` (TFSC_WS_*) needs for this grid,
 * bank size and options (0 if none).  Workspace contents need not be
 * initialised; calls sharing one workspace must not overlap in time.  The
 * statistic and VJP figures include 8 bytes per template for a bank given
 * in ln Mc (the calls form exp(ln Mc) there once); an mc bank needs only
 * the geometry tables and 256 bytes, and the calls check that need.       */
size_t tfsc_workspace_bytes(const tfsc_grid *grid, int64_t n_templates, const tfsc_options *opt, int which);

/* Data -> TF pixels (paper Sec. "Implementation details": each tranche is
 * Tukey-windowed and Fourier transformed once; a per-tranche PSD models
 * locally stationary noise; tranches overlapping gaps are left out of
 * Eq. (inner-tf)).
 *   x [C][N] time series (N = M Nt), x_dtype TFSC_F64 or TFSC_F32;
 *   psd0 [K] one-sided PSD S0(f_k) at f_k = k/dT (> 0 for 1 <= k < M/2);
 *   tranche_psd_scale [Nt] mu_m (> 0): tranche m has PSD mu_m S0;
 *   tranche_keep [Nt] uint8, 0 = exclude tranche m.
 * Writes out->pix (D = X sqrt(2 dt / (M W2 mu_m S0(f_k))), X the windowed
 * DFT with the tranche start as time origin, W2 = mean(w^2); excluded
 * tranches are 0), out->inv_asd, out->tranche_w, and out->layer_scale for
 * 16-bit stores (FP32: per layer max |component| for BF16 and F16, that
 * max / 32767 for I16, whose stored value is the nearest integer to
 * value / layer_scale).  A pixel whose PSD
 * mu_m S0(f_k) is not positive and finite (DC and Nyquist may be given as 0
 * or inf; they never enter the statistic) is written as 0, and so is its
 * weight (u_k = 0, or w_m = 0 when mu_m is not positive and finite), never
 * inf or NaN.  out->dtype may be F64 (x F64 only), F32, BF16, F16 or I16;
 * 16-bit outputs need TFSC_WS_TRANSFORM workspace.                                */
tfsc_status tfsc_transform(const tfsc_grid *grid, const void *x, int x_dtype, const double *psd0,
                           const double *tranche_psd_scale, const uint8_t *tranche_keep, tfsc_pixels *out,
                           void *ws, size_t ws_bytes, void *stream);

/* tfsc_transform for a PSD that varies between tranches in a general way
 * (paper Sec. "Search extension to data with gaps"): psd_tf[K][Nt] FP64
 * (device, bin-major, tranches contiguous) = S_m(f_k), positive and finite
 * for 1 <= k <= M/2 - 1.  The pixels are whitened pixel by pixel,
 * D_cmk = X_cmk sqrt(2 dt / (M W2 S_m(f_k))) (0 on excluded tranches), and
 * the template weights are written as u_k = 1/sqrt(S0_k) with S0_k the mean
 * of S_m(f_k) over the tranches, w_m = 1 (0 = excluded) and
 * rho_mk = sqrt(S0_k / S_m(f_k)) into out->rho, which must be set.  Where
 * S_m(f_k) (or the layer's mean S0_k) is not positive and finite, the pixel
 * and rho_mk (or u_k) are 0.  Same dtypes, layouts and workspace as
 * tfsc_transform.                                                          */
tfsc_status tfsc_transform_tf(const tfsc_grid *grid, const void *x, int x_dtype, const double *psd_tf,
                              const uint8_t *tranche_keep, tfsc_pixels *out, void *ws, size_t ws_bytes,
                              void *stream);

/* Per-template setup (paper Sec. "Methods": N_seg = tau / T_seg; here set
 * per template from fdot at t = 0, or fixed).  Writes seg->nseg and
 * seg->seg_offset; needs TFSC_WS_LAYOUT workspace.                         */
tfsc_status tfsc_segment_layout(const tfsc_grid *grid, const tfsc_bank *bank, tfsc_segments *seg, void *ws,
                                size_t ws_bytes, void *stream);

/* The statistic (paper Eqs. (Upsilon-seg), (overlap-n), (inner-segment-tf),
 * (inner-tranche-tf), (fresnel-ft)): for each template,
 *   z_n = sum_{c, m in segment n, k in the 21 bins} conj(D_cmk) Y_cmk,
 *   N_n = sum |Y_cmk|^2,  Upsilon_n = 2 |z_n|^2 / N_n (0 if N_n = 0),
 *   Upsilon = sum_n Upsilon_n,
 * with Y_cmk = T_c(t_m, f_m) h_m(f_k) u_k w_m, h_m the Fresnel-kernel
 * tranche spectrum of the TaylorT3 track expanded at the tranche start, and
 * the bins k = ceil(f_m dT) - 10 .. + 10 inside [1, M/2 - 1].
 * Outputs (FP64): seg_terms[seg_offset[n]], stat[n], flags[n] (TFSC_FLAG_*);
 * seg_zn[seg_offset[n]][3] = (Re z_n, Im z_n, N_n) if non-NULL (the VJP's
 * input).  The kernels use u_k 2^-e with e the binary exponent of
 * max_k u_k (an exact power-of-two rescaling that keeps FP32 sums in range);
 * Upsilon is unchanged by it, z_n and N_n carry factors 2^-e and 2^-2e.
 * n_active[n] (optional, may be NULL) receives the number of active tranches
 * with w_m != 0 each template visited (its pixel columns: 21 C pixels each,
 * minus bins outside [1, M/2 - 1]).  Needs TFSC_WS_STATISTIC workspace.     */
tfsc_status tfsc_bank_statistic(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc_bank *bank,
                                const tfsc_segments *seg, const tfsc_options *opt, double *seg_terms, double *stat,
                                double *seg_zn, int32_t *flags, int32_t *n_active, void *ws, size_t ws_bytes,
                                void *stream);

/* The statistic of tfsc_bank_statistic for n_real noise realisations of the
 * same grid in one pass over the bank (paper Sec. "Results": the background
 * comes from many noise-only realisations; Sec. "Hardware acceleration and
 * computational cost": large batches per launch).  Realisation r's pixel
 * store lies r * real_stride bytes after pix->pix (same dtype, layout,
 * inv_asd, tranche_w and rho for all; real_stride a multiple of 16 and at least
 * one store's size; n_real * real_stride < 4 GiB); 1 <= n_real <= 64.  Each
 * template's track, Fresnel spectrum and response are formed once per group
 * of `group` realisations (1, 2, 4 or 8; 0 = 8) and serve all of them; the
 * remainder goes in smaller groups.  The per-tranche bin table is parked in
 * LDS (21 complex values per lane), which limits residency to two waves per
 * SIMD: on the full-size workload one tfsc_bank_statistic launch per
 * realisation is faster, so this call serves callers that want one launch
 * and one output block for several realisations.  Outputs: stat[r * n + i],
 * seg_terms[r * seg_stride + seg_offset[i] + s] (seg_stride >= the total
 * number of segments; terms at or beyond seg_stride are not written, so a
 * short plane loses terms but never overruns), flags[n] and n_active[n]
 * (optional) once.  WAVE schedule; LAYER_MAJOR or LAYER_MAJOR_CI; one or
 * two channels (three: TFSC_ERR_UNSUPPORTED); FP32 pixels with FP32
 * precision or FP64 pixels with FP64 precision, else TFSC_ERR_DTYPE; no
 * seg_zn (the VJP takes one realisation).  Sums are
 * formed per bin rather than through the single-realisation kernel's
 * factored asymptotic sums, so the two agree to rounding, not bit for bit.
 * Needs TFSC_WS_STATISTIC workspace.                                       */
tfsc_status tfsc_bank_statistic_multi(const tfsc_grid *grid, const tfsc_pixels *pix, int32_t n_real,
                                      int64_t real_stride, int32_t group, const tfsc_bank *bank,
                                      const tfsc_segments *seg, const tfsc_options *opt, int64_t seg_stride,
                                      double *seg_terms, double *stat, int32_t *flags, int32_t *n_active, void *ws,
                                      size_t ws_bytes, void *stream);

/* Realisations interleaved in one store (real_stride = 0 in
 * tfsc_bank_statistic_multi): pix->pix holds [K][Nt][n_real][C] complex
 * values, each (bin, tranche) cell carrying every realisation's C channels
 * side by side (pix->layout TFSC_LAYER_MAJOR_CI; dtype TFSC_F32, or TFSC_I16
 * with pix->layer_scale [n_real C][K], realisation r's channel c in row
 * r C + c; F32 precision, n_real 2 or 4, group 0 or n_real, no rho, n_real
 * stores below 4 GiB; else TFSC_ERR_UNSUPPORTED).  One pass over the bank forms each
 * template's track, bins and response once per tranche for all n_real
 * realisations, and one wide load per bin brings every realisation's pixels;
 * outputs as above.  The bin sums are the single-realisation kernel's (with
 * the cell's n_real C values as channels), so each realisation agrees with
 * its own tfsc_bank_statistic to rounding.
 *
 * tfsc_interleave_store writes realisation r (0 <= r < n_real) of such a
 * store: src is one realisation's FP32 or I16 LAYER_MAJOR_CI store of this
 * grid (as tfsc_transform writes it), dst the interleaved store of the same
 * dtype and layout (dst->pix: device memory of b C n_real K Nt bytes, b = 8
 * for F32 and 4 for I16; for I16 also dst->layer_scale [n_real C][K], into
 * which src's scales are copied; owned by the caller).  inv_asd, tranche_w
 * and the rest of tfsc_pixels are those of any one realisation of the grid. */
tfsc_status tfsc_interleave_store(const tfsc_grid *grid, const tfsc_pixels *src, int32_t n_real, int32_t r,
                                  tfsc_pixels *dst, void *stream);

/* tfsc_bank_statistic for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, bit for bit, but the workspace
 * is a static device array of TFSC_NOALLOC_SCRATCH_BYTES inside the library
 * instead of a caller-provided one.  Each device holds its own copy until
 * the process ends (its address is looked up once per device, on the first
 * call with that device current); the call allocates nothing, neither do
 * the kernels it launches.  Grids of more than TFSC_NOALLOC_MAX_TRANCHES
 * tranches return TFSC_ERR_SCRATCH, and so does a bank given in ln Mc whose
 * 8 bytes per template do not fit beside the geometry tables.  All calls on one device share that
 * device's scratch (it keeps the last call's contents; the work counter is
 * cleared by a kernel at the start of every call): calls that overlap in
 * time on one device, on different streams or from different threads,
 * race and must be serialised by the caller.  Arguments, outputs and
 * errors otherwise as tfsc_bank_statistic.                                 */
#define TFSC_NOALLOC_MAX_TRANCHES 16384
#define TFSC_NOALLOC_SCRATCH_BYTES (3u << 20)
tfsc_status tfsc_bank_statistic_noalloc(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc_bank *bank,
                                        const tfsc_segments *seg, const tfsc_options *opt, double *seg_terms,
                                        double *stat, double *seg_zn, int32_t *flags, int32_t *n_active,
                                        void *stream);

/* Vector-Jacobian product of the statistic (gradient of Eq. (Upsilon-seg)
 * through Eqs. (overlap-n), (inner-segment-tf), (fresnel-ft) and the
 * response): g_params[n][5] =
 * d(sum_n g_seg_n Upsilon_n + g_stat Upsilon)/d(ln Mc, f0, cos theta, phi, psi)
 * per template, eta and cos iota held fixed, and the integer structure (bins,
 * Fresnel branches, track end, N_seg) held at the template's own values (the
 * almost-everywhere derivative).  The track, spectra and response are
 * recomputed with forward-mode tangents; nothing per pixel is stored.
 * seg_zn is the forward's output (tfsc_bank_statistic) for the same inputs;
 * g_stat[n] and/or g_seg[seg_offset[n]] may be NULL (not both).
 * opt->precision TFSC_F64 (also opt == NULL): every tangent in FP64;
 * TFSC_F32: spectra, response, pixel sums and their tangents in FP32, the
 * track, its tangents, the phases and every integer decision in FP64 (as in
 * the FP32 statistic); either arithmetic takes every pixel type and layout.
 * schedule and order are ignored, block_waves and groups_per_cu set the
 * launch.  Invalid and empty templates get 0.  Needs TFSC_WS_VJP workspace. */
tfsc_status tfsc_statistic_vjp(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc_bank *bank,
                               const tfsc_segments *seg, const tfsc_options *opt, const double *seg_zn,
                               const double *g_stat, const double *g_seg, double *g_params, void *ws,
                               size_t ws_bytes, void *stream);

/* A processing order for tfsc_bank_statistic (paper Sec. "Hardware
 * acceleration and computational cost": large batches of parameter sets per
 * launch): order[n] receives a permutation of 0..n-1 that groups templates
 * by the frequency bin of f0 (ascending; invalid templates last) and,
 * within a bin, by ln Mc in 256 classes of equal width over [ln 0.5,
 * ln 500) (ascending; chirp masses outside it join the end classes).
 * Templates that the WAVE schedule runs at the same time then start on the
 * same rows and, with similar chirps, stay on them, so the caches serve
 * their shared pixels (on the full-size workload the statistic kernel
 * takes 6% less time than in an order by f0 bin alone, 14% less with
 * three channels).
 * Results never depend on the order; within one bucket the order may differ
 * from call to call.  Needs TFSC_WS_ORDER workspace.                       */
tfsc_status tfsc_processing_order(const tfsc_grid *grid, const tfsc_bank *bank, int32_t *order, void *ws,
                                  size_t ws_bytes, void *stream);

/* One step of the gradient-ascent follow-up of candidates (the paper's
 * Outlook proposes differentiable templates for follow-up): for each
 * template, an Adam step (beta1 0.9, beta2 0.999) that increases Upsilon,
 * applied in place to bank->mc (through ln Mc), f0, cos_theta, phi and psi.
 * Step sizes are lr_scale times the statistic's resolution of the template:
 * delta f0 = 0.1 / T_seg, delta ln Mc = delta f0 / ((5/3) fdot(0) T_obs),
 * 0.05 for cos theta, phi and psi; (cos theta, phi) are reflected through a
 * pole when cos theta leaves [-1, 1], phi is wrapped to [0, 2 pi) and psi to
 * [0, pi).  stat[n] and g_params[n][5] are the forward's Upsilon and the
 * VJP's gradient at the current parameters; seg->nseg gives T_seg.
 * state[n][16] is caller-owned device memory: (Adam m[5], v[5], best
 * Upsilon, best mc, f0, cos theta, phi, psi); step = 1 initialises it, so it
 * needs no clearing.  Before updating, a template whose stat exceeds its best
 * records its current parameters as the best.  lr_scale = 0 only records
 * (use it after the last step's forward).  Invalid templates are not moved.  */
tfsc_status tfsc_follow_up_step(const tfsc_grid *grid, tfsc_bank *bank, const tfsc_segments *seg,
                                const double *stat, const double *g_params, double *state, double lr_scale,
                                int step, void *stream);

/* Largest statistic per parameter tile (paper Sec. "Results": the false-alarm
 * probability of a candidate comes from the background distribution of the
 * largest statistic a noise-only search returns in its tile).  stat[n] and
 * tile[n] are device arrays (tile[i] in 0..n_tiles-1, or negative to leave
 * template i out; stat[i] that is negative or NaN is also left out);
 * tile_max[n_tiles] receives each tile's largest stat (0 for a tile with no
 * template) and tile_arg[n_tiles] the smallest index attaining it (-1 for an
 * empty tile).  Exact: a maximum, not a sum, so the result is independent of
 * scheduling.  Plain kernels only (no memset), so the call can be captured
 * into a HIP graph.  n = 0 is allowed; n_tiles >= 1.                       */
tfsc_status tfsc_tile_max(const double *stat, const int32_t *tile, int64_t n, int32_t n_tiles, double *tile_max,
                          int64_t *tile_arg, void *stream);

/* Multi-harmonic templates (paper Sec. "Outlook": the time-frequency
 * representation extends to several harmonics by computing {A, f, fdot,
 * phi} for each harmonic and applying the Fresnel expressions to each).
 * harmonics[n_harm] (host memory, 1 <= n_harm <= TFSC_MAX_HARMONICS) are
 * distinct harmonic numbers h = 1..8 of the orbital phase: harmonic h has
 * phase (h/2) Phi, frequency (h/2) f and chirp (h/2) fdot of the template's
 * TaylorT3 track, amplitude a_h f^(2/3) with amp[(i n_harm + q) 2 + {0, 1}]
 * = (Re, Im) a_h of template i (device, FP64 [n][n_harm][2]), the
 * polarisation pattern of the dominant harmonic and its own TDI transfer
 * T_c(t_m, f_h).  Each harmonic fills its own 21 bins around
 * ceil(f_h dT); a bin in several windows (low frequencies) holds the sum.
 * The track ends at the merger condition or where the highest harmonic
 * violates the band or compactness condition.  Upsilon, segment terms,
 * (z_n, N_n), flags and n_active as in tfsc_bank_statistic.  WAVE schedule,
 * LAYER_MAJOR or LAYER_MAJOR_CI, F64 pixels with F64 precision or F32 with
 * F32 (else TFSC_ERR_DTYPE), no rho, the paper's Fresnel forms (else
 * TFSC_ERR_UNSUPPORTED).  h = {2}, a = 1 is tfsc_bank_statistic's template.
 * Needs TFSC_WS_STATISTIC workspace.                                       */
#define TFSC_MAX_HARMONICS 4
tfsc_status tfsc_bank_statistic_harmonics(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc_bank *bank,
                                          const tfsc_segments *seg, const tfsc_options *opt, int32_t n_harm,
                                          const int32_t *harmonics, const double *amp, double *seg_terms,
                                          double *stat, double *seg_zn, int32_t *flags, int32_t *n_active, void *ws,
                                          size_t ws_bytes, void *stream);

/* The rigid analytic orbit's spacecraft positions at the tranche starts,
 * out[(3 i + x) Nt + m] (light-seconds, FP64 [3][3][Nt], device), in the
 * layout of tfsc_pixels.orbit (paper Sec. "Implementation details").        */
tfsc_status tfsc_orbit_positions(const tfsc_grid *grid, double *out, void *stream);

/* The six link light times of an orbit without point-ahead differences,
 * out[l Nt + m] = |p_r - p_s| (seconds, FP64 [6][Nt], device, rows as
 * tfsc_pixels.links) of the caller's positions orbit (layout of
 * tfsc_pixels.orbit) or, for orbit = NULL, of the analytic orbit: the
 * varying arm lengths of a numerical orbit (paper Sec. "Outlook").         */
tfsc_status tfsc_link_lengths(const tfsc_grid *grid, const double *orbit, double *out, void *stream);

/* Launch-shape autotuner of the WAVE statistic (paper Sec. "Hardware
 * acceleration and computational cost": large batches per launch): times
 * tfsc_bank_statistic on the given (tuning) bank for eight launch shapes
 * (waves per block x resident blocks per CU: 4x4, 4x3, 4x2, 2x8, 2x6, 2x4,
 * 1x12, 1x8), the fastest of two launches each, after one warm-up launch;
 * stores the fastest under tune_key for the rest of the process and writes
 * it to *block_waves, *groups_per_cu.  Blocks the calling thread until the
 * timed launches on `stream` are done.  opt as for tfsc_bank_statistic (its
 * schedule, launch shape and tune_key are ignored); the outputs and the
 * workspace are overwritten.                                               */
tfsc_status tfsc_tune_statistic(const tfsc_grid *grid, const tfsc_pixels *pix, const tfsc_bank *bank,
                                const tfsc_segments *seg, const tfsc_options *opt, const char *tune_key,
                                double *seg_terms, double *stat, int32_t *flags, void *ws, size_t ws_bytes,
                                void *stream, int32_t *block_waves, int32_t *groups_per_cu);

/* The FP64 track behind every statistic call, for inspection: out[n][Nt][4]
 * holds (Phi_m, f_m, fdot_m, code_m) at each tranche start t_m = m dT, with
 * code_m = 0 for an active tranche, else the TFSC_FLAG_* bit of the
 * condition that ends the track there (Phi, f, fdot are 0 where the merger
 * condition holds).  Invalid templates give code TFSC_FLAG_INVALID.  Same
 * arithmetic, bit for bit, as the statistic kernels (paper Sec.
 * "Time-frequency waveform representation": second-order expansion at the
 * tranche start; Appendix A compactness).                                  */
tfsc_status tfsc_track(const tfsc_grid *grid, const tfsc_bank *bank, double *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* TFSC_H */
