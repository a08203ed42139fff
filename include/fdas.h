/*
 * fdas.h -- C ABI of the MI355X (gfx950) FDAS correlation library.
 *
 * Fourier Domain Acceleration Search, correlation step (Dimoudi et al.
 * 2018, "Pulsar acceleration searches on the GPU for the Square Kilometre
 * Array"): the complex Fourier amplitudes of a spectrum are correlated with
 * a bank of K complex FIR templates, one per trial frequency derivative z,
 * by overlap-save FFT segments, and the |.|^2 f-fdot power plane is
 * written out (Sec. 3, Fig. 1 and Fig. 3 caption; Sec. 4.1 workflow).
 * Around it: the batched path and its autotuner, the adjoint, interbinning,
 * two-bin Fourier interpolation, a half-size (+-z symmetric) bank, the
 * real-to-complex front end that makes the spectrum from a time series, and
 * harmonic summing with peak candidates on the plane (Sec. 3 processing
 * steps).
 *
 * Definition of the result (Sec. 2, eq. 23): with taps j in [0, M) at bin
 * offsets e_j = j - M/2 and the spectrum A taken as zero outside [0, N),
 *     Y[z][r] = sum_j A[r + e_j] * conj(T[z][j]),   P[z][r] = |Y[z][r]|^2,
 * for r in [0, N).  The segment length L (Sec. 3: blocks of L = B + M
 * bins, B useful outputs each) is a performance parameter: every supported
 * L gives the same plane up to FP32 rounding.
 *
 * Conventions for every call:
 *  - Complex data is fdas_cf32 (interleaved float re, im; the layout of a
 *    torch.complex64 element).  Pointers suffixed _dev are device pointers
 *    on the current HIP device; _host are host pointers.
 *  - The caller owns every buffer.  Calls on the hot path (fdas_correlate,
 *    fdas_correlate_batched, fdas_correlate_backward) never allocate.
 *  - Calls are asynchronous on `stream` (0 = the null stream) and validate
 *    all arguments before launching anything; on any non-zero status no
 *    kernel has been launched and no output was touched.
 *  - Outputs are fully overwritten, never accumulated into.
 *  - Status codes: FDAS_OK 0; FDAS_INVALID_ARG 1 (null/misaligned pointer,
 *    negative size, inconsistent grid); FDAS_UNSUPPORTED 2 (geometry outside
 *    the supported set: L not a power of two in [256, 8192], M odd, M < 2 or
 *    M > L/2, K < 1 or K > 4096); FDAS_WORKSPACE_TOO_SMALL 3; FDAS_HIP_ERROR 4
 *    (a HIP call failed; fdas_last_error() has the text).  Nothing aborts
 *    and no C++ exception crosses the ABI.
 */
#ifndef FDAS_H
#define FDAS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    float re, im;
} fdas_cf32;

enum {
    FDAS_OK = 0,
    FDAS_INVALID_ARG = 1,
    FDAS_UNSUPPORTED = 2,
    FDAS_WORKSPACE_TOO_SMALL = 3,
    FDAS_HIP_ERROR = 4
};

/* Library version string (static storage). */
const char *fdas_version(void);

/* Static text for a status code. */
const char *fdas_status_string(int status);

/* Detail of the last failure on the calling thread ("" if none). */
const char *fdas_last_error(void);

/*
 * Number of trial templates for the z grid z_k = (k - (K-1)/2) * dz,
 * k in [0, K), i.e. -zmax .. +zmax in steps of dz, K = 2*zmax/dz + 1.
 * zmax >= 0, dz > 0 and zmax must be an integer multiple of dz (relative
 * tolerance 1e-9), else FDAS_INVALID_ARG.  The paper's grid steps z by 2,
 * one template apart (Sec. 5.2).
 */
int fdas_num_templates(double zmax, double dz, int *K);

/*
 * Predicted normalised Fourier response R(q, z) of a unit-amplitude
 * constant-fdot signal (Sec. 2, text before eq. 23), evaluated on the host
 * in FP64: the response at bin k of a signal that sits at bin r at
 * mid-observation and drifts by z bins over the observation, q = r - k,
 *     R(q, z) = int_0^1 exp(i 2 pi [q u + z (u^2 - u)/2]) du.
 * Writes the real and imaginary parts.  Never fails for finite input.
 */
int fdas_template_response(double q, double z, double *re, double *im);

/*
 * Template bank on the host: taps_host[k*M + j] = R(j - M/2, z_k), FP64
 * rounded once to FP32.  Templates are not renormalised after truncation
 * to M taps.  M even, 2 <= M <= 16384.  Writes K*M elements.
 */
int fdas_make_templates_host(double zmax, double dz, int M, fdas_cf32 *taps_host);

/* Number of fdas_cf32 elements of a prepared bank: (K + 1) * L. */
int64_t fdas_bank_elems(int K, int L);

/*
 * Prepare the Fourier-domain bank for segment length L from K templates of
 * M taps (Sec. 3, Fig. 1: each filter is placed at the two ends of an
 * L-array so that it is centred on bin 0 -- tap j at index (M/2 - j) mod L,
 * zeros strictly between M/2 and L - M/2 + 1 -- conjugated, and Fourier
 * transformed).  Layout of bank_dev ((K + 1) * L elements, 16-byte
 * aligned):
 *   rows 0..K-1 : H_z[k] = (1/L) sum_j conj(T[z][j]) exp(-2 pi i ((M/2-j) mod L) k / L),
 *                 natural frequency order, accumulated in FP64, rounded once;
 *   row K       : twiddles exp(-2 pi i n / L), n in [0, L), FP64 rounded once.
 * The 1/L of the inverse DFT (printed without it in Sec. 4.2) is folded in.
 * taps_dev: K*M elements, 8-byte aligned.  Not on the hot path.
 */
int fdas_prepare_bank(const fdas_cf32 *taps_dev, int K, int M, int L,
                      fdas_cf32 *bank_dev, hipStream_t stream);

/*
 * Templates for the grid (zmax, dz) with M taps, computed on the host in
 * FP64 and copied to taps_dev (K*M elements, required); if bank_dev is not
 * NULL the bank for segment length L is prepared from those taps as by
 * fdas_prepare_bank (L is ignored when bank_dev is NULL).  Blocks the host
 * until the copy has been consumed.  Not on the hot path.
 */
int fdas_make_templates(double zmax, double dz, int M, int L,
                        fdas_cf32 *taps_dev, fdas_cf32 *bank_dev,
                        hipStream_t stream);

/*
 * Forward correlation of one spectrum: the fused overlap-save pipeline of
 * Sec. 3 / Sec. 4.2 (segment load with zero fill, forward FFT, K template
 * multiplies, inverse FFTs, |.|^2 and edge rejection) in one launch.
 *   spec_dev  : N complex bins, 8-byte aligned (read only);
 *   N         : bins, 0 <= N <= 2^32 (N = 0 is a no-op);
 *   bank_dev  : prepared bank for (K, M, L) from fdas_prepare_bank;
 *   plane_dev : K*N floats, row-major [z][r], 4-byte aligned; every element
 *               is written.
 * Segment s covers outputs [s*B, s*B + B), B = L - M, and reads input bins
 * [s*B - M/2, s*B - M/2 + L).
 */
int fdas_correlate(const fdas_cf32 *spec_dev, int64_t N, const fdas_cf32 *bank_dev,
                   int K, int M, int L, float *plane_dev, hipStream_t stream);

/*
 * Same as fdas_correlate with an explicit launch shape, for tuning: grid
 * persistent workgroups (0 = as many as the device holds resident, the
 * default; at most 2^20).  The (segment, template) work is split into
 * `grid` contiguous ranges; the plane does not depend on grid.
 */
int fdas_correlate_ex(const fdas_cf32 *spec_dev, int64_t N, const fdas_cf32 *bank_dev,
                      int K, int M, int L, float *plane_dev, int grid,
                      hipStream_t stream);

/*
 * Forward correlation with interbinning (Sec. 3, eq. f-interp and the
 * paragraph after it, which the paper's GPU code applies after the
 * correlation): the Fourier amplitude midway between bins r and r+1 is
 * estimated as (pi/4)(Y[z][r] - Y[z][r+1]).  Output plane2_dev has 2N
 * floats per row, [K][2N] row-major:
 *     plane2[z][2r]   = |Y[z][r]|^2,
 *     plane2[z][2r+1] = |(pi/4)(Y[z][r] - Y[z][r+1])|^2,
 * where Y[z][N] is the same correlation sum one bin past the end (the
 * spectrum is zero outside [0, N)).  Arguments and errors as
 * fdas_correlate; plane2_dev holds K*2N floats, 8-byte aligned.
 */
int fdas_correlate_interbin(const fdas_cf32 *spec_dev, int64_t N, const fdas_cf32 *bank_dev,
                            int K, int M, int L, float *plane2_dev, hipStream_t stream);

/* Same with an explicit number of persistent workgroups (0 = resident). */
int fdas_correlate_interbin_ex(const fdas_cf32 *spec_dev, int64_t N, const fdas_cf32 *bank_dev,
                               int K, int M, int L, float *plane2_dev, int grid,
                               hipStream_t stream);

/*
 * Symmetric bank (Sec. 4.2 notes that the templates of -z are the complex
 * conjugates of those of +z).  On the grid z_k = (k - (K-1)/2) dz with K
 * odd, T[K-1-k][j] = conj(T[k][j]), so the prepared filters satisfy
 * H_{-z}[p] = conj(H_z[(L - p) mod L]): only the (K+1)/2 rows z >= 0 are
 * stored, ((K+1)/2 + 1) * L complex values with the twiddle row last, and
 * the forward reads row -z as the conjugate mirror of row z.  This halves
 * the bank's memory and cache footprint; it removes no transform (for a
 * complex spectrum Y_z and Y_{-z} are inverse transforms of different
 * products).
 *
 * fdas_bank_sym_elems: elements of such a bank (0 if K is even or < 1).
 * fdas_prepare_bank_sym: as fdas_prepare_bank, reading only the taps of the
 *   templates k >= (K-1)/2 (taps_dev still holds all K rows); K must be
 *   odd (else FDAS_INVALID_ARG).  The caller asserts the symmetry above,
 *   which fdas_make_templates' taps satisfy.
 * fdas_correlate_sym(_ex): fdas_correlate(_ex) with such a bank; same plane.
 */
int64_t fdas_bank_sym_elems(int K, int L);
int fdas_prepare_bank_sym(const fdas_cf32 *taps_dev, int K, int M, int L, fdas_cf32 *bank_dev,
                          hipStream_t stream);
int fdas_correlate_sym(const fdas_cf32 *spec_dev, int64_t N, const fdas_cf32 *bank_sym_dev, int K,
                       int M, int L, float *plane_dev, hipStream_t stream);
int fdas_correlate_sym_ex(const fdas_cf32 *spec_dev, int64_t N, const fdas_cf32 *bank_sym_dev,
                          int K, int M, int L, float *plane_dev, int grid, hipStream_t stream);

/*
 * Two-bin Fourier interpolation (Sec. 3: the more accurate alternative to
 * interbinning, which doubles the template and signal resolution before the
 * correlations).  Plane [K][2N] (plane2_dev, 8-byte aligned):
 *     plane2[z][2r]   = |Y[z][r]|^2                     (the plain plane),
 *     plane2[z][2r+1] = |sum_k A[k] conj(R(r + 1/2 - k, z))|^2,
 * the half-bin matched filter over the M bins k in [r - M/2 + 1, r + M/2]
 * (A zero outside [0, N)).  The half-bin sum is a correlation of the kind
 * fdas_correlate computes, with M + 2 taps at offsets j - (M+2)/2 holding
 * R(1/2 - offset, z) (taps 0 and 1 zero), so it runs on the same kernels
 * with a second bank:
 *
 * fdas_make_templates_half: as fdas_make_templates for those K x (M + 2)
 *   half-bin taps (taps_half_dev) and, if bank_half_dev is not NULL, their
 *   bank for segment length L (fdas_bank_elems(K, L) values); needs
 *   M + 2 <= L/2.  Synchronises the stream.
 * fdas_correlate_fourier2(_ex): both planes into plane2_dev in one launch
 *   (both inverse transforms per template on a shared segment FFT, segments
 *   of B = L - M - 2 outputs); bank_dev from fdas_make_templates (M taps),
 *   bank_half_dev from fdas_make_templates_half, same K and L.  Errors as
 *   fdas_correlate.
 */
int fdas_make_templates_half(double zmax, double dz, int M, int L, fdas_cf32 *taps_half_dev,
                             fdas_cf32 *bank_half_dev, hipStream_t stream);
int fdas_correlate_fourier2(const fdas_cf32 *spec_dev, int64_t N, const fdas_cf32 *bank_dev,
                            const fdas_cf32 *bank_half_dev, int K, int M, int L, float *plane2_dev,
                            hipStream_t stream);
int fdas_correlate_fourier2_ex(const fdas_cf32 *spec_dev, int64_t N, const fdas_cf32 *bank_dev,
                               const fdas_cf32 *bank_half_dev, int K, int M, int L,
                               float *plane2_dev, int grid, hipStream_t stream);

/* Bytes of device workspace fdas_correlate_batched needs for nspec spectra
 * (the per-spectrum segment prefix sums), rounded up to 256. */
size_t fdas_batched_workspace_bytes(int nspec);

/*
 * Batched ragged correlation: many spectra of uneven lengths (dedispersion
 * trials x beams) against one shared bank in a single persistent launch.
 * The paper processes independent time series one after another or one per
 * GPU (Sec. 5.1, Sec. 6); here they share one launch so short spectra
 * still fill the device.
 *   specs_dev   : spectra packed back to back, 8-byte aligned; spectrum b is
 *                 specs_dev[offsets[b] .. offsets[b+1]);
 *   offsets_dev : DEVICE array of nspec + 1 int64, non-decreasing; read at
 *                 execution time, so a captured graph can be replayed for new
 *                 batches after the caller rewrites offsets and spectra in
 *                 place;
 *   capacity    : elements specs_dev holds (planes_dev holds K * capacity
 *                 floats), 0 <= capacity <= 2^40.  Since the offsets are read
 *                 on the device, the kernels clamp every offset to
 *                 [0, capacity]: a spectrum reaching past the capacity is
 *                 cut there and a negative length is empty, so no access
 *                 leaves the buffers whatever the offsets hold;
 *   planes_dev  : plane b starts at planes_dev + K * offsets[b], layout
 *                 [K][N_b] row-major (so K * offsets[nspec] floats in all);
 *   ws_dev      : device workspace of ws_bytes >= fdas_batched_workspace_bytes
 *                 (else FDAS_WORKSPACE_TOO_SMALL), 8-byte aligned; its
 *                 contents are scratch.
 * Results are bitwise identical to fdas_correlate on each spectrum with the
 * same L.  nspec = 0 is a no-op.  Launches two kernels on `stream` and makes
 * no host-side wait, allocation or memset, so it can be captured in a graph.
 */
int fdas_correlate_batched(const fdas_cf32 *specs_dev, const int64_t *offsets_dev, int nspec,
                           int64_t capacity, const fdas_cf32 *bank_dev, int K, int M, int L,
                           float *planes_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream);

/*
 * Same with an explicit launch shape (what fdas_autotune_batched chooses):
 *   E    : complex values per lane of the segment transforms, 0 = the
 *          default (4 at L = 256, 8 at L = 512, 16 from L = 1024); 8 and 16
 *          are both available from L = 1024 on, else FDAS_UNSUPPORTED.  A
 *          different E changes the radix plan and so the FP32 rounding of
 *          the plane, not its definition;
 *   grid : persistent workgroups (0 = as many as the device holds resident;
 *          at most 2^20); the plane does not depend on it.
 */
int fdas_correlate_batched_ex(const fdas_cf32 *specs_dev, const int64_t *offsets_dev,
                              int nspec, int64_t capacity, const fdas_cf32 *bank_dev, int K,
                              int M, int L, float *planes_dev, int E, int grid, void *ws_dev,
                              size_t ws_bytes, hipStream_t stream);

/*
 * Allocation-free form of fdas_correlate_batched, for callers that cannot
 * allocate device memory: code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results (bitwise) and
 * launches as fdas_correlate_batched at the default launch shape, without
 * ws_dev / ws_bytes: the per-spectrum segment prefix sums (nspec + 1 int64)
 * live in a fixed device array inside the library, one per GPU, of
 * FDAS_NOALLOC_MAX_SPECTRA + 1 entries (512 KB), held from the first call on
 * that GPU until the process ends.  nspec above FDAS_NOALLOC_MAX_SPECTRA is
 * rejected with FDAS_INVALID_ARG before anything is launched.  The call
 * makes no hipMalloc, hipFree or other allocating call; its first call on a
 * device looks up the array's device address (hipGetSymbolAddress).  Every
 * call on a GPU shares that GPU's array, and the scan rewrites every entry a
 * call reads, so no state carries over between calls; calls that overlap in
 * time on one GPU (other streams, other threads) race on it and must be
 * serialised by the caller.
 */
#define FDAS_NOALLOC_MAX_SPECTRA 65536
int fdas_correlate_batched_noalloc(const fdas_cf32 *specs_dev, const int64_t *offsets_dev,
                                   int nspec, int64_t capacity, const fdas_cf32 *bank_dev, int K,
                                   int M, int L, float *planes_dev, hipStream_t stream);

/* Bytes of device workspace for fdas_correlate_backward(_ex) with the same
 * (N, K, M, L, zchunk; 0 = default), a multiple of 256; 0 for an invalid
 * geometry.  Holds the per-window partial gradients,
 * ceil(K/zchunk) * ceil(N/B) * L + ceil(N/B) * K * M complex values, and
 * up to 2048 / ceil(K M / 64) chunk sums of the taps gradient (K * M FP64
 * complex values each). */
size_t fdas_backward_workspace_bytes(int64_t N, int K, int M, int L, int zchunk);

/*
 * Adjoint of fdas_correlate for the loss Lw = sum_{z,r} w[z][r] P[z][r]
 * (not in the paper; derived from the definition in the header comment),
 * in PyTorch's complex convention grad = dLw/dRe + i dLw/dIm.  With
 * g[z][r] = 2 w[z][r] Y[z][r]:
 *     grad_spec[k]    = sum_z sum_j T[z][j] g[z][k - e_j]
 *     grad_taps[z][j] = sum_r conj(g[z][r]) A[r + e_j].
 *   dLdP_dev      : w, K*N floats [z][r] (4-byte aligned);
 *   grad_spec_dev : N complex outputs, or NULL to skip;
 *   grad_taps_dev : K*M complex outputs, or NULL to skip (the templates
 *                   enter through bank_dev, prepared from them);
 *   ws_dev        : >= fdas_backward_workspace_bytes(N, K, M, L, 0) bytes,
 *                   256-byte aligned; scratch.
 * The complex plane Y is recomputed from the spectrum segment by segment,
 * never stored.  The partial sums of every segment are reduced in FP64 in a
 * fixed order, so results are deterministic.  Both gradients NULL is a
 * no-op; N = 0 writes zero taps gradients.
 */
int fdas_correlate_backward(const fdas_cf32 *spec_dev, int64_t N, const fdas_cf32 *bank_dev,
                            int K, int M, int L, const float *dLdP_dev,
                            fdas_cf32 *grad_spec_dev, fdas_cf32 *grad_taps_dev,
                            void *ws_dev, size_t ws_bytes, hipStream_t stream);

/* Same with an explicit number of templates per workgroup (0 = default);
 * the workspace must be sized with the same zchunk. */
int fdas_correlate_backward_ex(const fdas_cf32 *spec_dev, int64_t N, const fdas_cf32 *bank_dev,
                               int K, int M, int L, const float *dLdP_dev,
                               fdas_cf32 *grad_spec_dev, fdas_cf32 *grad_taps_dev, int zchunk,
                               void *ws_dev, size_t ws_bytes, hipStream_t stream);

/* Gradients a batched adjoint call computes (fdas_backward_batched_workspace_bytes). */
#define FDAS_WANT_SPECTRA 1
#define FDAS_WANT_TAPS 2

/*
 * Bytes of device workspace for fdas_correlate_backward_batched with the
 * same (capacity, nspec, K, M, L, zchunk) and the gradients in `want`
 * (FDAS_WANT_SPECTRA | FDAS_WANT_TAPS); 0 for an invalid geometry.  With W =
 * capacity / (L - M) + nspec (a bound on the batch's windows) and
 * nzc = ceil(K / zchunk): nspec + 1 int64, then nzc * W * L complex values
 * for the spectra's gradient and W * K * M complex values plus up to 2048 /
 * ceil(K M / 64) FP64 chunk sums of K * M for the taps' gradient.
 */
size_t fdas_backward_batched_workspace_bytes(int64_t capacity, int nspec, int K, int M, int L,
                                             int zchunk, int want);

/*
 * Adjoint of fdas_correlate_batched for Lw = sum_b sum_{z,r} w_b[z][r]
 * P_b[z][r] (not in the paper; the single-spectrum adjoint of
 * fdas_correlate_backward applied to every spectrum of the batch), in one
 * launch of a grid fixed by the host's bound on the window count (one
 * workgroup per (window, template chunk) item of all spectra; those past the
 * batch's actual windows exit at once), plus a scan and the FP64
 * reductions; offsets are read on the device, so the call makes no host
 * wait, allocation or memset (for nspec >= 1) and can be captured in a
 * graph.
 *   specs_dev, offsets_dev, nspec, capacity : as fdas_correlate_batched
 *                   (offsets clamped to [0, capacity]);
 *   bank_dev      : prepared bank for (K, M, L);
 *   dLdP_dev      : w, packed like the planes: w_b at dLdP_dev + K *
 *                   offsets[b], [K][N_b] row-major (K * capacity floats);
 *   grad_specs_dev: capacity complex outputs packed like the spectra (bins
 *                   outside every spectrum are set to 0), or NULL;
 *   grad_taps_dev : K*M complex outputs, the taps gradient summed over the
 *                   whole batch in FP64 in a fixed order, or NULL;
 *   zchunk        : templates per work item (0 = default);
 *   ws_dev        : >= fdas_backward_batched_workspace_bytes(capacity,
 *                   nspec, K, M, L, zchunk, want) bytes for the gradients
 *                   requested, 256-byte aligned; scratch.
 * Each spectrum's grad_specs is bitwise the one fdas_correlate_backward_ex
 * gives for that spectrum alone with the same zchunk; grad_taps equals the
 * sum of the single-spectrum taps gradients up to FP32 rounding.  Offsets
 * must be non-decreasing for these results (overlapping ranges give
 * unspecified values but no access outside the buffers).  Both gradients
 * NULL is a no-op; nspec = 0 writes zero gradients.
 */
int fdas_correlate_backward_batched(const fdas_cf32 *specs_dev, const int64_t *offsets_dev,
                                    int nspec, int64_t capacity, const fdas_cf32 *bank_dev, int K,
                                    int M, int L, const float *dLdP_dev,
                                    fdas_cf32 *grad_specs_dev, fdas_cf32 *grad_taps_dev,
                                    int zchunk, void *ws_dev, size_t ws_bytes, hipStream_t stream);

/* Bytes of device workspace fdas_autotune_batched needs: a bank for the
 * largest segment length plus the batched workspace. */
size_t fdas_autotune_workspace_bytes(int K, int nspec);

/* A launch shape of the batched forward and, from the tuner, its time. */
typedef struct {
    int L;            /* segment length */
    int E;            /* complex values per lane of the segment transforms */
    int grid_factor;  /* persistent grid = grid_factor x resident workgroups */
    int grid;         /* that grid as fdas_correlate_batched_ex takes it (0 = resident) */
    int from_cache;   /* 1 if fdas_autotune_batched took the choice from a cache */
    double ms;        /* measured ms per batched call (0 in a candidate list) */
} fdas_tuning;

/* fdas_autotune_batched flags */
#define FDAS_TUNE_NO_CACHE 1   /* neither read nor write the process or file cache */
#define FDAS_TUNE_REFRESH 2    /* time again and replace the cached choice */

/*
 * The launch shapes fdas_autotune_batched times for (K, M), in its order:
 * every supported L from 512 to 8192 with M <= L/2, every E of that L
 * (fdas_correlate_batched_ex) and grid factors 1 and 2.  Writes
 * min(capacity, count) entries (grid = 0, ms = 0) and the full count.
 * Host only.
 */
int fdas_autotune_candidates(int K, int M, fdas_tuning *list, int capacity, int *count);

/* Workgroups of the batched kernel for (L, E, M) the current device holds
 * resident: the grid a call with grid = 0 launches. */
int fdas_batched_resident_grid(int L, int E, int M, int *grid);

/*
 * Autotuner for the batched forward (the paper tunes the segment length and
 * launch shape per card by hand, Sec. 5.1.2): prepares a bank from taps_dev
 * for every candidate L (fdas_autotune_candidates) and times
 * fdas_correlate_batched_ex on the caller's batch for every candidate
 * (L, E, grid) in three rounds (per round one warm-up launch and the mean of
 * three; a candidate's better round counts), and writes the fastest to *out.
 * The choice is cached for the life of the process and in a JSON file
 * ($FDAS_TUNE_CACHE, an empty value disabling it; else
 * $XDG_CACHE_HOME/fdas/autotune.json or ~/.cache/fdas/autotune.json; one
 * entry per line, rewritten atomically), keyed by the device architecture,
 * its compute-unit count, K, M and floor(log2) of the batch's total bins and
 * of nspec; a cached choice is returned without timing (from_cache = 1)
 * unless flags has FDAS_TUNE_REFRESH; FDAS_TUNE_NO_CACHE bypasses both
 * caches.  offsets_dev/capacity as fdas_correlate_batched; planes_dev
 * (K * capacity floats) is scratch for the trials: its contents afterwards
 * are unspecified, on a cache hit as on a miss.  ws_dev holds at least
 * fdas_autotune_workspace_bytes(K, nspec) bytes (256-byte aligned).
 * Synchronises the stream.  Not on the hot path.
 */
int fdas_autotune_batched(const fdas_cf32 *taps_dev, int K, int M, const fdas_cf32 *specs_dev,
                          const int64_t *offsets_dev, int nspec, int64_t capacity,
                          float *planes_dev, void *ws_dev, size_t ws_bytes, int flags,
                          hipStream_t stream, fdas_tuning *out);

/* ---- real-to-complex front end -------------------------------------------- */

/* Bytes of device workspace fdas_r2c needs for n samples (0 if n is not
 * supported): n/2 complex work values. */
size_t fdas_r2c_workspace_bytes(int64_t n);

/*
 * Real-to-complex transform of a time series (Sec. 4.1: the input is an
 * array of n FP32 samples taken to the Fourier domain by a real-to-complex
 * FFT; Sec. 3 lists it as the first processing step):
 *     spec[k] = scale * sum_{t=0}^{n-1} x[t] exp(-2 pi i k t / n),
 *     k = 0 .. n/2   (n/2 + 1 bins, the Nyquist bin included).
 * scale = 1 is the unnormalised transform; 1/sqrt(n) gives bins of unit
 * mean power for unit-variance white noise.  The first n/2 bins are a
 * spectrum for fdas_correlate (N = n/2) or the whole array (N = n/2 + 1).
 *  x_dev     n floats, 8-byte aligned, read only.
 *  n         a power of two in [2^13, 2^27]; else FDAS_UNSUPPORTED.
 *  spec_dev  n/2 + 1 fdas_cf32, 8-byte aligned, fully overwritten (also used
 *            as scratch during the call); must not overlap x_dev or ws_dev.
 *  ws_dev    fdas_r2c_workspace_bytes(n) bytes, 256-byte aligned.
 * Asynchronous on `stream`; no allocation.
 */
int fdas_r2c(const float *x_dev, int64_t n, float scale, fdas_cf32 *spec_dev, void *ws_dev,
             size_t ws_bytes, hipStream_t stream);

/*
 * The same for nseries equal-length time series in one launch per pass (the
 * independent series of a search, e.g. dedispersion trials, whose count
 * processed in real time the paper reports, Sec. 6).  Series b is x_dev[b n .. (b+1) n) and its
 * n/2 + 1 bins go to spec_dev[b (n/2 + 1) ..], so spec_dev holds
 * nseries (n/2 + 1) values; with offsets b (n/2 + 1), b = 0 .. nseries, it
 * is a packed batch for fdas_correlate_batched whose spectra have n/2 + 1
 * bins (the Nyquist bin included).  ws_dev: fdas_r2c_batched_workspace_bytes(n,
 * nseries) bytes, 256-byte aligned.  Each series' bins are bitwise those of
 * fdas_r2c.  nseries in [1, 65535]; errors and alignment as fdas_r2c.
 */
size_t fdas_r2c_batched_workspace_bytes(int64_t n, int nseries);
int fdas_r2c_batched(const float *x_dev, int64_t n, int nseries, float scale,
                     fdas_cf32 *spec_dev, void *ws_dev, size_t ws_bytes, hipStream_t stream);

/* ---- harmonic summing and peak candidates ---------------------------------- */

/*
 * Harmonic sums of the f-fdot plane (Sec. 3: the powers of a pulsed
 * signal's harmonics are added to that of its fundamental before the search
 * for peaks; the paper names the step without a formula).  A constant-fdot
 * signal at (r, z) has its h-th harmonic at (h r, h z), so on a plane
 * P[K][N] with rows z_k = (k - c) dz, c = (K - 1)/2 (fdas_correlate's
 * layout, K odd), the H-fold sum at the fundamental (k, r) is
 *     S_H[k][r] = sum_{h=1}^{H} P[c + h (k - c)][h r],
 * for the fundamentals whose harmonics all lie on the plane: r in
 * [0, N_H), N_H = ceil(N/H), and |k - c| <= floor(c/H), i.e. K_H =
 * 2 floor(c/H) + 1 rows; S_H is stored [K_H][N_H] row-major, its row i
 * being plane row c - floor(c/H) + i.  The sum is formed in FP32 in the
 * order h = 1..H.  The columns may be of any uniform resolution: the
 * interbinned or two-bin plane ([K][2N], half bins) is summed as a plane of
 * 2N columns.
 */

/* K_H and N_H of the H-fold sum (K odd in [1, 4096], H a power of two in
 * [1, 64], N in [0, 2^32]); FDAS_INVALID_ARG otherwise. */
int fdas_harmonic_shape(int64_t N, int K, int H, int *KH, int64_t *NH);

/*
 * S_H of plane_dev [K][N] into sums_dev [K_H][N_H] (fully overwritten).
 * prev_dev: NULL, or the H/2-fold sum of the same plane (H >= 2); then only
 * harmonics H/2 + 1 .. H are read from the plane and added to it, and the
 * result is bitwise the same as from scratch.  Buffers are device float
 * arrays (4-byte aligned); sums_dev must not overlap plane_dev or prev_dev.
 * Asynchronous on `stream`; no allocation.
 */
int fdas_harmonic_sum(const float *plane_dev, int64_t N, int K, int H, const float *prev_dev,
                      float *sums_dev, hipStream_t stream);

/* One candidate: the fundamental's frequency bin, its template row in the
 * plane (z = (row - (K-1)/2) dz) and its H-fold summed power. */
typedef struct {
    int64_t r;
    int32_t row;
    float power;
} fdas_candidate;

/*
 * Candidates of one fold (Sec. 3: the power is compared with a precomputed
 * threshold, and the search is for peaks): the points of S_H (sums_dev,
 * [K_H][N_H] as fdas_harmonic_sum writes it for this N, K, H) whose value
 * exceeds `threshold` and is >= each of its up to 8 neighbours inside the
 * fold.  *count_dev (device unsigned) receives the number of such points;
 * the first min(count, capacity) of them are written to out_dev (device,
 * 8-byte aligned) in no particular order.  The call zeroes *count_dev
 * itself (with a kernel, so it can be captured in a graph).  Asynchronous
 * on `stream`; no allocation.
 */
int fdas_find_candidates(const float *sums_dev, int64_t N, int K, int H, float threshold,
                         fdas_candidate *out_dev, int capacity, unsigned *count_dev,
                         hipStream_t stream);

/*
 * The same over the planes of fdas_correlate_batched (plane b at
 * planes_dev + K * offsets[b], [K][N_b]; offsets_dev the same device array,
 * read at execution time), every spectrum in one launch.  Fold H of
 * spectrum b is stored at sums_dev + K_H * C_H[b] as [K_H][ceil(N_b/H)],
 * with C_H[b] = sum_{b' < b} ceil(N_b'/H) (empty spectra contribute
 * nothing), so sums_dev holds K_H * C_H[nspec] floats; prev_dev (or NULL)
 * is the H/2-fold in the same layout.  ws_dev: at least
 * fdas_harmonic_batched_workspace_bytes(nspec) bytes (8-byte aligned,
 * scratch).  Bitwise equal to fdas_harmonic_sum on each spectrum.  No host
 * wait, allocation or memset: capturable in a graph.
 */
size_t fdas_harmonic_batched_workspace_bytes(int nspec);
int fdas_harmonic_sum_batched(const float *planes_dev, const int64_t *offsets_dev, int nspec,
                              int K, int H, const float *prev_dev, float *sums_dev, void *ws_dev,
                              size_t ws_bytes, hipStream_t stream);

/*
 * Candidates of fold H of every spectrum (sums_dev as written by
 * fdas_harmonic_sum_batched for the same offsets, K, H), as
 * fdas_find_candidates; a record's r is the packed bin index offsets[b] + r,
 * which also names the spectrum.  ws_dev as above.
 */
int fdas_find_candidates_batched(const float *sums_dev, const int64_t *offsets_dev, int nspec,
                                 int K, int H, float threshold, fdas_candidate *out_dev,
                                 int capacity, unsigned *count_dev, void *ws_dev,
                                 size_t ws_bytes, hipStream_t stream);

/*
 * Measurement helpers (not part of the method): streaming passes over device
 * memory that give the bandwidth a plain streaming kernel reaches on the
 * device, against which the correlation's plane write and the harmonic
 * gathers are read beside the published peak.
 *
 * fdas_stream_write: dst_dev[i] = value for i < n (float, device, 16-byte
 * aligned), one pass of 16-byte stores.  fdas_stream_read: reads the n
 * floats of src_dev (16-byte aligned) with non-temporal 16-byte loads and
 * writes FDAS_STREAM_PARTIALS partial sums to sums_dev (device float, one
 * per workgroup, summed in an unspecified order; their total is the sum of
 * the buffer).  n == 0 is valid (the write does nothing, the read writes
 * zeros).  Asynchronous on `stream`; no allocation.
 */
#define FDAS_STREAM_PARTIALS 2048
int fdas_stream_write(float *dst_dev, int64_t n, float value, hipStream_t stream);
int fdas_stream_read(const float *src_dev, int64_t n, float *sums_dev, hipStream_t stream);

/*
 * LDS bank probe (measurement helper, not part of the correlation): the
 * bank rules that the segment transforms' LDS layout is built for were
 * measured with it.  `groups` single-wave workgroups each fill a 64 KB LDS
 * array, then lane l repeats `iters` times one access at element
 * pattern_dev[l] (64 int32 on the device; an element is 8 bytes for
 * mode 0 = 64-bit write and mode 1 = 64-bit read, 16 bytes for
 * mode 2 = 128-bit write; indices are masked into the array, so any pattern
 * stays in bounds), with a wave barrier between repetitions.
 * cycles_dev[g] (int64, `groups` entries) receives workgroup g's loop time
 * in clock64 cycles; sink_dev (64 * groups floats) keeps the reads live.
 * 1 <= iters <= 2^20, 1 <= groups <= 2^16, else FDAS_INVALID_ARG.
 */
int fdas_lds_probe(const int *pattern_dev, int mode, int iters, int groups,
                   long long *cycles_dev, float *sink_dev, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* FDAS_H */
