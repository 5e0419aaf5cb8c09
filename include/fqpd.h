/*
 * fqpd.h -- C ABI of the MI355X (gfx950) ultrafast power-Doppler reconstruction path.
 *
 * Reconstruction hot path of 3D-FQFlow (arXiv 2509.05464): per-element RF of tilted
 * plane-wave transmits on a 2-D matrix array -> RF-to-IQ demodulation -> 3-D delay-and-sum
 * with coherent compounding over transmits (one IQ volume per frame) -> Casorati Gram ->
 * FP64 Hermitian eigendecomposition and rank selection -> SVD clutter filter -> power
 * Doppler.  Beside the SVD filter sits a learned slow-time convolutional filter (BF16
 * training and inference kernels) with the SVD result as its fallback.
 *
 * Conventions (all entry points):
 *  - Array arguments are DEVICE pointers, caller-owned, C-order; complex arrays are
 *    interleaved (re, im) pairs (layout-compatible with torch.complex64/complex128).
 *    Parameter structs (fq_probe, fq_tx, fq_grid, fq_pulse) are HOST pointers.
 *  - Units are SI (m, s, Hz, m/s) and radians.
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null stream).
 *    The library keeps no pointer after return except for work queued on `stream`;
 *    buffers must stay alive until that work completes.  Hot calls never allocate:
 *    the caller supplies workspaces whose sizes the *_workspace_size queries return.
 *  - Return value: FQ_OK or an FQ_E_* status; fq_last_error() gives a thread-local
 *    message for the last failure.  Outputs are undefined after a failure.  Nothing
 *    throws or aborts across the ABI.  Numeric failures detected on the device
 *    (eigensolver non-convergence) are reported through device status words.
 *  - Pointers must be 16-byte aligned (FQ_E_INVALID otherwise).
 *
 * Geometry (shared by every entry point):
 *  - element e = ix + nx_el*iy sits at ((ix-(nx_el-1)/2) pitch_x, (iy-(ny_el-1)/2) pitch_y, 0);
 *  - transmit a is a plane wave with direction u_a = (sin tx, sin ty, sqrt(1 - sin^2 tx - sin^2 ty))
 *    fired so that t = 0 when the first element fires: tau_tx(a, r) = u_a.r/c - min_e u_a.p_e/c;
 *  - receive delay tau_rx(e, r) = |r - p_e| / c;
 *  - voxel v = ix + nx*(iy + ny*iz) is centred at (x0 + ix dx, y0 + iy dy, z0 + iz dz).
 */
#ifndef FQPD_H
#define FQPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FQ_MAX_ANGLES 32
#define FQ_MAX_NT 512
#define FQ_SSM_MAX_MODES 64
#define FQ_GRAM_SCRATCH_BYTES (48u << 20)   /* static scratch of casorati_gram_noalloc, per GPU */

enum { FQ_OK = 0, FQ_E_INVALID = 1, FQ_E_WORKSPACE = 2, FQ_E_HIP = 3, FQ_E_NUMERIC = 4 };
enum { FQ_INTERP_LINEAR = 0, FQ_INTERP_HERMITE = 1 };
enum { FQ_GRAM_FP32 = 0, FQ_GRAM_SPLIT_BF16 = 1, FQ_GRAM_BF16 = 2, FQ_GRAM_SPLIT4_BF16 = 3 };
enum { FQ_CUTOFF_KNEE = -1, FQ_CUTOFF_SSM = -2 };
enum { FQ_DISP_POWER = 0, FQ_DISP_IQ = 1, FQ_DISP_UNIT = 2 };
enum { FQ_MIP_XY = 0, FQ_MIP_XZ = 1, FQ_MIP_YZ = 2 };
enum { FQ_PROBE_LDS_READ = 0, FQ_PROBE_FP32_FMA = 1 };

typedef struct {
    int32_t nx_el, ny_el;     /* regular matrix array, nx_el*ny_el elements */
    double pitch_x, pitch_y;  /* element pitch, m */
    double fc_hz;             /* transmit centre frequency */
    double fs_hz;             /* RF sampling rate */
    double c_mps;             /* speed of sound */
} fq_probe;

typedef struct {
    int32_t n_angles;                     /* 1..FQ_MAX_ANGLES transmits per frame */
    double tilt_rad[FQ_MAX_ANGLES][2];    /* (theta_x, theta_y) of each plane wave */
} fq_tx;

typedef struct {
    int32_t nx, ny, nz;                   /* voxel counts */
    double x0, y0, z0;                    /* centre of voxel (0,0,0), m */
    double dx, dy, dz;                    /* voxel spacing, m */
} fq_grid;

typedef struct {
    double n_cycles;      /* Gaussian envelope FWHM in carrier cycles (2) */
    double trunc_sigmas;  /* pulse support +-trunc_sigmas * sigma (5) */
    double r_ref_m;       /* reference distance of the 1/r receive amplitude (1e-3) */
} fq_pulse;

/* ---------------------------------------------------------------------------------
 * rf_synth -- RF of point scatterers under tilted plane-wave transmits.
 * Weak scattering / linear superposition (Section 2.3) with the analytic echo of a
 * point scatterer: a Gaussian-envelope pulse g(t) = exp(-t^2/2s^2) cos(2 pi fc t),
 * s = n_cycles/(2 sqrt(2 ln 2) fc), zero for |t| > trunc_sigmas*s, delayed by
 * tau_tx + tau_rx and scaled by amp * r_ref/|r - p_e|:
 *     rf[f][a][e][n] (+)= sum_s amp[s] (r_ref/rho) g(n/fs - tau_tx(a, r_s(f)) - rho/c).
 *  pos        float32 [n_frames][n_scat][3] (metres), or [1][n_scat][3] if pos_static;
 *  pos_static 1: every frame sees the same positions; each trace is synthesised once and
 *             written to all frames (the static-tissue reuse of Algorithm 1);
 *  amp        float32 [n_scat] reflectivities;
 *  accumulate 0: rf is overwritten; 1: the echoes are added to rf (RF_total = RF_phantom +
 *             RF_flow of Algorithm 1 by two calls);
 *  rf         float32 [n_frames][n_angles][n_elem][n_samples].
 *  Two evaluations: a pulse cut at trunc_sigmas < 5, or narrower than s*fs = 3.3 samples,
 *  is summed sample by sample as written above (half-support trunc_sigmas*s*fs below 32
 *  samples).  Otherwise the pulse is kept whole (the part beyond 5 s is below 3.7e-6 of
 *  its peak) and its Gaussian envelope is split into two Gaussians (variances ~s^2/3 and
 *  ~2s^2/3): each scatterer adds complex taps to a half-rate trace, which a fixed Gaussian
 *  filter and the carrier turn into rf; the result is within ~4e-6 (relative L2) of the
 *  truncated sum for the 2-cycle pulse, for s*fs up to ~9 samples.
 *  Errors: FQ_E_INVALID for null pointers, non-positive sizes, n_samples > 8192, a pulse
 *  of the first kind whose half-support reaches 32 samples.  n_scat == 0 is valid.
 *  The order in which echoes are summed depends on scheduling, so results agree with a
 *  serial sum to FP32 rounding, not bit for bit.
 * ------------------------------------------------------------------------------- */
int rf_synth(const fq_probe* probe, const fq_tx* tx, const fq_pulse* pulse, int32_t n_frames,
             int64_t n_scat, const float* pos, int32_t pos_static, const float* amp,
             int32_t n_samples, int32_t accumulate, float* rf, void* stream);

/* ---------------------------------------------------------------------------------
 * fd_synth -- frequency-domain RF synthesis (Appendix D, Eq. 1 and Eq. 2; Algorithm 2):
 * every scatterer is a monopole; per frequency sample f_j = j df (df = fs / N,
 * N = n_samples + 2 ceil(6 s fs), s the pulse's Gaussian sigma) the element response is
 *   H_e(s, f) = sum over the v = n_sub_x n_sub_y sub-elements (centres of a regular
 *               subdivision of the w_x x w_y element; the coherent sum of Eq. 2) of
 *               (r_ref / r) e^{(i k - alpha) r} sinc(k b_x u_x) sinc(k b_y u_y),
 *   k = 2 pi f / c, b the sub-element half-widths, u the direction cosines towards the
 *   scatterer, sinc(x) = sin(x)/x (w = 0: no directivity), alpha from atten_db_cm_mhz;
 * transmit a gives the field T_a(s, f) = sum_e W_e e^{i 2 pi f dtau_ae} H_e(s, f) at
 * scatterer s (dtau of the plane-wave law of rf_synth, W = apod or 1), the echo at element
 * m is P_a(m, f) = sum_s H_m(s, f) R_s T_a(s, f), and
 *   rf[f][a][m][t] (=, or += with accumulate) = 2 Re sum_j q_j S(f_j) df P_a(m, f_j) e^{-i 2 pi j t / N}
 * with S the Fourier transform of the Gaussian pulse of rf_synth (q = 1/2 at j = 0 and
 * N/2) over the samples j whose S is at least spectral_floor x max S.  No elevation lens
 * (matrix array).  Scatterers with z <= 0 are ignored.
 *  pos, pos_static, amp, n_samples, accumulate, rf: as rf_synth (static scatterers are
 *     transformed once and written to every frame);
 *  apod  float32 [n_elem] transmit apodization, or NULL (all 1);
 *  ws    workspace; the scatterers are processed in blocks sized to fit it (the memory
 *        partition of Algorithm 2): fd_workspace_size(..., B) bytes hold blocks of B
 *        scatterers (B >= 256 is the minimum); results do not depend on the block size
 *        beyond FP32 summation order.
 *  FP64 geometry and phases at the start of every 4-frequency chunk, FP32 stepping and
 *  accumulation.  Errors: FQ_E_INVALID (parameters, band over 4096 samples),
 *  FQ_E_WORKSPACE.
 * ------------------------------------------------------------------------------- */
typedef struct {
    double elem_width_x, elem_width_y;   /* element size, m (0: point elements) */
    int32_t n_sub_x, n_sub_y;            /* sub-elements per element, product 1..64 */
    double atten_db_cm_mhz;              /* attenuation, dB / (cm MHz); 0: lossless */
    double spectral_floor;               /* frequency samples kept: S >= floor x max S */
} fq_fd_params;
size_t fd_workspace_size(const fq_probe* probe, const fq_tx* tx, const fq_pulse* pulse,
                         const fq_fd_params* fd, int32_t n_samples, int64_t scatterers_per_block);
int fd_synth(const fq_probe* probe, const fq_tx* tx, const fq_pulse* pulse, const fq_fd_params* fd,
             int32_t n_frames, int64_t n_scat, const float* pos, int32_t pos_static,
             const float* amp, const float* apod, int32_t n_samples, int32_t accumulate, void* ws,
             size_t ws_bytes, float* rf, void* stream);

/* ---------------------------------------------------------------------------------
 * das_beamform -- rf2iq then delay-and-sum with coherent compounding (Section 2.4.1,
 * Algorithm 3: per-transmit delay application reused for every frame, mean over
 * transmits, voxels processed independently in chunks).
 *  rf2iq:  b[n] = 2 sum_{k=-16..16} h_k rf[n-k] exp(-i 2 pi fc (n-k)/fs), rf = 0 outside
 *          [0, T); h_k = Hann(33) windowed sinc with cutoff fc, unit DC gain.
 *  DAS:    x = fs (tau_tx(a, r_v) + tau_rx(e, r_v)), n = floor(x), alpha = x - n;
 *          linear  B = (1-alpha) b[n] + alpha b[n+1];
 *          hermite B = Catmull-Rom cubic on b[n-1..n+2];  taps outside [0, T) read 0;
 *          iq[f][v] = (1/A) sum_a sum_e B_{f,a,e} exp(+i 2 pi fc x / fs).
 *  rf     float32 [n_frames][n_angles][n_elem][n_samples];
 *  iq     complex64 [n_frames][n_vox] (the Casorati matrix, frame-major);
 *  ws     device workspace of ws_bytes >= das_workspace_size(..., minimum=1); with
 *         das_workspace_size(..., minimum=0) bytes all frames are demodulated in one pass,
 *         otherwise frame blocks are processed in turn (results are identical).
 *  Errors: FQ_E_INVALID (null/misaligned pointers, bad sizes, unsupported geometry: the
 *  per-tile delay window must fit on chip), FQ_E_WORKSPACE (ws too small).
 * ------------------------------------------------------------------------------- */
size_t das_workspace_size(const fq_probe* probe, const fq_tx* tx, int32_t n_frames,
                          int32_t n_samples, int32_t minimum);
int das_beamform(const fq_probe* probe, const fq_tx* tx, const fq_grid* grid, int32_t n_frames,
                 int32_t n_samples, const float* rf, int32_t interp, void* ws, size_t ws_bytes,
                 float* iq, void* stream);

/* The two stages of das_beamform, for callers that keep the whole baseband resident
 * (ws_bytes >= das_workspace_size(..., minimum=0)):
 *  das_demodulate -- rf2iq of every trace into ws (Algorithm 3, "convert to IQ");
 *  das_delay_sum  -- delay-and-sum with coherent compounding from ws into iq
 *                    (Algorithm 3, "apply delays" and "average over transmits").
 * das_beamform(...) == das_demodulate(...) followed by das_delay_sum(...), bit for bit.
 * Errors as das_beamform; FQ_E_WORKSPACE if ws cannot hold all frames. */
int das_demodulate(const fq_probe* probe, const fq_tx* tx, int32_t n_frames, int32_t n_samples,
                   const float* rf, void* ws, size_t ws_bytes, void* stream);
int das_delay_sum(const fq_probe* probe, const fq_tx* tx, const fq_grid* grid, int32_t n_frames,
                  int32_t n_samples, int32_t interp, const void* ws, size_t ws_bytes, float* iq,
                  void* stream);

/* Host-only query (no device work): the delay rows per (transmit, element) that
 * das_delay_sum stages on chip for one 16 x 16 x 2-voxel tile.  The bound is the
 * tile's diameter (receive distances are 1-Lipschitz in the voxel position) plus the
 * transmit-plane spread over the tile, in samples, plus 8 rows of margin for the
 * interpolation taps and the integer/fraction splits, rounded up to a multiple of 8.
 * Every tap of every voxel of a tile falls inside its window.  Returns -1 (and sets
 * the error text) for invalid arguments. */
int das_window_rows(const fq_probe* probe, const fq_tx* tx, const fq_grid* grid);

/* ---------------------------------------------------------------------------------
 * casorati_gram -- G = S^H S for the Casorati matrix S[v][f] = iq[f][v] (Section 2.4.2:
 * the SVD clutter filter works on S; its right singular vectors and squared singular
 * values are the eigenpairs of G).
 *  gram_mode FQ_GRAM_FP32:       FP32 matrix-core products, FP32 accumulation within
 *                                64-voxel blocks, FP64 accumulation across blocks;
 *            FQ_GRAM_SPLIT_BF16: each FP32 operand split as hi = bf16(x), lo = bf16(x - hi);
 *                                three BF16 matrix-core products hi*hi + hi*lo + lo*hi, FP32
 *                                accumulation, FP64 across blocks;
 *            FQ_GRAM_SPLIT4_BF16: hi*hi + hi*lo + lo*hi + lo*lo: the three-product form
 *                                omits sum lo lo^H, a PSD bias of ~2^-18 of trace(G) that
 *                                swamps eigenvalues below that level; four products keep
 *                                the whole spectrum (the filter's projector is fine either way);
 *            FQ_GRAM_BF16:       hi*hi only (negative control).
 *  iq    complex64 [n_t][n_vox];  gram complex128 [n_t][n_t] (full Hermitian matrix).
 *  Errors: FQ_E_INVALID (n_t < 1 or > FQ_MAX_NT, n_vox < 1), FQ_E_WORKSPACE.
 * ------------------------------------------------------------------------------- */
size_t gram_workspace_size(int64_t n_vox, int32_t n_t, int32_t gram_mode);
int casorati_gram(const float* iq, int64_t n_vox, int32_t n_t, int32_t gram_mode, void* ws,
                  size_t ws_bytes, double* gram, void* stream);

/* casorati_gram_noalloc -- casorati_gram for callers that cannot allocate device memory
 * (work recorded under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): no workspace argument and no allocation of any kind; the partial tiles
 * live in a static device array of FQ_GRAM_SCRATCH_BYTES (48 MiB) that the library holds on
 * each GPU it runs on until the process ends (its address is looked up on the first call
 * on a device).  Same arguments, arithmetic and result as casorati_gram, except that the
 * voxel range is split into fewer parts when the partial tiles would not fit, so the
 * FP64 sums can differ from casorati_gram's in the last bits.  The array holds at least
 * 8 voxel ranges of partial tiles (FP64, 2 x 32 x 32 per tile: Re G, Im G) for every n_t
 * up to FQ_MAX_NT (136 tiles at n_t = 512: 17.8 MB).
 * Every call on a GPU shares that GPU's array and leaves it holding its partial tiles:
 * calls that overlap on one GPU (different streams, or threads) race and must be
 * serialised by the caller.
 *  Errors: as casorati_gram (FQ_E_INVALID also when n_t needs more scratch than the
 *  array holds); FQ_E_HIP if the array's device address cannot be looked up. */
int casorati_gram_noalloc(const float* iq, int64_t n_vox, int32_t n_t, int32_t gram_mode,
                          double* gram, void* stream);

/* ---------------------------------------------------------------------------------
 * svd_clutter_filter -- eigendecomposition of G in FP64 on the GPU (Householder
 * tridiagonalisation; every eigenvalue by multisection on Sturm counts; the K wanted
 * eigenvectors by inverse iteration, orthogonalised inside clusters of close eigenvalues;
 * back-transformation), rank selection, projection and power Doppler on the matrix cores
 * (Section 2.4.2; Section 3.2 marks the cutoff on the singular-value curve).
 *  cutoff >= 0: K = cutoff; cutoff == FQ_CUTOFF_KNEE (-1): knee rule on the dB spectrum
 *     d_k = 10 log10(max(l_k, 1e-6 l_1)/l_1) (read down to -60 dB, the dynamic range over
 *     which power Doppler is shown in Sections 3.1 and 3.3), chord l from (1, d_1) to (N, d_N),
 *     k* = argmax_{k in [2, N/2]} (chord_k - d_k) (first on ties), K = clamp(k*-1, 1, N/2-1);
 *  cutoff == FQ_CUTOFF_SSM (-2): K = the tissue rank that spatial_similarity (below) reads
 *     from the leading M = min(n_t, 64) spatial modes (K <= M/2).
 *  S_f = S - (S V_K) V_K^H (explicit subtraction);  pd[v] = (1/N_t) sum_f |S_f[v][f]|^2.
 *     With iq_filt NULL and K <= 16, pd is the same sum taken as the FP64 difference
 *     ||s_v||^2 - ||s_v V_K||^2 (s_v the voxel's row of S; V_K has orthonormal columns),
 *     from one read of S, clamped at 0.
 *  iq       complex64 [n_t][n_vox];  gram complex128 [n_t][n_t] from casorati_gram;
 *  iq_filt  complex64 [n_t][n_vox] or NULL;  pd float32 [n_vox] or NULL;
 *  sigma    float64 [n_t] singular values, descending (device);
 *  k_used   int32 [1] (device): the K applied;
 *  status   int32 [1] (device) or NULL: 0 ok, FQ_E_NUMERIC if an inverse-iteration vector
 *           vanished or overflowed (outputs are then undefined).
 *  K is limited to 64 (FQ_E_INVALID for a larger fixed cutoff; the knee result is
 *  clamped to 64 and the status word set to FQ_E_NUMERIC).
 * ------------------------------------------------------------------------------- */
/* svd_workspace_size covers every cutoff mode (the FQ_CUTOFF_SSM pass included). */
size_t svd_workspace_size(int64_t n_vox, int32_t n_t);
int svd_clutter_filter(const float* iq, int64_t n_vox, int32_t n_t, const double* gram,
                       int32_t cutoff, void* ws, size_t ws_bytes, float* iq_filt, float* pd,
                       double* sigma, int32_t* k_used, int32_t* status, void* stream);

/* svd_filter_apply -- the last stage of svd_clutter_filter alone (Section 2.4.2: S_f and
 * the power Doppler above, same kernels, same results bit for bit), on the V_K and K that
 * a svd_clutter_filter call on the same workspace left there (that call may pass NULL for
 * iq_filt and pd: it then stops after the eigendecomposition and the cutoff).  It lets the
 * eigendecomposition of one ensemble run on one stream while another stream forms the next
 * ensemble's Gram; order the two calls with an event.
 *  iq       complex64 [n_t][n_vox], the ensemble whose Gram was decomposed;
 *  ws       the workspace of that call, unchanged since (n_t the same, ws_bytes at least
 *           svd_workspace_size's figure without the SSM part);
 *  k_used   int32 [1] (device), as written by that call;
 *  iq_filt / pd  as above; at least one of them non-NULL (FQ_E_INVALID otherwise).
 * Errors: FQ_E_INVALID for bad sizes or pointers, FQ_E_WORKSPACE for a short workspace. */
int svd_filter_apply(const float* iq, int64_t n_vox, int32_t n_t, const void* ws, size_t ws_bytes,
                     const int32_t* k_used, float* iq_filt, float* pd, void* stream);

/* eigendecomposition only, every eigenvector (implicit QL with Wilkinson shifts on the
 * tridiagonal matrix, the rotations replayed on the identity): lam float64 [n_t]
 * descending (clamped >= 0), vecs complex128 [n_t][n_t] with column k the eigenvector of
 * lam[k], or NULL for eigenvalues only.  Same workspace as above; the status word is
 * FQ_E_NUMERIC if the QL iteration did not converge within 60 iterations per eigenvalue. */
int hermitian_eig(const double* gram, int32_t n_t, void* ws, size_t ws_bytes, double* lam,
                  double* vecs, int32_t* status, void* stream);

/* ---------------------------------------------------------------------------------
 * spatial_similarity -- the spatial-similarity matrix (SSM) of the singular-value
 * analyses of Section 3: correlation coefficients, over voxels, between the magnitudes of
 * the spatial modes (left singular vectors) U_k = S V_k / sigma_k, and the tissue rank
 * read from it.  The scale 1/sigma_k does not change a correlation, so |S V_k| is used.
 *   C_jk = cov_v(|U_j|, |U_k|) / (std_v |U_j| std_v |U_k|), clipped to [-1, 1];
 *          a mode whose magnitude does not vary over the voxels gets NaN.
 *   Tissue rank (the paper marks it by eye at the end of the leading block of mutually
 *   similar modes): mode k >= 1 joins the block while a_k > b_k,
 *          a_k = mean_{i<k} C_ik,  b_k = mean_{k<j<M} C_kj;
 *   K = the first k in [1, min(M-2, M/2)] that does not join (NaN does not join), else
 *   max(1, M/2).
 *  iq       complex64 [n_t][n_vox];
 *  vecs     complex128 [n_t][n_t], column k the k-th right singular vector (descending),
 *           as hermitian_eig writes it; columns 0 .. n_modes-1 are read;
 *  n_modes  M, 2 .. min(n_t, FQ_SSM_MAX_MODES);
 *  ssm      float64 [n_modes][n_modes] (device);
 *  k_tissue int32 [1] (device) or NULL.
 *  |U| is formed with FP32 matrix-core products and never stored; the moments are
 *  accumulated in FP64 and reduced in a fixed order (deterministic).
 *  Errors: FQ_E_INVALID (sizes, pointers), FQ_E_WORKSPACE.
 * ------------------------------------------------------------------------------- */
size_t ssm_workspace_size(int64_t n_vox, int32_t n_t);
int spatial_similarity(const float* iq, int64_t n_vox, int32_t n_t, const double* vecs,
                       int32_t n_modes, void* ws, size_t ws_bytes, double* ssm,
                       int32_t* k_tissue, void* stream);

/* ---------------------------------------------------------------------------------
 * power_doppler -- pd[v] = (1/n_t) sum_f |iq[f][v]|^2 (Section 2.4.2 power Doppler map).
 *  iq complex64 [n_t][n_vox]; pd float32 [n_vox].
 * ------------------------------------------------------------------------------- */
int power_doppler(const float* iq, int64_t n_vox, int32_t n_t, float* pd, void* stream);

/* ---------------------------------------------------------------------------------
 * display_db -- log compression over a dynamic range (Section 2.4.2: B-mode and uPDI
 * volumes are log-compressed and shown over a dynamic range; the results use 75 dB for
 * B-mode and 60 dB for power Doppler).
 *   p   = in[i] (kind FQ_DISP_POWER: float32 power values such as PD, >= 0) or
 *         |in[i]|^2 (kind FQ_DISP_IQ: complex64 IQ, so that 10 log10 p = 20 log10 |IQ|);
 *   out[i] = max(-dr_db, 10 log10(p / max_j p_j)) (float32 [n]); an all-zero input, and
 *         zero entries, are shown at -dr_db.  NaN inputs are not supported.
 *   kind | FQ_DISP_UNIT gives grey levels instead: out[i] = 1 + (the dB value) / dr_db,
 *         in [0, 1] (the floor at 0, the peak at 1).
 *  ws     workspace of display_workspace_size(n) bytes (block maxima);
 *  peak   float32 [1] (device) receives max_j p_j, or NULL.
 * mip -- maximum-intensity projection of vol[iz][iy][ix] (x fastest, the voxel order of
 *   fq_grid) onto a plane: FQ_MIP_XY -> out[ny][nx] (max over z), FQ_MIP_XZ -> out[nz][nx]
 *   (max over y), FQ_MIP_YZ -> out[nz][ny] (max over x).  Exact (a maximum has no
 *   rounding); apply it to PD or to display_db output alike (the logarithm is monotonic).
 * ------------------------------------------------------------------------------- */
size_t display_workspace_size(int64_t n);
int display_db(const float* in, int64_t n, int32_t kind, float dr_db, void* ws, size_t ws_bytes,
               float* out, float* peak, void* stream);
int mip(const float* vol, int32_t nx, int32_t ny, int32_t nz, int32_t plane, float* out,
        void* stream);

/* ---------------------------------------------------------------------------------
 * image_quality -- MSE, PSNR and SSIM of img against ref (Section 2.4.3; applied to the
 * maximum-intensity projections), both float32 [ny][nx] (device), nx, ny >= 11.
 *   MSE = mean (img - ref)^2;  PSNR = 10 log10(data_range^2 / MSE) (+inf when MSE = 0);
 *   SSIM (Wang et al., IEEE TIP 2004): 11 x 11 Gaussian window, sigma 1.5, weights summing
 *   to 1, K1 = 0.01, K2 = 0.03 (C = (K data_range)^2), window-weighted moments, mean over
 *   the positions where the window lies inside the image.
 *  out float64 [3] (device): MSE, PSNR, SSIM.  FP64 throughout, fixed reduction order.
 * ------------------------------------------------------------------------------- */
int image_quality(const float* img, const float* ref, int32_t nx, int32_t ny, double data_range,
                  double* out, void* stream);

/* ---------------------------------------------------------------------------------
 * Learned slow-time clutter filter.  Per voxel series s = iq[:, v]:
 *   x = [Re, Im](s) / r,  r = sqrt(mean_f |s_f|^2 + eps);
 *   h1 = GELU(conv9(x; W1[32][2][9], b1)), h2 = GELU(conv9(h1; W2[32][32][9], b2)),
 *   h3 = GELU(conv9(h2; W3[32][32][9], b3)), y = W4[2][32] h3 + b4;
 *   conv9(z)[o][t] = b[o] + sum_i sum_{k<9} W[o][i][k] z[i][t+k-4] (zeros outside [0, T));
 *   GELU(z) = z/2 (1 + erf(z/sqrt 2)); blood estimate s_b = r (y0 + i y1).
 * Parameter vector (19170 entries): W1 | b1 | W2 | b2 | W3 | b3 | W4 | b4 (row-major).
 * Weights are used in BF16 (w_bf16, RNE copies kept by lcf_adam_step), biases in FP32
 * (w), activations are stored in BF16, every accumulation is FP32.
 * ------------------------------------------------------------------------------- */
#define LCF_N_PARAM 19170
/* act workspace bytes for training on n_series series of n_t frames */
size_t lcf_act_size(int64_t n_series, int32_t n_t);

/*  x      complex64 [n_t][n_series] (frame-major, like iq);
 *  act    bf16 activation store of lcf_act_size bytes, or NULL (inference);
 *  y      complex64 [n_t][n_series] blood estimate, or NULL;
 *  pd     float32 [n_series] power Doppler of the estimate, or NULL. */
int lcf_forward(const float* w, const uint16_t* w_bf16, const float* x, int64_t n_series,
                int32_t n_t, float eps, uint16_t* act, float* y, float* pd, void* stream);

/*  After lcf_forward(..., act, ...) on the same x: gradient of
 *  loss = mean over (series, channel, t) of (y - [Re, Im](target)/r)^2.
 *  target complex64 [n_t][n_series]; act is consumed (the dz of each layer overwrites its
 *  pre-activation, and its tail holds per-wave gradient partials, reduced in a fixed
 *  order so the gradient is deterministic); grad float32 [19170] (overwritten);
 *  loss float32 [1] (device, overwritten). */
int lcf_backward(const float* w, const uint16_t* w_bf16, const float* x, const float* target,
                 int64_t n_series, int32_t n_t, float eps, uint16_t* act, float* grad,
                 float* loss, void* stream);

/*  Adam with bias correction on FP32 master weights; refreshes the BF16 copy.
 *  step is 1-based. */
int lcf_adam_step(float* w, uint16_t* w_bf16, float* m, float* v, const float* grad,
                  int32_t n_param, float lr, float beta1, float beta2, float eps, int32_t step,
                  void* stream);

/*  Gather training series: dst[t][b] = src[idx[b] / n_vox][t][idx[b] % n_vox]
 *  (src complex64 [n_vol][n_t][n_vox]; idx int64 [batch], device). */
int lcf_gather(const float* src, int64_t n_vox, int32_t n_t, int64_t n_vol, const int64_t* idx,
               int64_t batch, float* dst, void* stream);

/*  SVD fallback judge: D = 10 log10(sum (pd_l - pd_s)^2 / sum pd_s^2).  If D > tau_db or
 *  pd_l holds a non-finite value, out = pd_s and flag = 1; otherwise out = pd_l, flag = 0.
 *  d_db float32 [1] receives D (device).  ws >= fallback_workspace_size(n). */
size_t fallback_workspace_size(int64_t n);
int lcf_fallback(const float* pd_l, const float* pd_s, int64_t n, float tau_db, void* ws,
                 size_t ws_bytes, float* out, int32_t* flag, float* d_db, void* stream);

/* ---------------------------------------------------------------------------------
 * fq_workspace_size -- one query for every workspace the library takes.  Algorithm 3
 * takes the available memory as an input and partitions the work to fit it; here every
 * workspace is caller-owned, and this call gives its exact size for the given shapes.
 *  which   FQ_WS_DAS       das_beamform / das_demodulate / das_delay_sum with every frame
 *                          demodulated in one pass       (reads probe, tx, n_t, n_samples);
 *          FQ_WS_DAS_MIN   das_beamform's smallest workspace (one block of 8 frames at a
 *                          time; results identical)        (probe, tx, n_t, n_samples);
 *          FQ_WS_GRAM      casorati_gram                   (n = voxels, n_t, gram_mode);
 *          FQ_WS_SVD       svd_clutter_filter and hermitian_eig, every cutoff mode
 *                                                          (n = voxels, n_t);
 *          FQ_WS_SSM       spatial_similarity              (n = voxels, n_t);
 *          FQ_WS_FD        fd_synth with blocks of n scatterers
 *                                                          (probe, tx, pulse, fd, n, n_samples);
 *          FQ_WS_DISPLAY   display_db                      (n = values);
 *          FQ_WS_FALLBACK  lcf_fallback                    (n = values);
 *          FQ_WS_LCF_ACT   the activation store of lcf_forward / lcf_backward
 *                                                          (n = series, n_t);
 *  params  HOST pointer to an fq_ws_query; fields a query does not read are ignored.
 *  Returns the byte count (the same number as the per-call query named above), or 0 for
 *  an unknown `which`, a NULL params or NULL struct pointer it needs, or sizes the entry
 *  point would reject.  Pure host arithmetic: no device is touched.
 * ------------------------------------------------------------------------------- */
enum { FQ_WS_DAS = 0, FQ_WS_DAS_MIN = 1, FQ_WS_GRAM = 2, FQ_WS_SVD = 3, FQ_WS_SSM = 4, FQ_WS_FD = 5,
       FQ_WS_DISPLAY = 6, FQ_WS_FALLBACK = 7, FQ_WS_LCF_ACT = 8 };
typedef struct {
    const fq_probe* probe;        /* FQ_WS_DAS, FQ_WS_DAS_MIN, FQ_WS_FD */
    const fq_tx* tx;              /* FQ_WS_DAS, FQ_WS_DAS_MIN, FQ_WS_FD */
    const fq_pulse* pulse;        /* FQ_WS_FD */
    const fq_fd_params* fd;       /* FQ_WS_FD */
    int64_t n;                    /* voxels, values, series or scatterers per block (see which) */
    int32_t n_t;                  /* frames */
    int32_t n_samples;            /* RF samples per trace */
    int32_t gram_mode;            /* FQ_GRAM_* */
} fq_ws_query;
size_t fq_workspace_size(int32_t which, const void* params);

/* ---------------------------------------------------------------------------------
 * roof_probe -- measurement helper, not a step of the path: the on-chip ceilings the
 * kernels are priced against.  FQ_PROBE_LDS_READ: every thread of n_blocks workgroups of
 * 256 reads 8 x iters 16-byte LDS slots (conflict-free; 64 KB buffer per workgroup), so
 * the launch moves n_blocks * 256 * 128 * iters bytes from LDS to registers;
 * FQ_PROBE_FP32_FMA: every thread runs 8 independent FMA chains of 16 * iters steps
 * (n_blocks * 256 * 256 * iters FLOP).  The caller times the launch on `stream`.
 *  out   float32 [n_blocks * 256] (folded results, so nothing is optimised away).
 *  Errors: FQ_E_INVALID for a bad selector, sizes or pointer. */
int roof_probe(int32_t which, int32_t n_blocks, int32_t iters, float* out, void* stream);

/* Library identification and the thread-local message of the last failure. */
int fq_version(void);

const char* fq_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FQPD_H */
