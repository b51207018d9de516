/*
 * mnfpty — HDR-fused far-field ptychography on AMD MI355X (gfx950).
 *
 * C ABI of libmnfpty.so.  Every array argument is a plain pointer; the
 * comment on each argument says whether it lives in device (HBM) or host
 * memory, its element type and its C-contiguous row-major shape.  The caller
 * owns every buffer it passes; the library never returns memory.  A context
 * owns only its internal scratch (grown on demand and reused), FFT twiddle
 * tables and staging copies of small host arrays.
 *
 * All compute calls are asynchronous on the given stream (a hipStream_t
 * passed as void*, NULL = the device's null stream).  Host arrays are copied
 * before the call returns, so the caller may reuse them at once.  Calls on
 * one context must not overlap in time from several host threads.
 *
 * Errors: every int-returning call returns 0 or one of the negative codes
 * below and never prints, throws or exits.  mnf_last_error() returns a
 * human-readable message for the last failing call on that context.
 *
 * Complex numbers are interleaved {float re, im} (the layout of
 * torch.complex64 / std::complex<float>).
 */
#ifndef MNFPTY_H
#define MNFPTY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MNF_OK            0
#define MNF_EINVAL       -1   /* bad argument: null pointer, size <= 0, window outside the object, ... */
#define MNF_EUNSUPPORTED -2   /* detector size without a compiled FFT plan, too many levels/exposures */
#define MNF_EHIP         -3   /* a HIP runtime call failed; the message holds hipGetErrorString */
#define MNF_ENOMEM       -4   /* scratch allocation failed */
#define MNF_ENONFINITE   -5   /* a call produced a non-finite error, loss, object or probe value (from mnf_status) */
#define MNF_EDIVERGED    -6   /* an iteration's Fourier error exceeded max(10 x the call's first, 1e-6) (from mnf_status) */

typedef struct { float re, im; } mnf_c64;
typedef struct mnf_ctx mnf_ctx;

/* Create a context bound to HIP device `hip_device`.  *out receives the
 * context (NULL on failure).  Returns MNF_OK, MNF_EINVAL or MNF_EHIP. */
int mnf_create(mnf_ctx** out, int hip_device);

/* Release a context and its scratch.  Waits for the device first.  NULL is a no-op. */
void mnf_destroy(mnf_ctx* ctx);

/* Message of the last failing call on ctx ("" if none).  Valid until the next call on ctx.
 * With ctx == NULL: the message of the last call on the calling thread made without a
 * context (mnf_create, ptycho_plan_info with ctx NULL); "" after a success. */
const char* mnf_last_error(const mnf_ctx* ctx);

/* Numerical status of the work issued on ctx (a guard the paper does not
 * discuss; iterative phase retrieval can blow up on inconsistent data).
 * Kernels record, without synchronising, (1) a non-finite per-iteration
 * Fourier error or loss, or a non-finite object or probe element at the end
 * of a reconstruction call, and (2) divergence: an iteration whose Fourier
 * error (when err_out is given) exceeds max(10 x the first iteration of the
 * same call, 1e-6).  mnf_status waits for `stream`, returns MNF_ENONFINITE
 * (which takes precedence) or MNF_EDIVERGED if either was recorded since the
 * previous mnf_status on ctx, MNF_OK otherwise, and clears the record.  Work
 * still running on other streams may be reported by a later call. */
int mnf_status(mnf_ctx* ctx, void* stream);

/* Detector sizes with a compiled FFT plan: writes up to `cap` sizes to
 * `sizes` (host int32) and returns how many exist. */
int mnf_supported_sizes(int32_t* sizes, int cap);

/* ------------------------------------------------------------------------
 * Multi-scale non-linear fusion of exposure brackets
 * (Methods 3.4: exposure quality Eq. 5, pyramids Eqs. 6-7, modulation and
 * quantisation Eq. 8, per-exposure reconstruction and accumulation
 * Eqs. 9-10; the bracket itself is Eq. 1).
 *
 * For every scan position j, with I_k = raw[j][k] (detector counts):
 *   I_bar_k   = clamp((I_k - dark) / (sat - dark), 0, 1)
 *   W_k       = exp(-(I_bar_k - mu)^2 / (2 sigma^2)) / sum_k' (same)
 *   I_tilde_k = (I_k - dark) * t[0] / t[k]   (radiometric = 1)
 *             = I_bar_k                       (radiometric = 0)
 *   G_l: 5-tap binomial reduce, reflect-101 borders; U: zero-insert + 2 w_G
 *   out = collapse over l = L..0 of
 *         sum_k Q_{l,k}(G_l[W_k] (G_l[I_tilde_k] - U(G_{l+1}[I_tilde_k])))
 *         with base sum_k G_L[W_k] G_L[I_tilde_k],
 *   Q_{l,k}(x) = step * rint(x / step), step = delta[l] * t[0] / t[k]
 *   (radiometric) or delta[l] / (sat - dark) (literal); step 0 = identity.
 * With contrast_exp = e > 0 (not part of the paper's method, which weighs by
 * Eq. 5 alone) each raw weight is first multiplied by (C_k + 1e-6)^e,
 * C_k = |I_bar_k(y-1,x) + I_bar_k(y+1,x) + I_bar_k(y,x-1) + I_bar_k(y,x+1)
 *        - 4 I_bar_k(y,x)| with reflect-101 neighbours (the pixel itself along
 * an axis of length one); where every exposure is flat the Eq. 5 weights
 * remain.  This path stores the level-0 weights in scratch (4 K H W bytes
 * per position) and uses the per-pixel kernels.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t levels;        /* L band-pass levels (0..12); H and W must be divisible by 2^L, and H, W >= 2^(L+1) */
    float   mu;            /* weight centre in normalised units (paper's mu) */
    float   sigma;         /* weight width (paper's sigma), > 0 */
    float   sat;           /* detector full scale in ADU, > dark */
    float   dark;          /* dark level in ADU */
    float   delta[16];     /* quantisation step per level in ADU, l = 0 finest; 0 disables */
    int32_t radiometric;   /* 1: fuse counts scaled to the shortest exposure; 0: fuse I_bar */
    float   contrast_exp;  /* optional contrast factor, in [0, 4]; 0 (the paper's Eq. 5 weight) disables it */
} mnf_fuse_params;

/* raw        device uint16 [J][K][H][W]   exposure brackets
 * t          host   float  [K]            exposure times, t[0] the reference (> 0)
 * fused      device float  [J][H][W]      output I_MNF, same (detector-centred) layout as raw
 * weights_out device float [J][K][H][W]  normalised weights W_k, or NULL
 * K <= 16.  Returns MNF_OK, MNF_EINVAL, MNF_EUNSUPPORTED, MNF_ENOMEM or MNF_EHIP. */
int fuse_exposures(mnf_ctx* ctx, const uint16_t* raw, const float* t,
                   int J, int K, int H, int W, const mnf_fuse_params* params,
                   float* fused, float* weights_out, void* stream);

/* Linear baselines the fusion is compared against (the Introduction and
 * Results 2.2-2.3 name linear integration and single exposures without a
 * formula).
 * mode 0: per pixel, sum_k m_k (I_k - dark) / sum_k m_k t_k times t[0] over the
 *         frames below saturation (m_k = [I_k < sat]); the shortest frame's
 *         I_0 - dark where every frame is saturated.  For Poisson frames this
 *         is the maximum-likelihood rate, in counts of the shortest exposure.
 * mode 1: the shortest frame alone, I_0 - dark.
 * raw device uint16 [J][K][H][W]; t host float [K] (exposure 0 the shortest);
 * fused device float [J][H][W].  MNF_EINVAL for null pointers, sizes <= 0,
 * non-positive times, sat <= dark or another mode. */
int fuse_linear(mnf_ctx* ctx, const uint16_t* raw, const float* t, int J, int K, int H, int W, float sat,
                float dark, int mode, float* fused, void* stream);

/* ------------------------------------------------------------------------
 * Far-field forward model (Methods 3.3, Eqs. 2-3):
 *   I_out[j] = fftshift |F_unitary(pad_Nd(P * O[pos_j window]))|^2
 * O     device c64 [My][Mx];  P device c64 [Nw][Nw];
 * pos   host int32 [J][2] (y, x) top-left corner of each window in O;
 * I_out device float [J][Nd][Nd], detector-centred (zero frequency at Nd/2).
 * Nw <= Nd, Nd a supported size.  The exit wave sits at the top-left of the
 * Nd x Nd frame when Nw < Nd. */
int ptycho_forward(mnf_ctx* ctx, const mnf_c64* O, int My, int Mx,
                   const mnf_c64* P, int Nw, int Nd, const int32_t* pos, int J,
                   float* I_out, void* stream);

/* ------------------------------------------------------------------------
 * Mini-batched ePIE / rPIE reconstruction from fused intensities.
 * Exit wave (Eq. 2) -> unitary FFT (Eq. 3) -> Fourier-modulus projection
 * against A = sqrt(max(I, 0)) -> inverse FFT -> simultaneous object and probe
 * updates (ePIE: Maiden & Rodenburg 2009; rPIE: Maiden, Johnson & Li 2017),
 * numerators and denominators summed over each mini-batch of `batch`
 * consecutive positions of the iteration's order, both updates from the
 * batch-start state.  Denominators and error sums are float64.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t alg;              /* 0 = ePIE, 1 = rPIE */
    float   alpha;            /* object step (ePIE: den = max|P|^2/alpha; rPIE: (1-alpha)|P|^2 + alpha max|P|^2) */
    float   beta;             /* probe step, same forms with |O_j|^2 */
    int32_t batch;            /* mini-batch size B >= 1 */
    int32_t update_probe;     /* 0: probe fixed; 1: probe updated */
    int32_t probe_start_iter; /* first iteration index (it0-based) that updates the probe */
    int32_t it0;              /* index of the first iteration of this call (for probe_start_iter and resuming) */
    int32_t graph;            /* 1: capture the call's launches in one hipGraph and replay it on the stream */
} ptycho_params;

/* O      device c64 [My][Mx]   object, updated in place
 * P      device c64 [Nw][Nw]   probe, updated in place
 * I      device float [J][Nd][Nd] fused intensities, detector-centred
 * pos    host int32 [J][2]     window corners, every window inside O
 * order  host int32 [n_iter][J] one permutation of 0..J-1 per iteration, or NULL (identity)
 * err_out device double [n_iter] normalised Fourier error per iteration, or NULL
 * Returns MNF_OK, MNF_EINVAL, MNF_EUNSUPPORTED, MNF_ENOMEM or MNF_EHIP. */
int ptycho_iterate(mnf_ctx* ctx, mnf_c64* O, int My, int Mx, mnf_c64* P, int Nw,
                   const float* I, int Nd, const int32_t* pos, int J,
                   const int32_t* order, int n_iter, const ptycho_params* params,
                   double* err_out, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ptycho_iterate without
 * any allocation.  Arguments, layouts, ownership and results are those of
 * ptycho_iterate, except that params->graph must be 0 (MNF_EINVAL
 * otherwise) and launch timing (mnf_profile) is suspended for the call.
 * Every scratch buffer and staged host table of the call lives in one static
 * device array of 48 MiB per GPU, held from the context's creation until the
 * process ends; a call needing more (roughly batch x Nd^2 x 8 bytes of
 * pattern scratch plus 16 bytes per position per iteration of tables) fails
 * with MNF_EINVAL before any work is issued.  The fused intensities are
 * read directly (square roots taken in the column pass) instead of through
 * a per-call amplitude buffer.  All calls on one GPU share the array and it
 * keeps the last call's contents: calls that overlap in time on one GPU
 * (several streams, threads or contexts) race and must be serialised by
 * the caller.  Nothing in the array needs to start at zero. */
int ptycho_iterate_noalloc(mnf_ctx* ctx, mnf_c64* O, int My, int Mx, mnf_c64* P, int Nw,
                           const float* I, int Nd, const int32_t* pos, int J,
                           const int32_t* order, int n_iter, const ptycho_params* params,
                           double* err_out, void* stream);

/* ------------------------------------------------------------------------
 * Real-valued (sub-pixel) scan positions (Eq. 2 at positions such as the
 * Fermat spiral of Methods 3.3, which the integer entry points take rounded).
 * A position r = (y, x) is split into the nearest integer corner
 * p = floor(r + 1/2) and the fraction d = r - p in [-1/2, 1/2) per axis; the
 * fraction translates the probe: the exit wave is
 *     psi = S_d[P] * O[p window],
 *     S_d[P] = F^-1[ F[P](k) exp(-2 pi i (k_y d_y + k_x d_x) / Nw) ],
 * an Nw-periodic Fourier translation with k in [-Nw/2, Nw/2), which has the
 * far-field intensity of P(m) O(r + m) (translating the exit wave only adds
 * a phase ramp to Eq. 3).  Nw must be a supported transform size.
 * pos is host float [J][2]; the corners must satisfy the window bounds of the
 * integer entry points; non-finite or |r| > 1e8 coordinates give MNF_EINVAL.
 * Every other argument has the meaning, layout and ownership of ptycho_forward
 * and ptycho_iterate.  Positions with zero fractions take no transform.
 *
 * ptycho_forward_subpixel: I_out[j] = fftshift |F_unitary(pad_Nd(psi_j))|^2.
 * ptycho_iterate_subpixel: the ePIE / rPIE iteration of ptycho_iterate with
 * P_j = S_{d_j}[P] in the exit wave and in the object numerator
 * conj(P_j) dpsi_j, and probe numerators translated back to the untranslated
 * probe, P += sum_j S_{-d_j}[conj(O_j) dpsi_j] / sum_j d_P,j.  The step
 * denominators are those of ptycho_iterate (untranslated batch-start |P|^2,
 * integer windows |O_j|^2).  One scan per call; params->graph is honoured. */
int ptycho_forward_subpixel(mnf_ctx* ctx, const mnf_c64* O, int My, int Mx, const mnf_c64* P, int Nw, int Nd,
                            const float* pos, int J, float* I_out, void* stream);
int ptycho_iterate_subpixel(mnf_ctx* ctx, mnf_c64* O, int My, int Mx, mnf_c64* P, int Nw, const float* I, int Nd,
                            const float* pos, int J, const int32_t* order, int n_iter, const ptycho_params* params,
                            double* err_out, void* stream);

/* ------------------------------------------------------------------------
 * Mixed-state (multi-mode) probes for partially coherent illumination (the
 * incoherent sum of Eq. 4, e.g. the two harmonics of the XUV source in
 * Methods 3.2).  M mutually incoherent probe modes share one object:
 *     I_j = sum_m |F_unitary(pad_Nd(P_m * O[pos_j window]))|^2.
 * The iteration generalises ptycho_iterate (Thibault & Menzel 2013): each
 * mode's far field is scaled by A_j / sqrt(sum_m |Psi_jm|^2) (where the sum
 * is 0: A_j in mode 0, 0 in the others); the object takes
 * sum_j sum_m conj(P_m) dpsi_jm over denominators of the total probe
 * intensity Q = sum_m |P_m|^2 ((1-alpha) Q + alpha max Q for rPIE, max Q/alpha
 * for ePIE); each mode P_m takes sum_j conj(O_j) dpsi_jm over the
 * single-mode probe denominators; the error is sum (sqrt(sum_m |Psi|^2) - A)^2
 * normalised by sum A^2.  No orthogonalisation of the modes.
 * P     device c64 [M][Nw][Nw] (mode-major), 1 <= M <= 4, updated in place by
 *       ptycho_iterate_modes when the probe is updated;
 * batch * M <= 512; every other argument as for ptycho_forward / ptycho_iterate
 * (one scan per call, integer positions).  M = 1 is the single-mode path. */
int ptycho_forward_modes(mnf_ctx* ctx, const mnf_c64* O, int My, int Mx, const mnf_c64* P, int M, int Nw, int Nd,
                         const int32_t* pos, int J, float* I_out, void* stream);
int ptycho_iterate_modes(mnf_ctx* ctx, mnf_c64* O, int My, int Mx, mnf_c64* P, int M, int Nw, const float* I,
                         int Nd, const int32_t* pos, int J, const int32_t* order, int n_iter,
                         const ptycho_params* params, double* err_out, void* stream);

/* ------------------------------------------------------------------------
 * Many independent scans of uneven sizes in one call (the same iteration as
 * ptycho_iterate, applied to every scan).  Scans are grouped by detector
 * size; each pass of each mini-batch round is one launch covering the
 * current mini-batch of every scan of that size (grid y spans all of their
 * positions), so small scans share the GPU with large ones; the size classes
 * are issued on streams of their own (forked from and joined to `stream`),
 * so their passes overlap (one stream while kernel timing is enabled).  With
 * params->graph = 1 the whole call is captured in one hipGraph and replayed.
 * Each scan's fields have the meaning of the ptycho_iterate arguments of the
 * same name; `order` has n_iter rows of that scan's J entries or is NULL. */
typedef struct {
    mnf_c64* O; int32_t My, Mx;
    mnf_c64* P; int32_t Nw;
    const float* I; int32_t Nd;
    const int32_t* pos; int32_t J;
    const int32_t* order;
    double* err_out;
} ptycho_scan;

int ptycho_iterate_many(mnf_ctx* ctx, const ptycho_scan* scans, int n_scans, int n_iter,
                        const ptycho_params* params, void* stream);

/* Validates a ptycho_iterate_many call (the same checks, in the same order,
 * with the same return codes) and plans it on the host, with no device work:
 * the device pointers in `scans` are never dereferenced, and a plan can be
 * taken on a machine without a GPU.  ctx may be NULL (default launch shapes;
 * a failure's message is then read with mnf_last_error(NULL)); a context
 * contributes the launch shapes set on it.  `order` and `pos` are read.
 * info int64 [n_info] receives, in this order (entries past the last
 * defined one are set to 0; n_info may be 0):
 *   0  launches per call (one launch of each pass over a list of slots)
 *   1  slots per call (exit waves formed: n_iter x sum over scans of J x modes)
 *   2  groups per call (one per scan and mini-batch round)
 *   3  object-update blocks per call (16 x 64 tiles of each group's window box)
 *   4  slots of the largest launch
 *   5  bytes of pattern scratch (the largest launch's patterns, complex64)
 *   6  size classes (distinct detector sizes) */
int ptycho_plan_info(mnf_ctx* ctx, const ptycho_scan* scans, int n_scans, int n_iter,
                     const ptycho_params* params, int64_t* info, int n_info);

/* ------------------------------------------------------------------------
 * Loss on fused intensities and its gradient (the adjoint of Eqs. 2-3; the
 * Poisson model of the Introduction), exit waves recomputed per chunk of
 * `batch` positions:
 *   loss = sum_j sum_q l(Psi_j, I_j),  Psi_j = F_unitary(pad(P O_j)),
 *   Poisson (kind 0): l = |Psi|^2 - I ln(|Psi|^2 + eps), I = max(I, 0)
 *   amplitude (kind 1): l = (|Psi| - sqrt(I))^2
 * Gradients use g = dL/dRe + i dL/dIm (PyTorch's complex convention),
 * scaled by *upstream: a device double scalar read by the kernels (so an
 * autograd backward needs no device-to-host copy), or NULL for 1.
 * gO device c64 [My][Mx] and gP device c64 [Nw][Nw] are overwritten (either may be NULL).
 * loss_out device double [1] (may be NULL).  A non-finite loss is recorded
 * for mnf_status. */
int ptycho_grad(mnf_ctx* ctx, const mnf_c64* O, int My, int Mx, const mnf_c64* P, int Nw,
                const float* I, int Nd, const int32_t* pos, int J,
                int kind, float eps, int batch, const double* upstream,
                double* loss_out, mnf_c64* gO, mnf_c64* gP, void* stream);

/* Gradient-descent reconstruction on the loss of ptycho_grad (same kind, eps,
 * batch and data layout), O and P updated in place.  Pass s takes the loss
 * L_s and both gradients at the current (O, P); then (backtracking, a
 * reading: the paper prescribes no descent schedule)
 *   s = 0, or L_s <= L_ref + 1e-6 |L_ref| (L_ref: the loss of the last
 *          accepted pass; the 1e-6 bounds float32 evaluation error): accepted,
 *          the point, its gradients and L_s become the reference,
 *          O -= eta_O gO and P -= eta_P gP (the probe only with update_probe);
 *   otherwise: both step sizes are halved and the next point is the
 *          reference point minus the halved steps along its gradients.
 * Initial step sizes: eta_O = 0 takes 1 / (2 max_x sum_j |P(x - p_j)|^2) over
 * the object grid and eta_P = 0 takes 1 / (2 max_u sum_j |O(p_j + u)|^2) over
 * the probe window, from the starting O and P (the inverse of the largest
 * diagonal curvature of the amplitude loss); a positive value is used as given.
 * On return O and P are the last point formed (its loss not evaluated).
 * loss_out device double [n_steps]: L_s of each pass (may be NULL);
 * eta_out  device double [2]: the step sizes at the end of the call, halvings
 *          included, i.e. the values with which to resume (may be NULL).
 * Scratch: 8 (My Mx + Nw^2) bytes for the gradients and twice that for the
 * best point.  Returns MNF_EINVAL for a bad argument (as ptycho_grad;
 * negative or non-finite step sizes, n_steps < 0); a non-finite loss is
 * recorded for mnf_status. */
int ptycho_descend(mnf_ctx* ctx, mnf_c64* O, int My, int Mx, mnf_c64* P, int Nw,
                   const float* I, int Nd, const int32_t* pos, int J,
                   int kind, float eps, int batch, int n_steps, double eta_O, double eta_P,
                   int update_probe, double* loss_out, double* eta_out, void* stream);

/* ------------------------------------------------------------------------
 * Warm-start network: a four-level U-Net mapping a log-scaled fused pattern
 * [n][H][H] to the amplitude and phase of the illuminated object patch
 * [n][H/4][H/4][2] (channels last).  Level l (size H/2^l, width widths[l])
 * has two 3x3 convolutions + ReLU; 2x2 stride-2 convolutions + ReLU join the
 * levels; a 2x2 transposed convolution + ReLU returns from level 3 to level
 * 2, its output concatenated (first) with the level-2 encoder output; two
 * 3x3 convolutions (width widths[2]) + ReLU and a 1x1 head give 2 outputs.
 * Input x = ln(1 + max(I, 0)) * log_scale.  BF16 MFMA convolutions with
 * float32 accumulation; bf16 activations; float32 parameters, per layer
 * W[taps][c_in][c_out] then b[c_out], in the order above (taps 9, 4 or 1).
 * The network extends the method (the paper reconstructs without one); it
 * supplies a starting object for the iterations. */
typedef struct {
    int32_t H;          /* input size, a multiple of 8, >= 16 */
    int32_t widths[4];  /* channel widths of the four levels, multiples of 8, <= 256 */
} mnf_unet_shape;

/* Number of float32 parameters of the network (host call; -1 for NULL). */
long long unet_param_count(const mnf_unet_shape* shape);

/* params device float[count]; I device float [n][H][H]; out device float [n][H/4][H/4][2]. */
int unet_forward(mnf_ctx* ctx, const mnf_unet_shape* shape, const float* params, const float* I,
                 float log_scale, int n, float* out, void* stream);

/* One training step on a batch: forward, mean-squared-error loss against
 * target (device float [n][H/4][H/4][2]), backward, and (when adam_m and
 * adam_v are given) an Adam update of params (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected with `step` >= 1).  loss_out (device double[1]),
 * grad_out (device float[count]) and out (device float [n][H/4][H/4][2])
 * are optional. */
int unet_train_step(mnf_ctx* ctx, const mnf_unet_shape* shape, float* params, float* adam_m, float* adam_v,
                    int step, float lr, const float* I, float log_scale, const float* target, int n,
                    double* loss_out, float* grad_out, float* out, void* stream);

/* Single convolution layers (the network's building blocks).
 * mode 0: 3x3 stride 1 pad 1; 1: 2x2 stride 2; 2: 2x2 transposed stride 2; 3: 1x1.
 * x device bf16 (uint16 bits) [n][H][H][Ci]; W device float [taps][Ci][Co]; b device float [Co] or NULL;
 * y device float [n][Ho][Ho][Co] (Ho = H, H/2, 2H, H). */
int mnf_conv2d(mnf_ctx* ctx, int mode, const uint16_t* x, int n, int H, int Ci, const float* W, const float* b,
               int Co, int relu, float* y, void* stream);
/* Gradients of a layer given dy (bf16 [n][Ho][Ho][Co]) and, if not NULL, the layer's ReLU output act
 * (bf16, same layout; dy is masked by act > 0): dx (bf16 [n][H][H][Ci], may be NULL), dW (float
 * [taps][Ci][Co]) and db (float [Co]) (both or neither). */
int mnf_conv2d_grad(mnf_ctx* ctx, int mode, const uint16_t* x, int n, int H, int Ci, const float* W, int Co,
                    const uint16_t* dy, const uint16_t* act, uint16_t* dx, float* dW, float* db, void* stream);

/* ------------------------------------------------------------------------
 * Warm-start support.
 *
 * detector_expose: synthetic detector exposures of clean intensities, for
 * generating training and test data at scale (the forward model of the
 * measurement, Methods: a bracket of exposures t_k of one pattern).
 *   raw[j][k] = clip(rint(Poisson(scale * t_k * max(clean[j], 0)) + N(0, sigma_read^2)), 0, sat)
 * clean device float [J][H][W]; t host float [K] (K <= 16); raw device uint16 [J][K][H][W].
 * Random numbers come from the counter-based Philox4x32-10 generator keyed by
 * `seed`, one counter per output element, so the result depends only on the
 * seed and the element index.  Poisson draws are exact: inversion below a
 * mean of 10, Hoermann's transformed rejection with squeeze (PTRS, 1993)
 * above (means beyond 1e8 saturate and are not drawn); normals use
 * Box-Muller.
 * Errors: MNF_EINVAL for null pointers, non-positive sizes, K > 16,
 * negative scale or sigma_read, or sat outside (0, 65535]. */
int detector_expose(mnf_ctx* ctx, const float* clean, int J, int H, int W, const float* t, int K, float scale,
                    float sat, float sigma_read, unsigned long long seed, uint16_t* raw, void* stream);

/* ptycho_stitch: starting object from predicted patches (amplitude, phase)
 * of each scan window, averaged with the probe intensity as weight:
 *   O[x] = sum_j |P(x - p_j)|^2 c_j a_j(x - p_j) exp(i phi_j(x - p_j)) / sum_j |P(x - p_j)|^2
 * over the windows covering x, and O[x] = 1 where the weight is zero.
 * A single far-field pattern fixes its window only up to a constant phase,
 * so with sync != 0 the unit phasors c_j are chosen to align overlapping
 * windows: the leading eigenvector (200 power iterations from all ones) of
 *   C_jk = sum over the overlap of |P_j|^2 |P_k|^2 conj(z_j) z_k,  z = a e^{i phi},
 * projected to unit modulus, with sum_j c_j real and positive (J <= 1024).
 * With sync == 0, c_j = 1.
 * patches device float [J][Nw][Nw][2] (amplitude, phase; the network's output
 * layout); P device c64 [Nw][Nw]; pos host int32 [J][2] (y, x) window corners;
 * O device c64 [My][Mx], overwritten.  MNF_EINVAL for a window outside O or
 * J > 1024 with sync. */
int ptycho_stitch(mnf_ctx* ctx, const float* patches, const mnf_c64* P, int Nw, const int32_t* pos, int J,
                  int sync, mnf_c64* O, int My, int Mx, void* stream);

/* mnf_nrmse: normalised object error after the best complex scale,
 *   min_gamma ||gamma O - O_true|| / ||O_true|| = sqrt(1 - |<O, O_true>|^2 / (||O||^2 ||O_true||^2)),
 * over the n elements whose mask byte is non-zero (mask NULL = all), summed
 * in float64.  O, O_true device c64 [n]; mask device uint8 [n] or NULL;
 * out device double [1].  0 when O_true is zero on the mask; 1 when O is. */
int mnf_nrmse(mnf_ctx* ctx, const mnf_c64* O, const mnf_c64* O_true, const uint8_t* mask, long long n,
              double* out, void* stream);

/* detector_resample: one line of a discrete-spectrum measurement (Methods 3.3,
 * Eq. 4) from the reference-wavelength pattern, for an achromatic probe and
 * object: the pattern at wavelength lambda is the reference pattern sampled
 * at c + (k - c) * scale (scale = lambda_0 / lambda, c = Nd / 2, the centred
 * zero frequency), bilinear between pixels, zero outside the detector, times
 * scale^2 (which keeps the pattern's total):
 *   out[j][k] = (accumulate ? out[j][k] : 0) + weight * scale^2 * I(c + (k - c) scale)
 * I device float [J][Nd][Nd] (detector-centred); out device float [J][Nd][Nd],
 * not aliasing I.  MNF_EINVAL for null pointers, sizes <= 0, scale <= 0 or
 * aliasing buffers. */
int detector_resample(mnf_ctx* ctx, const float* I, int J, int Nd, float scale, float weight, int accumulate,
                      float* out, void* stream);

/* ------------------------------------------------------------------------
 * Launch-shape tuning.  Every pattern pass is compiled in two shapes (rows:
 * the default lines per block or half as many; columns: 32 columns per block
 * or 16); bit 0 of a variant selects the row shape, bit 1 the column shape.
 * Bit 2 selects the pass structure of a single-scan, integer-position,
 * single-mode reconstruction whose object box is at most 1024 pixels wide:
 * three launches per mini-batch (the object update fused with the next
 * mini-batch's exit-wave rows) instead of four.  Such a reconstruction with
 * mini-batches of one on a detector of at most 64^2 runs as a whole in one
 * workgroup (pattern and probe in LDS, one launch per call) unless bit 3 is
 * set.  Variants change only launch geometry and pass structure, never the
 * algorithm or the mini-batch, and give identical objects and probes (the
 * errors up to the order of float64 partial sums).
 *
 * mnf_autotune times the eight variants on a synthetic mini-batch of
 * `nslots` windows spread as in a scan larger than the batch taken in a
 * shuffled order (drawn from a raster of step Nd/8 over an object of side
 * about 4 Nd; one mini-batch per iteration, `reps` iterations)
 * in three interleaved rounds, keeps for size Nd on this context the variant
 * with the lowest median time if it beats variant 0 by at least 3 % (else 0)
 * and returns its index (0..7), or a negative error.  times_us (host
 * double[8] or NULL) receives each variant's median time of one iteration.
 * It synchronises the stream.  mnf_set_variant / mnf_get_variant store or
 * read a variant (e.g. from a tuning cache kept by the caller). */
int mnf_autotune(mnf_ctx* ctx, int Nd, int nslots, int reps, double* times_us, void* stream);
int mnf_set_variant(mnf_ctx* ctx, int Nd, int variant);   /* variant 0..15 */
int mnf_get_variant(mnf_ctx* ctx, int Nd);

/* ------------------------------------------------------------------------
 * Launch timing, for measurement.  With bit c of class_mask set, every
 * launch of kernel class c is bracketed by HIP events recorded on its
 * stream.  Classes: 0 rows_fwd (gather + row transforms), 1 cols_modulus
 * (column transforms + modulus projection + inverse column transforms),
 * 2 rows_inv (inverse row transforms + exit-wave difference), 3 probe_update
 * (the translated probe update of real positions), 4 object_update, 5 small
 * (copies, reductions), 6 fuse, 7 forward, 8 grad_cols, 9 grad_scatter,
 * 10 shift (Fourier translation of probes), 11 small_run (a whole run of
 * mini-batches of one in one workgroup).  mask 0 disables timing.
 * mnf_profile_read waits for the recorded events and returns the launch
 * count and summed duration (ms) of class cls since the last reset.
 *
 * mnf_profile_sampled times only every period-th launch of each class in
 * the mask (the first, then every period-th after it, counted per class
 * from the last reset); mnf_profile_read then counts and sums the timed
 * launches only, so total_ms / launches stays the mean duration of a launch
 * while the events' own cost (a few microseconds per timed launch) falls by
 * the period.  period < 1: MNF_EINVAL.  mnf_profile resets the period to 1. */
int mnf_profile(mnf_ctx* ctx, uint32_t class_mask);
int mnf_profile_sampled(mnf_ctx* ctx, uint32_t class_mask, int period);
int mnf_profile_read(mnf_ctx* ctx, int cls, long long* launches, double* total_ms);
int mnf_profile_reset(mnf_ctx* ctx);
const char* mnf_kernel_class_name(int cls);

#ifdef __cplusplus
}
#endif

#endif /* MNFPTY_H */
