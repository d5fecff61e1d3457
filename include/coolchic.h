/*
 * coolchic.h -- C ABI of the MI355X (gfx950) Cool-chic 5.0 encoding step.
 *
 * One encoding iteration (Section IV of the paper) for one image or a batch
 * of images: the training quantisation proxy of the latent grids (Section
 * IV-C, eq. q-train / eq. softround), the autoregressive Laplace entropy model
 * with inter-feature context that gives the rate (Section III-A, eq.
 * factorized-probability / eq. laplace-distribution), the learned upsampling
 * and the synthesis (Section III-B) with linear stabilizers (Section III-C),
 * the MSE + lambda * rate cost (Section IV-A, eq. training-loss), its gradient
 * and an Adam update (Section IV-B).
 *
 * Conventions shared by every call
 *   - Every function returns CC_OK (0) or a negative error code; the message
 *     of the last failure on the calling thread is cc_last_error().  No C++
 *     exception crosses this boundary.
 *   - Device pointers are HIP device addresses on the current device; the
 *     caller owns every device buffer (the state slab, images, outputs).  The
 *     library owns only the opaque cc_state descriptor (host memory).
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     work asynchronously on it; a call that fills a host output pointer
 *     synchronises the stream before returning.
 *   - The library never allocates device memory: all scratch lives in the
 *     caller-provided state slab of cc_state_bytes() bytes.
 *   - Latent layout ("flat pyramid"): grid k = 0 .. L-1 of shape
 *     (H/2^k, W/2^k) stored row-major, grid 0 first.
 *   - Decoder parameter layout: ARM layers (W [out,in] row-major, then b),
 *     ARM stabilizer (W [2,ctx], b [2]), IFCE k = 0..n_ifce_grids-1
 *     (W [F, L-k-1], b [F]), upsampling level j = 1..L-1 (4 free taps h0..h3
 *     of the symmetric kernel h0 h1 h2 h3 h3 h2 h1 h0), synthesis 1x1 layers
 *     (W [out,in], b), synthesis stabilizer (W [3,L], b [3]), residual 3x3
 *     layers (W [3,3,3,3] as out,in,ky,kx, b [3]).
 *   - Images are planar float32 [3, H, W] with values in [0, 1].
 */
#ifndef COOLCHIC_H
#define COOLCHIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CC_OK = 0,
  CC_EINVAL = -1,      /* bad argument, unsupported shape or configuration */
  CC_ENOMEM = -2,      /* state slab smaller than cc_state_bytes()          */
  CC_EDEVICE = -3,     /* a HIP runtime call failed                         */
  CC_ENONFINITE = -4,  /* the loss of an earlier step was NaN or infinite   */
  CC_ESTATE = -5       /* state not initialised or inconsistent             */
};

enum { CC_SOFT = 0, CC_HARD = 1 };              /* quantisation mode   */
enum { CC_FP32_PLAIN = 0, CC_BF16_FUSED = 1 };  /* arithmetic of the MLPs */
enum { CC_OPT_ADAM = 0, CC_OPT_SOAP = 1 };      /* decoder-parameter optimiser */

#define CC_MAX_BATCH 32

/* Decoder shape (Table II gives the named presets).  The ARM always has
 * two hidden layers (Table II).  Supported shapes are listed by
 * cc_config_supported(). */
typedef struct cc_config {
  int L;              /* latent grids, 2..8                                  */
  int n_spatial;      /* causal spatial neighbours s                         */
  int n_ifce_feat;    /* inter-feature context size F (0 = no IFCE)          */
  int n_ifce_grids;   /* grids 0..n_ifce_grids-1 use an IFCE, 0..3           */
  int arm_hidden[2];  /* widths of the two hidden ARM layers                 */
  int arm_stab;       /* 1 = linear stabilizer beside the ARM                */
  int n_syn_hidden;   /* hidden 1x1 synthesis layers, 1 or 2                 */
  int syn_hidden[2];
  int syn_stab;       /* 1 = linear stabilizer beside the synthesis trunk    */
  int n_res;          /* residual 3x3 post-filter layers, 0..4               */
  float logscale_min; /* clamp of the ARM log-scale output                   */
  float logscale_max;
  float p_min;        /* floor of a latent's probability                     */
  int precision;      /* CC_FP32_PLAIN or CC_BF16_FUSED                      */
  /* Hyperlatent grids (Section III-A.3): n_hyper extra grids of resolutions
   * 1/2^b .. 1/2^(b + n_hyper - 1), b = hyper_first, stored after the L
   * latent grids in every flat latent array.  The ARM codes them with their
   * spatial context (no IFCE of their own), every IFCE takes them as inputs
   * after the coarser latent grids (nearest upsampling), and the upsampling
   * and synthesis never see them.  0..4 grids; n_ifce_grids <= b and
   * b + n_hyper <= L (each resolution is one of the latent grids'). */
  int n_hyper;
  int hyper_first;
  /* Upsampling Conv refinement (Section III-B: the upsampling combines
   * symmetric separable convolutions and transposed convolutions): 1 =
   * before its transposed convolution, level j filters T_j with the
   * symmetric 7-tap kernel (c3 c2 c1 c0 c1 c2 c3) on rows then columns
   * (stride 1, replicate edge, every channel); its 4 free taps per level
   * follow the transposed convolutions' taps in the parameter vector and
   * start at (1, 0, 0, 0), the identity.  0 = none. */
  int ups_conv;
} cc_config;

/* Per-iteration scalars (Table I schedules are evaluated by the caller). */
typedef struct cc_step_params {
  int64_t t;          /* 1-based iteration: noise counter and Adam step      */
  float lr;           /* Adam learning rate                                  */
  float temperature;  /* softround temperature T                             */
  float sigma;        /* std of the Gaussian noise                           */
  int quant_mode;     /* CC_SOFT: s_T(s_T(y) + n); CC_HARD: round half even  */
  int update_latents; /* 0 = latents frozen (hard-round stage)               */
} cc_step_params;

typedef struct cc_rd_result {
  double bits, bpp, mse, psnr, loss;
} cc_rd_result;

typedef struct cc_state cc_state;

/* 1 if the GPU path supports this decoder shape and image size, else 0.
 * H and W must be multiples of 2^(L-1). */
int cc_config_supported(const cc_config* cfg, int H, int W);

/* 1 if precision CC_BF16_FUSED runs this decoder shape's ARM on the matrix
 * cores (the fused MFMA kernel covers the shape), 0 if that form falls back
 * to the plain FP32 ARM kernel; -1 for an unsupported configuration.  The
 * cfg's own precision field is ignored.  Host only. */
int cc_arm_fused_available(const cc_config* cfg);

/* Sizes. */
int64_t cc_n_latents(const cc_config* cfg, int H, int W);
int cc_n_params(const cc_config* cfg);
size_t cc_state_bytes(const cc_config* cfg, int H, int W);

/* Initialise a state in the caller's device slab `mem` (>= cc_state_bytes,
 * 256-byte aligned).  Copies the image in, sets the latents (host array of
 * cc_n_latents floats, NULL = all zero) and decoder parameters (host array of
 * cc_n_params floats, NULL = seeded default: U(+-1/sqrt(fan_in)) weights and
 * biases, zero ARM output layer, bicubic upsampling), zero Adam moments.
 * `seed` keys the Philox noise.  Synchronises `stream`. */
int cc_init_state(const cc_config* cfg, int H, int W, const float* img_dev,
                  double lambda, uint64_t seed, const float* init_latents_host,
                  const float* init_params_host, void* mem, size_t bytes,
                  void* stream, cc_state** out);

/* One encoding iteration (forward, backward, Adam).  If `out3` is not NULL
 * it receives (loss, bits, mse) of this iteration's forward pass and the
 * stream is synchronised; a non-finite loss then returns CC_ENONFINITE and
 * marks the state.  With `out3` NULL the call is fully asynchronous. */
int cc_encode_step(cc_state* s, const cc_step_params* p, double* out3, void* stream);

/* The same iteration for n <= CC_MAX_BATCH independent states in one set of
 * launches; p[i] applies to states[i]; out (3 n doubles, may be NULL). */
int cc_encode_step_batch(cc_state* const* states, int n, const cc_step_params* p,
                         double* out, void* stream);

/* Concurrency of the two branches of an iteration.  The rate branch (ARM
 * forward and backward, IFCE gradient pooling) and the distortion branch
 * (upsampling, synthesis and their backward) meet only at the latent-gradient
 * join (Section IV-A: the loss is a sum of the two terms), so by default the
 * rate branch runs on a second, library-owned non-blocking stream of the
 * state's device, forked from `stream` after the quantisation kernel and
 * joined back into it with events before the join; callers still see one
 * stream.  Results are bitwise the same either way (no kernel shares an
 * output with the other branch).  Calls on one device serialise their
 * launches on a per-device lock.  enable = 0 runs both branches on `stream`
 * in order.  Process-wide; returns the previous setting (1 or 0). */
int cc_set_branch_overlap(int enable);

/* Loss of the current state for the iteration's quantisation (noise from
 * p->t), without gradient or update: (loss, bits, mse).  Synchronises. */
int cc_eval_loss(cc_state* s, const cc_step_params* p, double* out3, void* stream);

/* Rate and distortion with hard quantisation, no gradient.  Synchronises. */
int cc_rd_eval(cc_state* s, cc_rd_result* out, void* stream);

/* cc_rd_eval for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels in the same order, so `out` is bit for bit cc_rd_eval's,
 * but every buffer the evaluation writes (a copy of the state's descriptor,
 * quantised latents, upsampled planes, synthesis activations, FP64 partial
 * sums) lives in a static device array of 64 MiB that the library holds on
 * each device it runs on until the process ends; the state slab is only read.
 * The array covers images up to about 0.75 megapixel with the workload's
 * decoder (a 512x768 state uses 34 MiB); a larger state returns CC_ENOMEM
 * before anything is queued.  Allocates nothing (no hipMalloc, no library
 * allocation); synchronises `stream`.  Every call on a device shares that
 * device's array and leaves its contents behind: calls that overlap on one
 * device (two streams or threads at once) race and must be serialised by
 * the caller. */
int cc_rd_eval_noalloc(cc_state* s, cc_rd_result* out, void* stream);

/* Quantisation and transmission rate of the decoder parameters (Section
 * IV-E).  Submodules a = 0 ARM, 1 synthesis (with the residual layers),
 * 2 upsampling, 3 IFCE; w = 0 weights, 1 biases.  For every submodule in
 * that order, each pair of steps (2^-8 ... 2^-1 for the weights and for the
 * biases) is tried with the submodules before it quantised at their choice
 * and the ones after it unquantised: the parameters become step * rint(p /
 * step) (ties to even), the integers v are coded with Exp-Golomb (u = 2v - 1
 * for v > 0, -2v otherwise; the order 0..11 with the fewest bits per group),
 * and the pair with the lowest MSE + lambda (R(latents) + R_NN) / (H W),
 * latents hard-quantised, is kept (the first one on ties).  The state is left
 * with the chosen quantised decoder parameters.  step_index / step / kappa:
 * -1 / 0 / -1 for a group without parameters.  Synchronises `stream`. */
typedef struct cc_nnq_result {
  int step_index[4][2];   /* e: step 2^(e-8) */
  double step[4][2];
  int kappa[4][2];        /* Exp-Golomb order */
  double nn_bits;         /* R_NN: bits of all parameter codes */
  double bits, mse, psnr; /* latent bits and distortion with the quantised decoder */
  double loss;            /* mse + lambda (bits + nn_bits) / (H W) */
} cc_nnq_result;
int cc_nn_quantize(cc_state* s, cc_nnq_result* out, void* stream);

/* Decoded image [3, H, W] (hard quantisation -> upsampling -> synthesis)
 * into the caller's device buffer. */
int cc_decode(cc_state* s, float* out_img_dev, void* stream);

/* Copy state to / from host arrays (any pointer may be NULL to skip).
 * latents: cc_n_latents floats; params, grad: cc_n_params floats for the
 * decoder part, latents first for `grad_host` (n_latents + n_params). */
int cc_get_state(cc_state* s, float* latents, float* params, float* adam_m,
                 float* adam_v, int64_t* t, void* stream);
int cc_set_state(cc_state* s, const float* latents, const float* params,
                 const float* adam_m, const float* adam_v, int64_t t, void* stream);
/* Gradient of the last cc_encode_step (n_latents + n_params floats). */
int cc_get_grad(cc_state* s, float* grad_host, void* stream);

/* Diagnostics: copy `count` floats of an internal buffer of the last step
 * to the host: "yhat" (quantised latents), "dq" (d yhat / d y), "dyd"
 * (direct rate gradient), "dyq" (distortion gradient of the latents),
 * "xhat" (decoded image), "dx0" (gradient at the synthesis trunk output).
 * Synchronises `stream`. */
int cc_debug_read(cc_state* s, const char* buffer, float* host, int64_t count, void* stream);

/* Switch the arithmetic of the MLP kernels (CC_FP32_PLAIN / CC_BF16_FUSED). */
int cc_set_precision(cc_state* s, int precision);

/* Optimiser of the decoder parameters (Section IV-B trains them with SOAP,
 * the latents with Adam).  CC_OPT_ADAM (default): the latents' Adam.
 * CC_OPT_SOAP: SOAP (Vyas et al., 2024) with its published defaults --
 * beta1 = beta2 = 0.95, factor average 0.95, eps 1e-8, basis refresh every
 * 10 updates, bias correction -- one Kronecker factor per dimension of each
 * weight tensor (dimensions up to 48), Adam in SOAP's step form for
 * one-dimensional tensors; the first step after selecting SOAP only
 * initialises its factors and bases.  Selecting SOAP clears its state
 * (enqueued on `stream`).  Every state of one cc_encode_step_batch call must
 * use the same optimiser.  CC_EINVAL for an unknown value or a parameter
 * tensor above 1024 values. */
int cc_set_optimizer(cc_state* s, int optimizer, void* stream);

/* Floats of all SOAP Kronecker factors of a configuration (equally, of all
 * bases): the size of the `p` and `q` buffers below.  Host only; -1 if the
 * configuration is not supported. */
int64_t cc_soap_factor_size(const cc_config* cfg);

/* SOAP state to / from host memory, in the layout of the decoder parameters:
 * m, v: first and second moments, n_params floats each (v in the rotated
 * coordinates); p, q: every factor and every basis, row-major, tensor by
 * tensor in parameter order, dimension by dimension (cc_soap_factor_size
 * floats each); calls: SOAP calls made (0: the next call initialises).
 * Any pointer may be NULL to skip that part.  Synchronises `stream`. */
int cc_get_soap_state(cc_state* s, float* m, float* v, float* p, float* q, int* calls,
                      void* stream);
int cc_set_soap_state(cc_state* s, const float* m, const float* v, const float* p,
                      const float* q, int calls, void* stream);

/* Per-module forward and backward on caller buffers (for autograd
 * wrappers).  The state supplies the decoder shape and serves as workspace:
 * its latent, parameter and scratch buffers are overwritten, so run these on a
 * state that is not being encoded, and call a module's backward right after
 * its forward on the same state.  `params` / `grad_params`: the full decoder
 * parameter vector (cc_n_params floats, documented order); a backward writes
 * only its module's range of grad_params.  Any gradient pointer may be NULL.
 *
 * ARM (Section III-A, eq. factorized-probability and eq.
 * laplace-distribution): bits = sum over all latents of -log2 of the
 * Laplace bin probability given the causal and inter-feature context, for
 * given quantised latents `yhat` (flat pyramid, cc_n_latents floats); with
 * gradient pointers also d bits / d yhat and d bits / d (ARM, IFCE
 * parameters).  bits_out: host double (the stream is synchronised).
 *
 * Upsampling (Section III-B): zhat [L, H, W] = f_upsilon(yhat); the backward
 * takes d/d zhat and writes d/d yhat (cc_n_latents) and the tap gradients.
 *
 * Synthesis (Sections III-B, III-C): xhat [3, H, W] = f_theta(zhat) (trunk,
 * stabilizer, residual layers); the backward takes d/d xhat and writes
 * d/d zhat [L, H, W] and the synthesis parameter gradients. */
int cc_arm_fwd_bwd(cc_state* s, const float* yhat, const float* params, double* bits_out,
                   float* grad_yhat, float* grad_params, void* stream);
int cc_ups_fwd(cc_state* s, const float* yhat, const float* params, float* zhat, void* stream);
int cc_ups_bwd(cc_state* s, const float* grad_zhat, float* grad_yhat, float* grad_params,
               void* stream);
int cc_syn_fwd(cc_state* s, const float* zhat, const float* params, float* xhat, void* stream);
int cc_syn_bwd(cc_state* s, const float* grad_xhat, float* grad_zhat, float* grad_params,
               void* stream);

/* Launch shape of the tunable kernels of a state (for an autotuner; the
 * results differ only by the order of the weight-gradient partial sums):
 *   arm_wgs            fused ARM workgroups per image, 1 .. the number of
 *                      2-row bands of all grids; the bands are packed onto
 *                      them longest first, each onto the least loaded one
 *                      (default: one band per workgroup, at most 512);
 *   syn_chunks_per_wg  64-pixel chunks per synthesis-backward workgroup,
 *                      4 .. 64;
 *   res_tiles_per_wg   8 x 64 tiles per residual-adjoint workgroup, 1 .. 16.
 * 0 keeps a value.  cc_set_launch_shape synchronises `stream` (the state's
 * last step must be finished before its descriptor changes); CC_EINVAL for
 * a value out of range.  cc_get_launch_shape also returns the number of
 * bands (the largest arm_wgs); any pointer may be NULL.  Host side only. */
int cc_set_launch_shape(cc_state* s, int arm_wgs, int syn_chunks_per_wg, int res_tiles_per_wg,
                        void* stream);
int cc_get_launch_shape(const cc_state* s, int* arm_wgs, int* syn_chunks_per_wg,
                        int* res_tiles_per_wg, int* arm_bands);

/* How the fused ARM splits an image's bands over nw workgroups (host only,
 * no GPU needed): *nbands = number of 2-row bands of all grids (band index:
 * grid 0's bands from the top, then grid 1's, ...), *default_nw = the
 * default workgroup count of a state of this shape; with wbeg (nw + 1 ints)
 * and blist (*nbands ints) also the packing itself: workgroup w takes the
 * bands blist[wbeg[w] .. wbeg[w + 1]).  Any pointer may be NULL; nw is read
 * only when wbeg or blist is given (CC_EINVAL outside [1, *nbands]). */
int cc_arm_band_plan(const cc_config* cfg, int H, int W, int nw, int* nbands, int* default_nw,
                     int* wbeg, int* blist);

/* Live kernel timing for measurement tools: HIP events are recorded on the
 * launch stream around every launch of one kernel class ("arm", "syn_bwd",
 * "res_bwd", "ups_fwd", "ups_bwd", "join" -- the latent-gradient join, which
 * also applies the latents' Adam update in an encode step and shares its
 * launch with the first pass of the weight-gradient reduction; "pool", the IFCE
 * gradient pooling and IFCE weight gradient; "syn_fwd", the synthesis trunk,
 * residual layers and MSE forward; NULL or "" switches
 * timing off; the upsampling and residual classes time all levels or layers of
 * one step as one span) by the calls that follow.  cc_timing_read waits for those events and returns the summed
 * duration (ms) and the number of timed launches, then resets the record.
 * Process-wide, not thread-safe. */
int cc_timing_enable(const char* kernel);
int cc_timing_read(double* total_ms, int* count);
/* Time one launch in n of the enabled class (default 1, every launch), to
 * keep the events' own cost small in a timed loop; CC_EINVAL for n < 1. */
int cc_timing_every(int n);

void cc_free_state(cc_state* s);
const char* cc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* COOLCHIC_H */
