// Internal definitions shared by the HIP kernels and the host side of the
// Cool-chic encode-step library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/coolchic.h"

#define CC_MAX_L 8    // latent grids
#define CC_MAX_G 12   // grids of the flat latent pyramid (latent + hyperlatent)
#define CC_MAX_NIN 10 // inputs of one IFCE (coarser latent grids + hyperlatent grids)
#define CC_MAX_S 32
#define CC_MAX_PROD 32
#define CC_NOALLOC_SCRATCH_BYTES (64u << 20)  // static scratch of cc_rd_eval_noalloc, per device

// One producer of weight-gradient partial rows (a kernel whose workgroups
// each write the sum of their positions' contributions to a parameter range).
struct ProdSeg {
  int pbeg;      // first parameter index (within the decoder parameters)
  int pcnt;      // number of parameters
  int nrows;     // partial rows (one per producing workgroup)
  int pad;
  long long off; // float offset of row 0 in the partial buffer; row stride pcnt
};

// Per-image descriptor, resident in device memory at the start of the state
// slab; kernels read it through uniform (scalar) loads.
struct DevDesc {
  // ---- shape
  int H, W, L, S, F, G, H1, H2, ctx, arm_stab, syn_stab, n_syn_hidden, n_res;
  int syn_w[4];                 // L, hidden..., 3 (n_syn_hidden + 2 entries)
  int n_lat, n_par, n_theta;
  // flat latent pyramid: the L latent grids, then n_hyper hyperlatent grids
  int NG, n_hyper, hyper_first;
  int goff[CC_MAX_G], gh[CC_MAX_G], gw[CC_MAX_G], glev[CC_MAX_G];  // glev: resolution level
  // IFCE of grid k < G: its inputs (pyramid grid, resolution shift)
  int nin[4], isrc[4][CC_MAX_NIN], ish[4][CC_MAX_NIN];
  int uoff[CC_MAX_L];           // U_j (j >= 1): (L-j) channels at grid j-1
  int ups_conv;                 // 1: level j filters T_j (7-tap Conv) before its transposed convolution
  int voff[CC_MAX_L];           // V_j = Conv_j(T_j) (j >= 1): (L-j) channels at grid j
  int dfoff[4][CC_MAX_L];       // IFCE df pyramid of child grid c at level f
  int dy[CC_MAX_S], dx[CC_MAX_S];
  // ---- parameter offsets (within the decoder parameters)
  int p_aw[3], p_ab[3], p_asw, p_asb, p_iw[4], p_ib[4], p_ups[CC_MAX_L], p_upc[CC_MAX_L];
  int p_sw[3], p_sb[3], p_ssw, p_ssb, p_rw[4], p_rb[4];
  int n_arm_par;                // ARM + IFCE parameters: [0, n_arm_par)
  // ---- scalars
  double lambda;
  float rate_scale, mse_scale, lmin, lmax, pmin, bits_max;
  unsigned seed_lo, seed_hi;
  // ---- per-step scalars (written by the quantiser kernel)
  float T, sr_c, sr_invT, sigma, lr, bc1, bc2;
  unsigned t_lo;
  int mode, upd;
  // ---- producer geometry
  int arm_nchunk, arm_nwg, syn_nchunk, syn_nwg, pix_nwg, nprod;
  int lat_ntile, pix_ntile, res_nwg;
  int ups_jc;                   // first upsampling level run by the per-source chain kernels (L: none)
  int arm_wgs;                  // fused ARM: workgroups per image (bands packed by the host)
  int syn_cpw, res_tpw;         // synthesis chunks / residual tiles per workgroup (launch shape)
  ProdSeg prod[CC_MAX_PROD];
  int prod_arm, prod_syn, prod_res0, prod_ups1, prod_upc1;   // producer indices
  int prod_ifce0;               // fused form: IFCE weight gradients of grid c from the pooling kernel
  // ---- buffers (device pointers inside the slab)
  float *img, *theta, *m, *v, *grad, *yhat, *dq, *dc, *df, *dyd, *dyq;
  float *U, *dU, *V, *dV, *X, *dXa, *dXb, *wp;
  double* wp2;
  unsigned* arm_gtab;
  unsigned* arm_ftab;           // fused ARM: parameter -> (grid, accumulator, row, column)
  // fused ARM: bands of workgroup w are arm_blist[arm_wbeg[w] .. arm_wbeg[w + 1])
  int *arm_blist, *arm_wbeg;
  int arm_nwg_plain, arm_nwg_fused, arm_fused;  // arm_fused: planes A/B hold the rate gradient
  unsigned* syn_gtab;
  double *lp_bits, *lp_mse, *scal;
  // ---- SOAP for the decoder parameters (k_soap.hip): one table row of
  // CC_SOAP_TAB ints per parameter tensor, first and second moments in
  // parameter order, then every Kronecker factor and every basis (row-major,
  // tensor by tensor, dimension by dimension)
  int soap_ntens, soap_nfac;
  int* soap_tab;
  float *soap_m, *soap_v, *soap_p, *soap_q;
  // ---- decoder-parameter quantisation (k_nnq.hip): group of every
  // parameter (2 * submodule + is_bias), the kept unquantised parameters,
  // Exp-Golomb code lengths per group and order
  unsigned char* nnq_group;
  float* nnq_keep;
  long long* nnq_bits;
};

// Read-only views used inside kernels: the descriptor and the decoder
// parameters never change during a kernel that reads them (only the
// optimiser and quantiser kernels write them, through plain pointers), so they are read in
// the constant address space, which lets uniform reads go through scalar
// loads (and weights feed FMAs as scalar operands).
typedef __attribute__((address_space(4))) const struct DevDesc CDesc;
typedef __attribute__((address_space(4))) const float CF;

// Kernel argument describing one batched launch: blockIdx.x in
// [tile0[i], tile0[i+1]) belongs to image i.
struct Launch {
  int n;
  int tile0[CC_MAX_BATCH + 1];
  const DevDesc* d[CC_MAX_BATCH];
};

struct StepArgs {
  float T, sr_c, sr_invT, sigma, lr, bc1, bc2;
  unsigned t_lo;
  int mode, upd;
};
struct StepPack {
  StepArgs a[CC_MAX_BATCH];
};
#define CC_NNQ_NG 8   // parameter groups: 4 submodules x (weights, biases)
#define CC_NNQ_NK 12  // Exp-Golomb orders 0..11
#define CC_NNQ_NSTEP 8  // quantisation steps 2^-8 .. 2^-1
// Per image: quantisation step of every group (0 = unquantised).
struct NnqPack {
  float step[CC_MAX_BATCH][CC_NNQ_NG];
};
// Per image: SOAP calls made before this one (0 = the initialising call).
struct SoapPack {
  int calls[CC_MAX_BATCH];
};

__device__ __forceinline__ int cc_find_img(const Launch& L, int b) {
  int i = 0;
  while (i + 1 < L.n && b >= L.tile0[i + 1]) ++i;
  return i;
}

// Workgroup index within image im, renumbered for the XCDs: the dispatcher
// hands consecutive workgroups of a launch to the CC_NXCD XCDs in turn, each
// XCD with its own L2, so here the workgroups of one XCD take consecutive
// indices and tiles that share halo rows or cache lines mostly run under one
// L2.  A bijection of [0, nwg): each index does the same work as before, only
// the XCD it runs on changes, so results do not depend on it.
#define CC_NXCD 8
__device__ __forceinline__ int cc_xcd_index(const Launch& L, int im) {
  const int nwg = L.tile0[im + 1] - L.tile0[im];
  const int loc = (int)blockIdx.x - L.tile0[im];
  const int q = nwg / CC_NXCD, r = nwg % CC_NXCD, o = loc % CC_NXCD;
  return o * q + min(o, r) + loc / CC_NXCD;
}

// -------------------------------------------------------------- host side
// Launchers implemented in the kernel translation units.
struct HostImg;  // defined in cc_api.hip
int cc_launch_qtrain(const Launch& l, const StepPack& a, hipStream_t st);
int cc_launch_arm(const Launch& l, const DevDesc& h, int bwd, int precision, hipStream_t st);
int cc_launch_pool(const Launch& l, hipStream_t st);
int cc_launch_join(const Launch& l, hipStream_t st, float* rate_only_out = nullptr, int adam = 0);
// join + first reduction pass in one launch (lj: lat_ntile + the reduction's
// blocks per image; the latents' Adam update when adam_latents); the second
// pass (the parameters' Adam update when adam_params)
int cc_launch_join_wreduce1(const Launch& lj, int adam_latents, hipStream_t st);
int cc_launch_wreduce2(const Launch& l2, int adam_params, hipStream_t st);
int cc_launch_poke(float* p, float v, hipStream_t st);
int cc_launch_ups_fwd(const Launch& l, int j, hipStream_t st);
int cc_launch_ups_bwd(const Launch& l, int j, hipStream_t st);
int cc_launch_ups_fwd_chain(const Launch& l, hipStream_t st);
int cc_launch_upc_fwd(const Launch& l, int j, hipStream_t st);
int cc_launch_upc_bwd(const Launch& l, int j, hipStream_t st);
int cc_launch_ups_bwd_chain(const Launch& l, hipStream_t st);
int cc_launch_syn_fwd(const Launch& l, const DevDesc& h, int final_mse, int precision, hipStream_t st);
int cc_launch_syn_bwd(const Launch& l, const DevDesc& h, int precision, hipStream_t st);
int cc_launch_res_fwd(const Launch& l, int r, int last, int want_mse, hipStream_t st);
int cc_launch_res_bwd(const Launch& l, int r, hipStream_t st);
int cc_launch_wreduce(const Launch& l1, const Launch& l2, int adam, hipStream_t st);
int cc_launch_lreduce(const Launch& l, hipStream_t st);
int cc_launch_copy_out(const Launch& l, float* out, hipStream_t st);
int cc_launch_soap(const Launch& l, const SoapPack& a, hipStream_t st);
int cc_launch_nnq(const Launch& l, const NnqPack& a, hipStream_t st);

// Tile geometry shared by host launch planning and kernels.
#define CC_ELT_TILE 256     // elementwise kernels: threads per block
#define CC_ARM_CHUNK 64     // ARM kernel: positions per chunk (= threads per block)
#define CC_ARM_CPW 4        // ARM kernel: chunks per workgroup
#define CC_SYN_CHUNK 64
#ifndef CC_SYN_CPW
#define CC_SYN_CPW 12       // synthesis backward: default chunks per workgroup
#endif
#define CC_SYN_CPW_MIN 4    // smallest tunable (the partial-row space is sized for it)
#define CC_SYN_CPW_MAX 64
#define CC_RES_TPW_MAX 16   // residual adjoint: largest tunable tiles per workgroup
#define CC_PIX_TILE 256     // per-pixel kernels (res conv, ups): threads per block
#define CC_WRED_SPLIT 32    // weight-gradient reduction: row splits of pass 1
#define CC_FUSED_BAND 2     // fused ARM kernel: rows per band (a multiple of 2)
#define CC_FUSED_HALO 4     // fused ARM kernel: causal reach in rows (and columns each side)
// halo planes of the fused ARM's context gradient: the bands above that a
// band's causal halo rows reach
#define CC_FUSED_HPLANES ((CC_FUSED_HALO + CC_FUSED_BAND - 1) / CC_FUSED_BAND)
#ifndef CC_FUSED_MAXWG
#define CC_FUSED_MAXWG 512  // fused ARM kernel: workgroups per image (each takes every n-th band)
#endif
#ifndef CC_UPS_TILE
#define CC_UPS_TILE 16      // upsampling adjoint: input tile side
#endif
#ifndef CC_SYN_BWD_WAVES
#define CC_SYN_BWD_WAVES 8   // waves per synthesis-backward workgroup (4 or 8)
#endif
#define CC_UPC_TH 16        // upsampling Conv (forward and adjoint): tile rows
#define CC_UPC_TW 64        // and columns
#define CC_UPS_COARSE 2048  // upsampling levels whose output grid has at most this many positions
                            // run as one workgroup per source grid, all such levels in LDS
#ifndef CC_UPS_CHAIN_T
#define CC_UPS_CHAIN_T 1024 // threads of those workgroups
#endif
#define CC_SOAP_TAB 12       // SOAP table row: poff, numel, ndim, dims[4], factor offsets[4], pad
#define CC_SOAP_MAXDIM 48    // SOAP: dimensions above this get no Kronecker factor
#define CC_SOAP_MAXNUMEL 1024  // SOAP: largest parameter tensor
#define CC_SOAP_REFRESH 10   // SOAP: basis refresh every this many updates
#define CC_SOAP_QR_TOL 1e-5  // SOAP: relative residual below which a refreshed column is replaced
#define CC_POOL_BLOCK 64    // IFCE gradient pooling: largest base block side (L <= 7)
#ifndef CC_RES_TH
#define CC_RES_TH 8         // residual-layer adjoint: tile rows (a multiple of 4)
#endif
#define CC_RES_TW 64        // residual-layer adjoint: tile columns (one per lane)
#ifndef CC_RES_TPW
#define CC_RES_TPW 1        // residual-layer adjoint: tiles per workgroup
#endif

int cc_arm_fused_supported(const DevDesc& h);
