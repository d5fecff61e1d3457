// SOAP for the decoder parameters (Section IV-B): Adam run in the eigenbases
// of Shampoo's Kronecker-factored preconditioner (Vyas et al., 2024), the
// latents keeping plain Adam.  The paper does not state SOAP's settings; the
// published defaults are used: beta1 = beta2 = 0.95, factor average 0.95,
// eps 1e-8, basis refresh every 10 updates, bias correction, no weight decay.
//
// One workgroup per parameter tensor.  A tensor of two or more dimensions
// has one factor P_d per dimension d (the mode-d Gram matrix of its
// gradient, averaged) unless the dimension exceeds CC_SOAP_MAXDIM; other
// tensors have none, which makes their update Adam in SOAP's step form.
//   first call   P_d = (1 - b) G_(d) G_(d)^T, Q_d = its eigenvectors by
//                descending eigenvalue (cyclic Jacobi in FP64); no update;
//   later calls  s = number of updates; M <- b1 M + (1 - b1) G (original
//                coordinates); G', M' = G, M rotated into the bases
//                (x_d Q_d^T for every d); V <- b2 V + (1 - b2) G'^2 (rotated
//                coordinates); theta -= lr sqrt(1 - b2^s) / (1 - b1^s)
//                * rotate_back(M' / (sqrt(V) + eps)); then P_d <- b P_d +
//                (1 - b) G_(d) G_(d)^T and, when s is a multiple of 10, per
//                dimension in order: rank the columns of Q_d by the estimated
//                eigenvalues diag(Q^T P Q), descending (ties by index),
//                permute V along d the same way, and take one power step
//                Q_d <- qr(P_d Q_d) (Gram-Schmidt with one re-orthogonalisation
//                pass, so R has a positive diagonal; columns that vanish
//                replaced by unit vectors, see qr_gs).
#include "cc_internal.h"

#include <math.h>

namespace {

constexpr float B1 = 0.95f, B2 = 0.95f, BP = 0.95f, EPS = 1e-8f;
constexpr int MAXN = CC_SOAP_MAXDIM;
constexpr int MAXE = CC_SOAP_MAXNUMEL;
constexpr int NT = 512;

struct Ten {
  int poff, numel, ndim, dim[4], fac[4];
};

__device__ Ten load_ten(const CDesc* d, int t) {
  const int* r = d->soap_tab + (size_t)t * CC_SOAP_TAB;
  Ten T;
  T.poff = r[0];
  T.numel = r[1];
  T.ndim = r[2];
  for (int i = 0; i < 4; ++i) {
    T.dim[i] = r[3 + i];
    T.fac[i] = r[7 + i];
  }
  return T;
}

__device__ __forceinline__ int stride_of(const Ten& T, int dd) {
  int s = 1;
#pragma unroll
  for (int e = 1; e < 4; ++e)
    if (e > dd && e < T.ndim) s *= T.dim[e];
  return s;
}

__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

// out = in x_d Q^T (fwd: out[..i..] = sum_j Q[j][i] in[..j..]) or in x_d Q
// (back: out[..i..] = sum_j Q[i][j] in[..j..]); Q staged in LDS.
__device__ void mode_product(const float* in, float* out, const Ten& T, int dd, const float* Q,
                             bool fwd) {
  const int n = T.dim[dd], st = stride_of(T, dd);
  // element (r, c) of the operator applied along dd: Q[c][r] forward, Q[r][c] back
  const int rs = fwd ? 1 : n, cs = fwd ? n : 1;
  for (int i = threadIdx.x; i < T.numel; i += NT) {
    const int id = (i / st) % n;
    const int base = i - id * st;
    const float* q = Q + id * rs;
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
    int j = 0;
    for (; j + 3 < n; j += 4) {
      s0 += q[j * cs] * in[base + j * st];
      s1 += q[(j + 1) * cs] * in[base + (j + 1) * st];
      s2 += q[(j + 2) * cs] * in[base + (j + 2) * st];
      s3 += q[(j + 3) * cs] * in[base + (j + 3) * st];
    }
    for (; j < n; ++j) s0 += q[j * cs] * in[base + j * st];
    out[i] = (s0 + s1) + (s2 + s3);
  }
}

// Rotates src along every factored dimension (bases in qall, at the
// tensor-local offsets qo), alternating between the scratch buffers a and b;
// returns the buffer holding the result (src itself if no dimension is
// factored).  src is not modified.
__device__ float* rotate(float* src, float* a, float* b, const float* qall, const Ten& T,
                         bool fwd) {
  float* cur = src;
  float* nxt = a;
  int off = 0;
  #pragma unroll
  for (int dd = 0; dd < 4; ++dd) {
    if (dd >= T.ndim || T.fac[dd] < 0) continue;
    mode_product(cur, nxt, T, dd, qall + off, fwd);
    off += T.dim[dd] * T.dim[dd];
    __syncthreads();
    cur = nxt;
    nxt = (nxt == a) ? b : a;
  }
  return cur;
}

// G_(d) G_(d)^T (n x n) of the tensor held in g, entry (a, b).
__device__ float gram_entry(const float* g, const Ten& T, int dd, int a, int b) {
  const int n = T.dim[dd], st = stride_of(T, dd), outer = T.numel / (n * st);
  const int cnt = outer * st;   // pairs summed: (o, in) in row-major order
  float s0 = 0.0f, s1 = 0.0f;
  int e = 0;
  for (; e + 1 < cnt; e += 2) {
    const int o0 = e / st, i0 = e - o0 * st, o1 = (e + 1) / st, i1 = e + 1 - o1 * st;
    const int b0 = o0 * n * st + i0, b1 = o1 * n * st + i1;
    s0 += g[b0 + a * st] * g[b0 + b * st];
    s1 += g[b1 + a * st] * g[b1 + b * st];
  }
  if (e < cnt) {
    const int o0 = e / st, i0 = e - o0 * st, b0 = o0 * n * st + i0;
    s0 += g[b0 + a * st] * g[b0 + b * st];
  }
  return s0 + s1;
}

// Stable descending ranking: order[k] = index of the k-th largest value.
__device__ void rank_desc(const double* val, int n, int* order) {
  for (int i = threadIdx.x; i < n; i += NT) {
    int r = 0;
    for (int j = 0; j < n; ++j) r += (val[j] > val[i]) || (val[j] == val[i] && j < i);
    order[r] = i;
  }
}

// Eigenvectors of the symmetric n x n matrix in A (FP64, destroyed) into
// the columns of Vm, by descending eigenvalue: cyclic Jacobi with the
// round-robin pairing (n/2 disjoint rotations at a time).
__device__ void jacobi_eig(double* A, double* Vm, int n, double* wk, int* order, double* red,
                           float* qout) {
  __shared__ double rc[MAXN / 2 + 1], rs[MAXN / 2 + 1];
  __shared__ int rp[MAXN / 2 + 1], rq[MAXN / 2 + 1];
  for (int i = threadIdx.x; i < n * n; i += NT) Vm[i] = (i / n == i % n) ? 1.0 : 0.0;
  const int m = n + (n & 1), npair = m / 2;
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = threadIdx.x; i < n * n; i += NT) {
      const double a = A[i];
      tot += a * a;
      if (i / n != i % n) off += a * a;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (!(off > 1e-28 * tot)) break;
    for (int r = 0; r < m - 1; ++r) {
      if ((int)threadIdx.x < npair) {
        const int k = threadIdx.x;
        auto pos = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + r) % (m - 1); };
        int p = pos(k), q = pos(m - 1 - k);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          if (fabs(apq) > 1e-300) {
            const double th = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
            const double t = fabs(th) > 1e150 ? 0.5 / th
                                              : (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        rc[k] = c;
        rs[k] = s;
        rp[k] = p;
        rq[k] = q < n ? q : -1;
      }
      __syncthreads();
      // rows p, q of A <- J^T A
      for (int i = threadIdx.x; i < npair * n; i += NT) {
        const int k = i / n, j = i - k * n, p = rp[k], q = rq[k];
        if (q < 0) continue;
        const double c = rc[k], s = rs[k];
        const double ap = A[p * n + j], aq = A[q * n + j];
        A[p * n + j] = c * ap - s * aq;
        A[q * n + j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns p, q of A <- A J and of V <- V J
      for (int i = threadIdx.x; i < npair * n; i += NT) {
        const int k = i / n, row = i - k * n, p = rp[k], q = rq[k];
        if (q < 0) continue;
        const double c = rc[k], s = rs[k];
        const double ap = A[row * n + p], aq = A[row * n + q];
        A[row * n + p] = c * ap - s * aq;
        A[row * n + q] = s * ap + c * aq;
        const double vp = Vm[row * n + p], vq = Vm[row * n + q];
        Vm[row * n + p] = c * vp - s * vq;
        Vm[row * n + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += NT) wk[i] = A[i * n + i];
  __syncthreads();
  rank_desc(wk, n, order);
  __syncthreads();
  for (int i = threadIdx.x; i < n * n; i += NT) {
    const int row = i / n, k = i - row * n;
    qout[i] = (float)Vm[row * n + order[k]];
  }
  __syncthreads();
}

// Q <- qr(Z) for the n x n matrix Z in A (FP64, columns replaced by Q in
// order): Gram-Schmidt with one re-orthogonalisation pass, so R has a
// positive diagonal.  A rank-deficient Z has no unique factorisation (its
// trailing columns would be set by rounding), so a column whose norm after
// orthogonalisation is below CC_SOAP_QR_TOL of its norm before is replaced
// by the first unit vector e_k, e_(k+1), ... (cyclic) that survives the same
// orthogonalisation.  rj, zc: scratch of n doubles each.
__device__ void qr_gs(double* A, int n, double* rj, double* zc, double* red) {
  constexpr int GRP = 8;   // threads per dot product
  const int tid = threadIdx.x, g = tid / GRP, l = tid % GRP;
  for (int k = 0; k < n; ++k) {
    double nv = 0.0;
    for (int cand = 0; cand <= n; ++cand) {
      const int e = (k + cand - 1) % n;
      for (int a = tid; a < n; a += NT) zc[a] = cand == 0 ? A[a * n + k] : (a == e ? 1.0 : 0.0);
      __syncthreads();
      double n0 = 0.0;
      for (int a = tid; a < n; a += NT) n0 += zc[a] * zc[a];
      n0 = sqrt(block_sum(n0, red));
      for (int pass = 0; pass < 2; ++pass) {
        for (int j = g; j < k; j += NT / GRP) {
          double r = 0.0;
          for (int a = l; a < n; a += GRP) r += A[a * n + j] * zc[a];
          for (int off = GRP / 2; off > 0; off >>= 1) r += __shfl_xor(r, off, GRP);
          if (l == 0) rj[j] = r;
        }
        __syncthreads();
        for (int a = g; a < n; a += NT / GRP) {
          double u = 0.0;
          for (int j = l; j < k; j += GRP) u += rj[j] * A[a * n + j];
          for (int off = GRP / 2; off > 0; off >>= 1) u += __shfl_xor(u, off, GRP);
          if (l == 0) zc[a] -= u;
        }
        __syncthreads();
      }
      nv = 0.0;
      for (int a = tid; a < n; a += NT) nv += zc[a] * zc[a];
      nv = sqrt(block_sum(nv, red));
      if (n0 > 0.0 && nv > CC_SOAP_QR_TOL * n0) break;
    }
    for (int a = tid; a < n; a += NT) A[a * n + k] = zc[a] / nv;
    __syncthreads();
  }
}

__global__ __launch_bounds__(NT) void k_soap(Launch L, SoapPack A) {
  // float work buffers and the FP64 buffers of the basis computations share
  // storage (never live at the same time)
  constexpr int UF = 6 * MAXE;
  constexpr int UD = 2 * MAXN * MAXN;
  constexpr int UBYTES = (UF * 4 > UD * 8 ? UF * 4 : UD * 8);
  __shared__ __align__(16) char ubuf[UBYTES];
  __shared__ float fv[MAXE];
  __shared__ float qall[2 * MAXN * MAXN], pall[2 * MAXN * MAXN];
  __shared__ double wk[MAXN], zcol[MAXN], red[NT / 64];
  __shared__ int order[MAXN];
  float* fg = reinterpret_cast<float*>(ubuf);
  float* fm = fg + MAXE;
  float* fth = fm + MAXE;
  float* w0 = fth + MAXE;
  float* w1 = w0 + MAXE;
  float* w2 = w1 + MAXE;
  double* dA = reinterpret_cast<double*>(ubuf);
  double* dB = dA + MAXN * MAXN;

  const int im = cc_find_img(L, blockIdx.x);
  const CDesc* d = (const CDesc*)L.d[im];
  const int t = blockIdx.x - L.tile0[im];
  const int calls = A.calls[im];
  const Ten T = load_ten(d, t);
  const int tid = threadIdx.x;
  const float* grad = d->grad + d->n_lat + T.poff;
  float* theta = d->theta + d->n_lat + T.poff;
  float* M = d->soap_m + T.poff;
  float* V = d->soap_v + T.poff;
  // the factors (and bases) of one tensor are contiguous in the state; in
  // pall / qall they start at 0, dimension by dimension
  int nf = 0;
#pragma unroll
  for (int dd = 0; dd < 4; ++dd)
    if (dd < T.ndim && T.fac[dd] >= 0) nf += T.dim[dd] * T.dim[dd];
  int f0 = -1;
#pragma unroll
  for (int dd = 0; dd < 4; ++dd)
    if (dd < T.ndim && T.fac[dd] >= 0 && f0 < 0) f0 = T.fac[dd];

  if (calls == 0) {
    // initialising call: factors and their eigenbases, no update (the
    // gradient is held in fv, outside the storage the FP64 buffers share)
    for (int i = tid; i < T.numel; i += NT) fv[i] = grad[i];
    __syncthreads();
    int off = 0;
    #pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
      if (dd >= T.ndim || T.fac[dd] < 0) continue;
      const int n = T.dim[dd];
      for (int i = tid; i < n * n; i += NT) {
        const float p = (1.0f - BP) * gram_entry(fv, T, dd, i / n, i % n);
        d->soap_p[T.fac[dd] + i] = p;
        dA[i] = (double)p;
      }
      __syncthreads();
      jacobi_eig(dA, dB, n, wk, order, red, qall + off);
      for (int i = tid; i < n * n; i += NT) d->soap_q[T.fac[dd] + i] = qall[off + i];
      __syncthreads();
      off += n * n;
    }
    return;
  }

  // everything this tensor needs, in one round of loads
  for (int i = tid; i < T.numel; i += NT) {
    fg[i] = grad[i];
    fm[i] = M[i];
    fv[i] = V[i];
    fth[i] = theta[i];
  }
  if (f0 >= 0)
    for (int i = tid; i < nf; i += NT) {
      qall[i] = d->soap_q[f0 + i];
      pall[i] = d->soap_p[f0 + i];
    }
  __syncthreads();

  const int s = calls;
  const double scale =
      (double)d->lr * sqrt(1.0 - pow((double)B2, (double)s)) / (1.0 - pow((double)B1, (double)s));
  // first moment (original coordinates)
  for (int i = tid; i < T.numel; i += NT) {
    const float m = B1 * fm[i] + (1.0f - B1) * fg[i];
    fm[i] = m;
    M[i] = m;
  }
  __syncthreads();
  // second moment in the rotated coordinates
  const float* gr = rotate(fg, w0, w1, qall, T, true);
  for (int i = tid; i < T.numel; i += NT) {
    const float v = B2 * fv[i] + (1.0f - B2) * gr[i] * gr[i];
    fv[i] = v;
    V[i] = v;
  }
  __syncthreads();
  // update: rotate_back(rotate(M) / (sqrt(V) + eps))
  float* mr = rotate(fm, w0, w1, qall, T, true);
  for (int i = tid; i < T.numel; i += NT) mr[i] = mr[i] / (sqrtf(fv[i]) + EPS);
  __syncthreads();
  float* sa = mr == w0 ? w1 : w0;
  float* sb = (mr == w2 || sa == w2) ? (mr == w1 || sa == w1 ? w0 : w1) : w2;
  const float* nb = rotate(mr, sa, sb, qall, T, false);
  for (int i = tid; i < T.numel; i += NT) theta[i] = fth[i] - (float)(scale * (double)nb[i]);

  // factors with this gradient
  {
    int off = 0;
    #pragma unroll
    for (int dd = 0; dd < 4; ++dd) {
      if (dd >= T.ndim || T.fac[dd] < 0) continue;
      const int n = T.dim[dd];
      for (int i = tid; i < n * n; i += NT) {
        const float p = BP * pall[off + i] + (1.0f - BP) * gram_entry(fg, T, dd, i / n, i % n);
        pall[off + i] = p;
        d->soap_p[T.fac[dd] + i] = p;
      }
      off += n * n;
    }
  }
  __syncthreads();
  if (s % CC_SOAP_REFRESH != 0) return;

  // periodic basis refresh, dimension by dimension (the FP64 buffers reuse
  // the float work storage from here on)
  int off = 0;
  #pragma unroll
  for (int dd = 0; dd < 4; ++dd) {
    if (dd >= T.ndim || T.fac[dd] < 0) continue;
    const int n = T.dim[dd];
    const float* P = pall + off;
    float* Q = qall + off;
    off += n * n;
    // W = P Q, estimated eigenvalues diag(Q^T W)
    for (int i = tid; i < n * n; i += NT) {
      const int a = i / n, c = i - a * n;
      double w = 0.0;
      for (int b = 0; b < n; ++b) w += (double)P[a * n + b] * (double)Q[b * n + c];
      dB[i] = w;
    }
    __syncthreads();
    for (int c = tid; c < n; c += NT) {
      double e = 0.0;
      for (int a = 0; a < n; ++a) e += (double)Q[a * n + c] * dB[a * n + c];
      wk[c] = e;
    }
    __syncthreads();
    rank_desc(wk, n, order);
    __syncthreads();
    // V permuted along dd; Z = P Q[:, order] into dA
    const int st = stride_of(T, dd);
    for (int i = tid; i < T.numel; i += NT) {
      const int id = (i / st) % n;
      V[i] = fv[i + (order[id] - id) * st];
    }
    for (int i = tid; i < n * n; i += NT) {
      const int a = i / n, k = i - a * n;
      dA[i] = dB[a * n + order[k]];
    }
    __syncthreads();
    for (int i = tid; i < T.numel; i += NT) fv[i] = V[i];
    qr_gs(dA, n, wk, zcol, red);
    for (int i = tid; i < n * n; i += NT) {
      const float q = (float)dA[i];
      Q[i] = q;
      d->soap_q[T.fac[dd] + i] = q;
    }
    __syncthreads();
  }
}

inline int check_launch() { return hipGetLastError() == hipSuccess ? CC_OK : CC_EDEVICE; }

}  // namespace

int cc_launch_soap(const Launch& l, const SoapPack& a, hipStream_t st) {
  if (l.tile0[l.n] == 0) return CC_OK;
  hipLaunchKernelGGL(k_soap, dim3(l.tile0[l.n]), dim3(NT), 0, st, l, a);
  return check_launch();
}
