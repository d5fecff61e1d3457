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
//                pass, so R has a positive diagonal).
#include "cc_internal.h"

#include <math.h>

namespace {

constexpr float B1 = 0.95f, B2 = 0.95f, BP = 0.95f, EPS = 1e-8f;
constexpr int MAXN = CC_SOAP_MAXDIM;
constexpr int MAXE = CC_SOAP_MAXNUMEL;
constexpr int NT = 256;

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

__device__ int stride_of(const Ten& T, int dd) {
  int s = 1;
  for (int e = dd + 1; e < T.ndim; ++e) s *= T.dim[e];
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
  for (int i = threadIdx.x; i < T.numel; i += NT) {
    const int id = (i / st) % n;
    const int base = i - id * st;
    float s = 0.0f;
    for (int j = 0; j < n; ++j) s += (fwd ? Q[j * n + id] : Q[id * n + j]) * in[base + j * st];
    out[i] = s;
  }
}

// Rotates buf (in place via the scratch buffer) along every factored
// dimension; returns the buffer holding the result.
__device__ float* rotate(float* buf, float* tmp, float* qs, const CDesc* d, const Ten& T, bool fwd) {
  for (int dd = 0; dd < T.ndim; ++dd) {
    if (T.fac[dd] < 0) continue;
    const int n = T.dim[dd];
    for (int i = threadIdx.x; i < n * n; i += NT) qs[i] = d->soap_q[T.fac[dd] + i];
    __syncthreads();
    mode_product(buf, tmp, T, dd, qs, fwd);
    __syncthreads();
    float* x = buf;
    buf = tmp;
    tmp = x;
  }
  return buf;
}

// G_(d) G_(d)^T (n x n) of the tensor held in g, entry (a, b).
__device__ float gram_entry(const float* g, const Ten& T, int dd, int a, int b) {
  const int n = T.dim[dd], st = stride_of(T, dd), outer = T.numel / (n * st);
  float s = 0.0f;
  for (int o = 0; o < outer; ++o)
    for (int in = 0; in < st; ++in) {
      const int base = o * n * st + in;
      s += g[base + a * st] * g[base + b * st];
    }
  return s;
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

// Q <- qr(Z) for the n x n matrix Z in A (FP64, columns orthonormalised in
// place, in order); classical Gram-Schmidt with one re-orthogonalisation
// pass.  A column that vanishes against the earlier ones is replaced by the
// unit vector of its index, orthogonalised the same way.
__device__ void gram_schmidt(double* A, int n, double* wk, double* red) {
  for (int k = 0; k < n; ++k) {
    double n0 = 0.0;
    for (int a = threadIdx.x; a < n; a += NT) n0 += A[a * n + k] * A[a * n + k];
    n0 = block_sum(n0, red);
    for (int attempt = 0; attempt < 2; ++attempt) {
      if (attempt == 1) {
        for (int a = threadIdx.x; a < n; a += NT) A[a * n + k] = (a == k) ? 1.0 : 0.0;
        n0 = 1.0;
        __syncthreads();
      }
      for (int pass = 0; pass < 2; ++pass) {
        for (int j = threadIdx.x; j < k; j += NT) {
          double r = 0.0;
          for (int a = 0; a < n; ++a) r += A[a * n + j] * A[a * n + k];
          wk[j] = r;
        }
        __syncthreads();
        for (int a = threadIdx.x; a < n; a += NT) {
          double z = A[a * n + k];
          for (int j = 0; j < k; ++j) z -= wk[j] * A[a * n + j];
          A[a * n + k] = z;
        }
        __syncthreads();
      }
      double nn = 0.0;
      for (int a = threadIdx.x; a < n; a += NT) nn += A[a * n + k] * A[a * n + k];
      nn = block_sum(nn, red);
      if (nn > 1e-26 * n0 && nn > 0.0) {
        const double inv = 1.0 / sqrt(nn);
        for (int a = threadIdx.x; a < n; a += NT) A[a * n + k] *= inv;
        __syncthreads();
        break;
      }
    }
  }
}

__global__ __launch_bounds__(NT) void k_soap(Launch L, SoapPack A) {
  __shared__ double dA[MAXN * MAXN], dB[MAXN * MAXN];
  __shared__ float f0[MAXE], f1[MAXE], f2[MAXE];
  __shared__ float qs[MAXN * MAXN];
  __shared__ double wk[MAXN], red[NT / 64];
  __shared__ int order[MAXN];
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

  for (int i = tid; i < T.numel; i += NT) f0[i] = grad[i];
  __syncthreads();

  if (calls == 0) {
    // initialising call: factors and their eigenbases, no update
    for (int dd = 0; dd < T.ndim; ++dd) {
      if (T.fac[dd] < 0) continue;
      const int n = T.dim[dd];
      for (int i = tid; i < n * n; i += NT) {
        const float p = (1.0f - BP) * gram_entry(f0, T, dd, i / n, i % n);
        d->soap_p[T.fac[dd] + i] = p;
        dA[i] = (double)p;
      }
      __syncthreads();
      jacobi_eig(dA, dB, n, wk, order, red, qs);
      for (int i = tid; i < n * n; i += NT) d->soap_q[T.fac[dd] + i] = qs[i];
      __syncthreads();
    }
    return;
  }

  const int s = calls;
  const double scale =
      (double)d->lr * sqrt(1.0 - pow((double)B2, (double)s)) / (1.0 - pow((double)B1, (double)s));
  // first moment (original coordinates)
  for (int i = tid; i < T.numel; i += NT) {
    const float m = B1 * M[i] + (1.0f - B1) * f0[i];
    M[i] = m;
    f1[i] = m;
  }
  __syncthreads();
  // second moment in the rotated coordinates
  float* gr = rotate(f0, f2, qs, d, T, true);
  for (int i = tid; i < T.numel; i += NT) {
    const float v = B2 * V[i] + (1.0f - B2) * gr[i] * gr[i];
    V[i] = v;
    gr[i] = v;
  }
  __syncthreads();
  float* freeb = gr == f0 ? f2 : f0;
  float* mr = rotate(f1, freeb, qs, d, T, true);
  for (int i = tid; i < T.numel; i += NT) mr[i] = mr[i] / (sqrtf(gr[i]) + EPS);
  __syncthreads();
  freeb = mr == f1 ? freeb : f1;
  float* nb = rotate(mr, freeb, qs, d, T, false);
  for (int i = tid; i < T.numel; i += NT) theta[i] -= (float)(scale * (double)nb[i]);
  __syncthreads();

  // factors with this gradient, and the periodic basis refresh
  for (int i = tid; i < T.numel; i += NT) f0[i] = grad[i];
  __syncthreads();
  for (int dd = 0; dd < T.ndim; ++dd) {
    if (T.fac[dd] < 0) continue;
    const int n = T.dim[dd];
    for (int i = tid; i < n * n; i += NT) {
      float* p = d->soap_p + T.fac[dd] + i;
      *p = BP * *p + (1.0f - BP) * gram_entry(f0, T, dd, i / n, i % n);
    }
  }
  __syncthreads();
  if (s % CC_SOAP_REFRESH != 0) return;
  for (int dd = 0; dd < T.ndim; ++dd) {
    if (T.fac[dd] < 0) continue;
    const int n = T.dim[dd];
    const float* P = d->soap_p + T.fac[dd];
    float* Q = d->soap_q + T.fac[dd];
    for (int i = tid; i < n * n; i += NT) dA[i] = (double)Q[i];
    __syncthreads();
    // W = P Q, estimated eigenvalues diag(Q^T W)
    for (int i = tid; i < n * n; i += NT) {
      const int a = i / n, c = i - a * n;
      double w = 0.0;
      for (int b = 0; b < n; ++b) w += (double)P[a * n + b] * dA[b * n + c];
      dB[i] = w;
    }
    __syncthreads();
    for (int c = tid; c < n; c += NT) {
      double e = 0.0;
      for (int a = 0; a < n; ++a) e += dA[a * n + c] * dB[a * n + c];
      wk[c] = e;
    }
    __syncthreads();
    rank_desc(wk, n, order);
    __syncthreads();
    // V permuted along dd; Z = P Q[:, order] into dA
    const int st = stride_of(T, dd);
    for (int i = tid; i < T.numel; i += NT) f0[i] = V[i];
    __syncthreads();
    for (int i = tid; i < T.numel; i += NT) {
      const int id = (i / st) % n;
      V[i] = f0[i + (order[id] - id) * st];
    }
    for (int i = tid; i < n * n; i += NT) {
      const int a = i / n, k = i - a * n;
      dA[i] = dB[a * n + order[k]];
    }
    __syncthreads();
    gram_schmidt(dA, n, wk, red);
    for (int i = tid; i < n * n; i += NT) Q[i] = (float)dA[i];
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
