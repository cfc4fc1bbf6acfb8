// FP64 dense linear algebra used by the stabilization of the B-chains:
// an MFMA GEMM, a blocked Householder QR (compact WY form, panel factored in
// registers by one workgroup), a blocked upper-triangular solve and small
// elementwise helpers.  All on the context's stream.
#include <algorithm>

#include "common.h"

namespace kdqmc {

typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// GEMM: C = alpha op(A) op(B) + beta C, row-major, 64 x 64 tile per
// workgroup, K staged through LDS in steps of 16, v_mfma_f64_16x16x4.
// ---------------------------------------------------------------------------
template <bool TA, bool TB>
__global__ void __launch_bounds__(256)
k_gemm_f64(int M, int N, int K, double alpha, const double* __restrict__ A, int lda,
           const double* __restrict__ B, int ldb, double beta, double* __restrict__ C, int ldc) {
  __shared__ double As[16][64 + 2];
  __shared__ double Bs[16][64 + 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  v4d acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;  // 0..1023
      int i, k;
      if (TA) { i = e & 63; k = e >> 6; } else { k = e & 15; i = e >> 4; }
      const int gi = m0 + i, gk = k0 + k;
      double v = 0.0;
      if (gi < M && gk < K) v = TA ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk];
      As[k][i] = v;
      int j, kk;
      if (TB) { kk = e & 15; j = e >> 4; } else { j = e & 63; kk = e >> 6; }
      const int gj = n0 + j, gkk = k0 + kk;
      double w = 0.0;
      if (gj < N && gkk < K) w = TB ? B[(size_t)gj * ldb + gkk] : B[(size_t)gkk * ldb + gj];
      Bs[kk][j] = w;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
      double a[2], b[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        a[bi] = As[k4 + lk][wr + 16 * bi + lr];
        b[bi] = Bs[k4 + lk][wc + 16 * bi + lr];
      }
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = m0 + wr + 16 * bi + lk + 4 * j, cc = n0 + wc + 16 * bj + lr;
        if (r < M && cc < N) {
          double v = alpha * acc[bi][bj][j];
          if (beta != 0.0) v += beta * C[(size_t)r * ldc + cc];
          C[(size_t)r * ldc + cc] = v;
        }
      }
}

int gemm_f64(kdqmc_ctx* c, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
             int lda, const double* B, int ldb, double beta, double* C, int ldc) {
  if (M <= 0 || N <= 0) return KDQMC_OK;
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  const int e0 = prof_mark(c);
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm_f64<false, false>), grid, dim3(256), 0, c->stream, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm_f64<true, false>), grid, dim3(256), 0, c->stream, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm_f64<false, true>), grid, dim3(256), 0, c->stream, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  else
    hipLaunchKernelGGL((k_gemm_f64<true, true>), grid, dim3(256), 0, c->stream, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  prof_pair(c, PH_GEMM, e0, prof_mark(c));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

// ---------------------------------------------------------------------------
// Householder panel: one workgroup of 1024 threads factors the m x nbp panel (nbp <= 16)
// A[j:n, j:j+nbp] held in registers (thread t owns rows j+t and j+t+1024).
// H_c = I - tau_c v_c v_c^T with v_c[jc] = 1 (LAPACK convention); the block
// reflector H_0 ... H_{nbp-1} = I - V T V^T.  Outputs: R in A (zeros below
// the diagonal of the panel), explicit V in Vq (unit diagonal, zeros above),
// T in Tq (nbp x nbp, row stride 16), tau.
// ---------------------------------------------------------------------------
constexpr int kNB = 16;
constexpr int kPanelThreads = 1024;

// Sum of vals[0..kNB) over the workgroup (vals is consumed); result in out[]
// (LDS) for every thread.
__device__ __forceinline__ void block_reduce_nb(double (&cur)[kNB], double* red, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // transposed butterfly: after log2(kNB) stages lane holds the partial sum
  // of value (lane % kNB) over the lanes that share bits >= log2(kNB)
  int cnt = kNB;
#pragma unroll
  for (int b = 0; (1 << b) < kNB; ++b) {
    const int bit = (lane >> b) & 1;
    cnt >>= 1;
#pragma unroll
    for (int i = 0; i < kNB / 2; ++i) {
      if (i < cnt) {
        const double keep = bit ? cur[2 * i + 1] : cur[2 * i];
        const double send = bit ? cur[2 * i] : cur[2 * i + 1];
        cur[i] = keep + __shfl_xor(send, 1 << b);
      }
    }
  }
  double v = cur[0];
#pragma unroll
  for (int o = kNB; o < 64; o <<= 1) v += __shfl_xor(v, o);
  if (lane < kNB) red[wave * kNB + lane] = v;
  __syncthreads();
  if (threadIdx.x < kNB) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w * kNB + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ double block_reduce1(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

template <int RPT>
__global__ void __launch_bounds__(kPanelThreads)
k_qr_panel(double* __restrict__ A, int lda, int n, int j, int nbp, double* __restrict__ Vq,
           double* __restrict__ Tq, double* __restrict__ tau_out) {
  __shared__ double red[16 * kNB];
  __shared__ double dots[kNB];
  __shared__ double Ts[kNB][kNB + 1];
  __shared__ double betas[kNB];
  __shared__ double taus[kNB];
  __shared__ double bcast[2];
  const int tid = threadIdx.x;
  double a[RPT][kNB];
  int row[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    row[q] = j + tid + q * kPanelThreads;
#pragma unroll
    for (int cc = 0; cc < kNB; ++cc)
      a[q][cc] = (row[q] < n && cc < nbp) ? A[(size_t)row[q] * lda + j + cc] : 0.0;
  }
  for (int idx = tid; idx < kNB * (kNB + 1); idx += kPanelThreads) (&Ts[0][0])[idx] = 0.0;
  __syncthreads();

#pragma unroll 1
  for (int cc = 0; cc < nbp; ++cc) {
    const int jc = j + cc;
    // norm^2 of column cc over rows >= jc, and the diagonal value
    double ss = 0.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      double x = 0.0;
#pragma unroll
      for (int t = 0; t < kNB; ++t)
        if (t == cc) x = a[q][t];
      if (row[q] >= jc && row[q] < n) ss += x * x;
      if (row[q] == jc) bcast[0] = x;
    }
    ss = block_reduce1(ss, red);  // contains a barrier after bcast write
    const double alpha = bcast[0];
    const double sub = ss - alpha * alpha;
    double tau_c, beta, scale;
    if (!(sub > 0.0)) {  // nothing below the diagonal: H = I
      tau_c = 0.0;
      beta = alpha;
      scale = 0.0;
    } else {
      const double nrm = sqrt(ss);
      beta = (alpha >= 0.0) ? -nrm : nrm;
      tau_c = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // column cc becomes v (unit at jc, zero above within the panel rows)
    double vq[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      double x = 0.0;
#pragma unroll
      for (int t = 0; t < kNB; ++t)
        if (t == cc) x = a[q][t];
      double v;
      if (row[q] < jc || row[q] >= n) v = 0.0;
      else if (row[q] == jc) v = 1.0;
      else v = x * scale;
      vq[q] = v;
      if (row[q] >= jc) {
#pragma unroll
        for (int t = 0; t < kNB; ++t)
          if (t == cc) a[q][t] = v;
      }
    }
    // dots[t] = v^T col_t for all panel columns (previous v's and the trailing columns)
    double part[kNB];
#pragma unroll
    for (int t = 0; t < kNB; ++t) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < RPT; ++q) s += vq[q] * a[q][t];
      part[t] = s;
    }
    block_reduce_nb(part, red, dots);
    if (tid == 0) {
      betas[cc] = beta;
      taus[cc] = tau_c;
    }
    // T column: T[0:cc, cc] = -tau_c T[0:cc, 0:cc] (V^T v_cc)[0:cc],  T[cc][cc] = tau_c
    if (tid < cc) {
      double s = 0.0;
      for (int t = tid; t < cc; ++t) s += Ts[tid][t] * dots[t];
      Ts[tid][cc] = -tau_c * s;
    }
    if (tid == cc) Ts[cc][cc] = tau_c;
    // trailing columns: a[:, t] -= tau v dots[t], t > cc
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (row[q] >= jc && row[q] < n) {
#pragma unroll
        for (int t = 0; t < kNB; ++t)
          if (t > cc) a[q][t] -= tau_c * vq[q] * dots[t];
      }
    }
    __syncthreads();
  }
  // write back: R in A (upper part within the panel rows, zeros below), V explicit
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int r = row[q];
    if (r >= n) continue;
#pragma unroll
    for (int cc = 0; cc < kNB; ++cc) {
      if (cc >= nbp) continue;
      const int jc = j + cc;
      double rv, vv;
      if (r < jc) { rv = a[q][cc]; vv = 0.0; }
      else if (r == jc) { rv = betas[cc]; vv = 1.0; }
      else { rv = 0.0; vv = a[q][cc]; }
      A[(size_t)r * lda + jc] = rv;
      Vq[(size_t)r * lda + jc] = vv;
    }
  }
  for (int idx = tid; idx < kNB * kNB; idx += kPanelThreads) {
    const int r = idx / kNB, cc = idx % kNB;
    Tq[idx] = (r < nbp && cc < nbp) ? Ts[r][cc] : 0.0;
  }
  if (tid < nbp) tau_out[j + tid] = taus[tid];
}

__global__ void k_set_identity(double* __restrict__ Q, int n, int ld) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) {
    const int r = idx / n, cc = idx % n;
    Q[(size_t)r * ld + cc] = (r == cc) ? 1.0 : 0.0;
  }
}

__global__ void k_zero(double* __restrict__ X, size_t count) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) X[idx] = 0.0;
}

// A (n x n, leading dimension ld) = Q R; Q explicit in Q (ld).  Scratch from
// the context: Vq (explicit reflectors), Tq (per-panel T), Wq (2 nb x n).
int qr_f64(kdqmc_ctx* c, int n, double* A, double* Q) {
  const int ld = c->N;
  const int nb = kNB;
  if (n > 2 * kPanelThreads) return set_error(KDQMC_EUNSUPPORTED, "QR order above 2048");
  const size_t nn = (size_t)n * ld;
  hipLaunchKernelGGL(k_zero, dim3((nn + 255) / 256), dim3(256), 0, c->stream, c->Vq, nn);
  const int npan = (n + nb - 1) / nb;
  double* W1 = c->Wq;
  double* W2 = c->Wq + (size_t)nb * ld;
  for (int p = 0; p < npan; ++p) {
    const int j = p * nb;
    const int nbp = std::min(nb, n - j);
    double* Tp = c->Tq + (size_t)p * nb * nb;
    const int e0 = prof_mark(c);
    if (n - j > kPanelThreads)
      hipLaunchKernelGGL(k_qr_panel<2>, dim3(1), dim3(kPanelThreads), 0, c->stream, A, ld, n, j, nbp, c->Vq, Tp, c->tau);
    else
      hipLaunchKernelGGL(k_qr_panel<1>, dim3(1), dim3(kPanelThreads), 0, c->stream, A, ld, n, j, nbp, c->Vq, Tp, c->tau);
    prof_pair(c, PH_QR_PANEL, e0, prof_mark(c));
    const int nt = n - j - nbp;
    if (nt > 0) {
      // A[j:, j+nbp:] -= V T^T (V^T A[j:, j+nbp:])
      const double* V = c->Vq + (size_t)j * ld + j;
      double* At = A + (size_t)j * ld + j + nbp;
      KDQMC_TRY(gemm_f64(c, true, false, nbp, nt, n - j, 1.0, V, ld, At, ld, 0.0, W1, ld));
      KDQMC_TRY(gemm_f64(c, true, false, nbp, nt, nbp, 1.0, Tp, nb, W1, ld, 0.0, W2, ld));
      KDQMC_TRY(gemm_f64(c, false, false, n - j, nt, nbp, -1.0, V, ld, W2, ld, 1.0, At, ld));
    }
  }
  // Q = H_0 H_1 ... : backward accumulation, Q[j:, j:] = (I - V T V^T) Q[j:, j:]
  hipLaunchKernelGGL(k_set_identity, dim3((n * n + 255) / 256), dim3(256), 0, c->stream, Q, n, ld);
  for (int p = npan - 1; p >= 0; --p) {
    const int j = p * nb;
    const int nbp = std::min(nb, n - j);
    const double* Tp = c->Tq + (size_t)p * nb * nb;
    const double* V = c->Vq + (size_t)j * ld + j;
    double* Qs = Q + (size_t)j * ld + j;
    const int mm = n - j;
    KDQMC_TRY(gemm_f64(c, true, false, nbp, mm, mm, 1.0, V, ld, Qs, ld, 0.0, W1, ld));
    KDQMC_TRY(gemm_f64(c, false, false, nbp, mm, nbp, 1.0, Tp, nb, W1, ld, 0.0, W2, ld));
    KDQMC_TRY(gemm_f64(c, false, false, mm, mm, nbp, -1.0, V, ld, W2, ld, 1.0, Qs, ld));
  }
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

// ---------------------------------------------------------------------------
// Upper-triangular solve R Y = X in place on X (n x n, ld = N): inverse of
// each 32 x 32 diagonal block by back substitution in LDS, then blocked
// backward substitution with GEMMs.
// ---------------------------------------------------------------------------
__global__ void k_trinv_blocks(const double* __restrict__ R, int n, int ld, double* __restrict__ Rinv) {
  __shared__ double Rb[kNB][kNB + 1];
  const int b = blockIdx.x;
  const int b0 = b * kNB;
  const int nbp = min(kNB, n - b0);
  for (int idx = threadIdx.x; idx < kNB * kNB; idx += blockDim.x) {
    const int r = idx / kNB, cc = idx % kNB;
    Rb[r][cc] = (r < nbp && cc < nbp) ? R[(size_t)(b0 + r) * ld + b0 + cc] : 0.0;
  }
  __syncthreads();
  const int col = threadIdx.x;  // column of the inverse
  if (col < kNB) {
    double x[kNB];
#pragma unroll
    for (int r = kNB - 1; r >= 0; --r) {
      double s = (r == col) ? 1.0 : 0.0;
#pragma unroll
      for (int t = r + 1; t < kNB; ++t) s -= Rb[r][t] * x[t];
      x[r] = (r < nbp) ? s / Rb[r][r] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < kNB; ++r) Rinv[(size_t)b * kNB * kNB + r * kNB + col] = x[r];
  }
}

int trsm_upper_f64(kdqmc_ctx* c, int n, const double* R, double* X) {
  const int ld = c->N, nb = kNB;
  const int nblk = (n + nb - 1) / nb;
  double* Rinv = c->Tq;  // nblk * nb * nb
  hipLaunchKernelGGL(k_trinv_blocks, dim3(nblk), dim3(64), 0, c->stream, R, n, ld, Rinv);
  double* Y = c->S[7];
  for (int b = nblk - 1; b >= 0; --b) {
    const int b0 = b * nb;
    const int nbp = std::min(nb, n - b0);
    const int b1 = b0 + nbp;
    if (b1 < n)
      KDQMC_TRY(gemm_f64(c, false, false, nbp, n, n - b1, -1.0, R + (size_t)b0 * ld + b1, ld,
                         Y + (size_t)b1 * ld, ld, 1.0, X + (size_t)b0 * ld, ld));
    KDQMC_TRY(gemm_f64(c, false, false, nbp, n, nbp, 1.0, Rinv + (size_t)b * nb * nb, nb,
                       X + (size_t)b0 * ld, ld, 0.0, Y + (size_t)b0 * ld, ld));
  }
  KDQMC_TRY(copy_f64(c, X, Y, (size_t)n * ld));
  return KDQMC_OK;
}

}  // namespace kdqmc
