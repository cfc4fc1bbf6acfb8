// QR-stabilized B-chains (UDT form) and the stable equal-time Green's
// function, FP64 on the GPU.
//
// Checkpoints c_j = j * n_stab, j = 0..nc (c_nc = L_tau).
//   right stack R_j: U D T of B_{c_j} ... B_1                  (R_0 = I)
//   left stack  L_j: U D T of (B_{L_tau} ... B_{c_j + 1})^T      (L_nc = I)
// One UDT step multiplies the stored U by the slices' B (or B^T) through the
// FFT kinetic kernel, scales the columns by D, sorts the columns by norm
// (pre-pivoting), and takes a Householder QR: C P = Q R, U' = Q,
// D' = |diag R|, T' = D'^{-1} R P^T T.
// G(c_j) = [I + U_R D_R T_R T_L^T D_L U_L^T]^{-1}
//        = U_L Db_L^{-1} M^{-1} Db_R^{-1} U_R^T,
// M = Db_R^{-1} (U_R^T U_L) Db_L^{-1} + Ds_R (T_R T_L^T) Ds_L,
// with Db = max(D, 1), Ds = min(D, 1) (Loh-Gubernatis scale separation).
#include <algorithm>
#include <cmath>

#include "common.h"

namespace kdqmc {

__global__ void k_ev_slice(const int8_t* __restrict__ s, int n, double ea, double eainv,
                           double* __restrict__ ev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ev[i] = s[i] > 0 ? ea : eainv;
}

__global__ void k_identity_udt(double* __restrict__ U, double* __restrict__ D, double* __restrict__ T, int n) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) {
    const int r = idx / n, c = idx % n;
    U[idx] = (r == c) ? 1.0 : 0.0;
    T[idx] = (r == c) ? 1.0 : 0.0;
    if (r == 0) D[c] = 1.0;
  }
}

__global__ void k_scale_cols(double* __restrict__ C, int n, const double* __restrict__ d) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) C[idx] *= d[idx % n];
}

// squared column norms: a workgroup owns 64 columns, its 4 waves split the
// rows (lanes over columns: coalesced), partial sums combined in LDS
__global__ void __launch_bounds__(256) k_colnorm2(const double* __restrict__ C, int n, double* __restrict__ nrm) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (c < n) {
#pragma unroll 4
    for (int r = wave; r < n; r += 4) {
      const double x = C[(size_t)r * n + c];
      s += x * x;
    }
  }
  part[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && c < n) nrm[c] = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
}

// perm[rank] = column, descending norm, ties by column index (stable); n <= 2048
__global__ void k_rank_perm(const double* __restrict__ nrm, int n, int* __restrict__ perm) {
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const double v = nrm[c];
    int rank = 0;
    for (int q = 0; q < n; ++q) {
      const double w = nrm[q];
      rank += (w > v) || (w == v && q < c);
    }
    perm[rank] = c;
  }
}

__global__ void k_gather_cols(double* __restrict__ dst, const double* __restrict__ src, int n,
                              const int* __restrict__ perm) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) {
    const int r = idx / n, c = idx % n;
    dst[idx] = src[(size_t)r * n + perm[c]];
  }
}

__global__ void k_gather_rows(double* __restrict__ dst, const double* __restrict__ src, int n,
                              const int* __restrict__ perm) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) {
    const int r = idx / n, c = idx % n;
    dst[idx] = src[(size_t)perm[r] * n + c];
  }
}

// R <- D^{-1} R (rows), D = |diag R| computed beforehand by k_diag_abs
__global__ void k_diag_normalize(double* __restrict__ R, int n, const double* __restrict__ D) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) R[idx] /= D[idx / n];
}

__global__ void k_diag_abs(const double* __restrict__ R, int n, double* __restrict__ D) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) D[r] = fabs(R[(size_t)r * n + r]);
}

// M = Db_R^{-1} X1 Db_L^{-1} + Ds_R X2 Ds_L (in place in X1)
__global__ void k_combine_M(double* __restrict__ X1, const double* __restrict__ X2, int n,
                            const double* __restrict__ DR, const double* __restrict__ DL) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) {
    const int r = idx / n, c = idx % n;
    const double dr = DR[r], dl = DL[c];
    const double br = fmax(dr, 1.0), sr = fmin(dr, 1.0);
    const double bl = fmax(dl, 1.0), sl = fmin(dl, 1.0);
    X1[idx] = X1[idx] / (br * bl) + sr * X2[idx] * sl;
  }
}

// dst = Db^{-1} src^T
__global__ void k_transpose_scale(double* __restrict__ dst, const double* __restrict__ src, int n,
                                  const double* __restrict__ D) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) {
    const int r = idx / n, c = idx % n;
    dst[idx] = src[(size_t)c * n + r] / fmax(D[r], 1.0);
  }
}

// X <- Db^{-1} X (rows)
__global__ void k_scale_rows_big(double* __restrict__ X, int n, const double* __restrict__ D) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) X[idx] /= fmax(D[idx / n], 1.0);
}

template <typename T>
__global__ void k_maxabs_partial(const T* __restrict__ G, const double* __restrict__ F, size_t count,
                                 double* __restrict__ part) {
  __shared__ double red[16];
  double m = 0.0;
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count;
       idx += (size_t)gridDim.x * blockDim.x) {
    const double d = fabs(double(G[idx]) - F[idx]);
    m = (d > m || d != d) ? d : m;  // propagates NaN
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const double x = __shfl_xor(m, o);
    m = (x > m || x != x) ? x : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = (red[w] > r || red[w] != red[w]) ? red[w] : r;
    part[blockIdx.x] = r;
  }
}

__global__ void k_max_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int i = 0; i < n; ++i) r = (part[i] > r || part[i] != part[i]) ? part[i] : r;
    out[0] = r;
  }
}

template <typename TO, typename TI>
__global__ void k_convert(TO* __restrict__ dst, const TI* __restrict__ src, size_t count) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) dst[idx] = TO(src[idx]);
}

__global__ void k_copy_f64(double* __restrict__ dst, const double* __restrict__ src, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

int copy_f64(kdqmc_ctx* c, double* dst, const double* src, size_t n) {
  hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, dst, src, n);
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

namespace {

inline dim3 grid_for(size_t count) { return dim3((unsigned)((count + 255) / 256)); }

double* stackU(kdqmc_ctx* c, bool left, int j) { return (left ? c->LU : c->RU) + (size_t)j * c->N * c->N; }
double* stackT(kdqmc_ctx* c, bool left, int j) { return (left ? c->LT : c->RT) + (size_t)j * c->N * c->N; }
double* stackD(kdqmc_ctx* c, bool left, int j) { return (left ? c->LD : c->RD) + (size_t)j * c->N; }

// One UDT step.  slices: the B's to apply in order (first applied first);
// transposed: apply B^T = exp(V) exp(-dtau (K - mu)) instead of B.
int udt_step(kdqmc_ctx* c, const double* Uin, const double* Din, const double* Tin,
             const int* slices, int nsl, bool transposed, double* Uout, double* Dout, double* Tout) {
  const int n = c->N;
  const size_t nn = (size_t)n * n;
  double* C = c->S[0];
  double* Cp = c->S[1];
  double* Tp = c->S[3];
  double* evs = c->nrm + n;  // second half of the norm buffer holds the slice scale
  KDQMC_TRY(copy_f64(c, C, Uin, nn));
  const double ea = std::exp(c->alpha), eainv = std::exp(-c->alpha);
  for (int q = 0; q < nsl; ++q) {
    const int l = slices[q];
    hipLaunchKernelGGL(k_ev_slice, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                       c->fields + (size_t)(l - 1) * n, n, ea, eainv, evs);
    if (transposed)
      KDQMC_TRY(launch_kinetic_f64(c, C, n, true, c->tab_mu64, nullptr, nullptr, evs));
    else
      KDQMC_TRY(launch_kinetic_f64(c, C, n, true, c->tab_mu64, evs, nullptr, nullptr));
  }
  hipLaunchKernelGGL(k_scale_cols, grid_for(nn), dim3(256), 0, c->stream, C, n, Din);
  hipLaunchKernelGGL(k_colnorm2, dim3((n + 63) / 64), dim3(256), 0, c->stream, C, n, c->nrm);
  hipLaunchKernelGGL(k_rank_perm, dim3(1), dim3(1024), 0, c->stream, c->nrm, n, c->perm);
  hipLaunchKernelGGL(k_gather_cols, grid_for(nn), dim3(256), 0, c->stream, Cp, C, n, c->perm);
  KDQMC_TRY(qr_f64(c, n, Cp, Uout));
  hipLaunchKernelGGL(k_diag_abs, dim3((n + 255) / 256), dim3(256), 0, c->stream, Cp, n, Dout);
  hipLaunchKernelGGL(k_diag_normalize, grid_for(nn), dim3(256), 0, c->stream, Cp, n, Dout);
  hipLaunchKernelGGL(k_gather_rows, grid_for(nn), dim3(256), 0, c->stream, Tp, Tin, n, c->perm);
  KDQMC_TRY(gemm_f64(c, false, false, n, n, n, 1.0, Cp, n, Tp, n, 0.0, Tout, n));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

}  // namespace

int stab_identity(kdqmc_ctx* c, bool left, int j) {
  const size_t nn = (size_t)c->N * c->N;
  hipLaunchKernelGGL(k_identity_udt, grid_for(nn), dim3(256), 0, c->stream, stackU(c, left, j),
                     stackD(c, left, j), stackT(c, left, j), c->N);
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

int stab_build_left(kdqmc_ctx* c) {
  KDQMC_TRY(stab_identity(c, true, c->nc));
  int sl[1024];
  for (int j = c->nc - 1; j >= 0; --j) {
    // L_j^T-chain: B_{c_j+1}^T ... B_{c_{j+1}}^T applied to L_{j+1}: rightmost first
    const int lo = j * c->p.n_stab + 1, hi = (j + 1) * c->p.n_stab;
    int ns = 0;
    for (int l = hi; l >= lo; --l) sl[ns++] = l;
    KDQMC_TRY(udt_step(c, stackU(c, true, j + 1), stackD(c, true, j + 1), stackT(c, true, j + 1), sl,
                       ns, true, stackU(c, true, j), stackD(c, true, j), stackT(c, true, j)));
  }
  return KDQMC_OK;
}

int stab_right_step(kdqmc_ctx* c, int j) {
  int sl[1024];
  const int lo = (j - 1) * c->p.n_stab + 1, hi = j * c->p.n_stab;
  int ns = 0;
  for (int l = lo; l <= hi; ++l) sl[ns++] = l;
  return udt_step(c, stackU(c, false, j - 1), stackD(c, false, j - 1), stackT(c, false, j - 1), sl,
                  ns, false, stackU(c, false, j), stackD(c, false, j), stackT(c, false, j));
}

int stab_green(kdqmc_ctx* c, int j, double* out) {
  const int n = c->N;
  const size_t nn = (size_t)n * n;
  const double* UR = stackU(c, false, j);
  const double* DR = stackD(c, false, j);
  const double* TR = stackT(c, false, j);
  const double* UL = stackU(c, true, j);
  const double* DL = stackD(c, true, j);
  const double* TL = stackT(c, true, j);
  double* X1 = c->S[0];
  double* X2 = c->S[1];
  double* Y = c->S[4];
  KDQMC_TRY(gemm_f64(c, true, false, n, n, n, 1.0, UR, n, UL, n, 0.0, X1, n));
  KDQMC_TRY(gemm_f64(c, false, true, n, n, n, 1.0, TR, n, TL, n, 0.0, X2, n));
  hipLaunchKernelGGL(k_combine_M, grid_for(nn), dim3(256), 0, c->stream, X1, X2, n, DR, DL);
  KDQMC_TRY(qr_f64(c, n, X1, nullptr));
  hipLaunchKernelGGL(k_transpose_scale, grid_for(nn), dim3(256), 0, c->stream, Y, UR, n, DR);
  KDQMC_TRY(apply_qt_f64(c, n, Y));
  KDQMC_TRY(trsm_upper_f64(c, n, X1, Y));
  hipLaunchKernelGGL(k_scale_rows_big, grid_for(nn), dim3(256), 0, c->stream, Y, n, DL);
  KDQMC_TRY(gemm_f64(c, false, false, n, n, n, 1.0, UL, n, Y, n, 0.0, out, n));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

int copy_G_to64(kdqmc_ctx* c, double* out) {
  const size_t nn = (size_t)c->N * c->N;
  if (c->fp64) {
    KDQMC_TRY(copy_f64(c, out, (const double*)c->G, nn));
  } else {
    hipLaunchKernelGGL((k_convert<double, float>), grid_for(nn), dim3(256), 0, c->stream, out,
                       (const float*)c->G, nn);
    KDQMC_HIP(hipGetLastError());
  }
  return KDQMC_OK;
}

int copy_64_to_G(kdqmc_ctx* c, const double* in) {
  const size_t nn = (size_t)c->N * c->N;
  if (c->fp64) {
    if (in != c->G)
      KDQMC_TRY(copy_f64(c, (double*)c->G, in, nn));
  } else {
    hipLaunchKernelGGL((k_convert<float, double>), grid_for(nn), dim3(256), 0, c->stream,
                       (float*)c->G, in, nn);
    KDQMC_HIP(hipGetLastError());
  }
  return KDQMC_OK;
}

int max_abs_diff(kdqmc_ctx* c, const double* a, int /*n*/, double* out) {
  const size_t nn = (size_t)c->N * c->N;
  const int nblk = 256;
  if (c->fp64)
    hipLaunchKernelGGL((k_maxabs_partial<double>), dim3(nblk), dim3(256), 0, c->stream,
                       (const double*)c->G, a, nn, c->err);
  else
    hipLaunchKernelGGL((k_maxabs_partial<float>), dim3(nblk), dim3(256), 0, c->stream,
                       (const float*)c->G, a, nn, c->err);
  hipLaunchKernelGGL(k_max_final, dim3(1), dim3(64), 0, c->stream, c->err, nblk, out);
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

}  // namespace kdqmc
