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

__global__ void k_ev_slice(const int8_t* __restrict__ s, int n, const double* __restrict__ sc,
                           double* __restrict__ ev, size_t zs) {
  s = zw(s, zs);
  ev = zw(ev, zs);
  const double ea = zw(sc, zs)[SC_EA], eainv = zw(sc, zs)[SC_EAINV];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ev[i] = s[i] > 0 ? ea : eainv;
}

__global__ void k_identity_udt(double* __restrict__ U, double* __restrict__ D, double* __restrict__ T, int n,
                               size_t zs) {
  U = zw(U, zs);
  D = zw(D, zs);
  T = zw(T, zs);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) {
    const int r = idx / n, c = idx % n;
    U[idx] = (r == c) ? 1.0 : 0.0;
    T[idx] = (r == c) ? 1.0 : 0.0;
    if (r == 0) D[c] = 1.0;
  }
}

__global__ void k_scale_cols(double* __restrict__ C, int n, const double* __restrict__ d, size_t zs) {
  C = zw(C, zs);
  d = zw(d, zs);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) C[idx] *= d[idx % n];
}

// squared column norms: a workgroup owns 64 columns, its 4 waves split the
// rows (lanes over columns: coalesced), partial sums combined in LDS
__global__ void __launch_bounds__(256) k_colnorm2(const double* __restrict__ C, int n, double* __restrict__ nrm,
                                                  size_t zs) {
  __shared__ double part[4][64];
  C = zw(C, zs);
  nrm = zw(nrm, zs);
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

// perm[rank] = column, descending norm, ties by column index (stable); n <= 2048.
// Each workgroup ranks 256 columns against all n norms staged in LDS (every
// lane reads the same LDS word at a time: broadcast).  A norm that is not
// finite ranks as -inf (so the ranks stay a permutation: every comparison is
// of ordered values) and marks the chain's health record.
__global__ void __launch_bounds__(256) k_rank_perm(const double* __restrict__ nrm, int n, int* __restrict__ perm,
                                                   double* __restrict__ health, size_t zs) {
  __shared__ double sn[2048];
  nrm = zw(nrm, zs);
  perm = zw(perm, zs);
  health = zw(health, zs);
  for (int q = threadIdx.x; q < n; q += 256) {
    const double x = nrm[q];
    const bool fin = __builtin_isfinite(x);
    if (!fin) health[HL_NONFINITE] = 1.0;
    sn[q] = fin ? x : -__builtin_inf();
  }
  __syncthreads();
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  const double v = sn[c];
  int rank = 0;
  for (int q = 0; q < n; ++q) {
    const double w = sn[q];
    rank += (w > v) || (w == v && q < c);
  }
  perm[rank] = c;
}

// out[r] = a[b[r]]: the composition of two orders
__global__ void k_compose_perm(int* __restrict__ out, const int* __restrict__ a, const int* __restrict__ b, int n,
                               size_t zs) {
  out = zw(out, zs);
  a = zw(a, zs);
  b = zw(b, zs);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[r] = a[b[r]];
}

__global__ void k_gather_cols(double* __restrict__ dst, const double* __restrict__ src, int n,
                              const int* __restrict__ perm, size_t zs) {
  dst = zw(dst, zs);
  src = zw(src, zs);
  perm = zw(perm, zs);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) {
    const int r = idx / n, c = idx % n;
    dst[idx] = src[(size_t)r * n + perm[c]];
  }
}

__global__ void k_gather_rows(double* __restrict__ dst, const double* __restrict__ src, int n,
                              const int* __restrict__ perm, size_t zs) {
  dst = zw(dst, zs);
  src = zw(src, zs);
  perm = zw(perm, zs);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) {
    const int r = idx / n, c = idx % n;
    dst[idx] = src[(size_t)perm[r] * n + c];
  }
}

// R <- D^{-1} R (rows), D = |diag R| computed beforehand by k_diag_abs
__global__ void k_diag_normalize(double* __restrict__ R, int n, const double* __restrict__ D, size_t zs) {
  R = zw(R, zs);
  D = zw(D, zs);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) R[idx] /= D[idx / n];
}

__global__ void k_diag_abs(const double* __restrict__ R, int n, double* __restrict__ D, size_t zs) {
  R = zw(R, zs);
  D = zw(D, zs);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) D[r] = fabs(R[(size_t)r * n + r]);
}

// M = Db_R^{-1} X1 Db_L^{-1} + Ds_R X2 Ds_L (in place in X1)
__global__ void k_combine_M(double* __restrict__ X1, const double* __restrict__ X2, int n,
                            const double* __restrict__ DR, const double* __restrict__ DL, size_t zs) {
  X1 = zw(X1, zs);
  X2 = zw(X2, zs);
  DR = zw(DR, zs);
  DL = zw(DL, zs);
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
                                  const double* __restrict__ D, size_t zs) {
  dst = zw(dst, zs);
  src = zw(src, zs);
  D = zw(D, zs);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) {
    const int r = idx / n, c = idx % n;
    dst[idx] = src[(size_t)c * n + r] / fmax(D[r], 1.0);
  }
}

// X <- Db^{-1} X (rows)
__global__ void k_scale_rows_big(double* __restrict__ X, int n, const double* __restrict__ D, size_t zs) {
  X = zw(X, zs);
  D = zw(D, zs);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) X[idx] /= fmax(D[idx / n], 1.0);
}

template <typename T>
__global__ void k_maxabs_partial(const T* __restrict__ G, const double* __restrict__ F, size_t count,
                                 double* __restrict__ part, size_t zs) {
  __shared__ double red[16];
  G = zw(G, zs);
  F = zw(F, zs);
  part = zw(part, zs);
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

// out[0] = max of n partial maxima (one wave; NaN propagates); out is a
// caller array with records zo bytes apart, or null.  The chain's health
// record takes the value as its latest wrap error, raises its largest, and
// counts a violation when the value is not finite or above tol.
__global__ void k_max_final(const double* __restrict__ part, int n, double* __restrict__ out,
                            double* __restrict__ health, double tol, size_t zs, size_t zo) {
  part = zw(part, zs);
  out = zw(out, zo);
  health = zw(health, zs);
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) m = (part[i] > m || part[i] != part[i]) ? part[i] : m;
  for (int o = 32; o >= 1; o >>= 1) {
    const double x = __shfl_xor(m, o);
    m = (x > m || x != x) ? x : m;
  }
  if (threadIdx.x == 0) {
    if (out) out[0] = m;
    double w = health[HL_WORST];
    if (w == w) w = (m > w || m != m) ? m : w;  // once NaN, it stays NaN
    health[HL_WORST] = w;
    if (!(m <= tol)) health[HL_NVIOL] += 1.0;
    health[HL_LAST] = m;
  }
}

__global__ void k_zero_f64(double* __restrict__ x, int n, size_t zs) {
  x = zw(x, zs);
  if ((int)threadIdx.x < n) x[threadIdx.x] = 0.0;
}

int clear_health(kdqmc_ctx* c) {
  hipLaunchKernelGGL(k_zero_f64, dim3(1, 1, c->nch), dim3(64), 0, c->stream, c->health, (int)HL_COUNT, c->zs);
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

// dst and src records are zd and zsrc bytes apart between chains
template <typename TO, typename TI>
__global__ void k_convert(TO* __restrict__ dst, const TI* __restrict__ src, size_t count, size_t zd,
                          size_t zsrc) {
  dst = zw(dst, zd);
  src = zw(src, zsrc);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) dst[idx] = TO(src[idx]);
}

__global__ void k_copy_f64(double* __restrict__ dst, const double* __restrict__ src, size_t n, size_t zs) {
  dst = zw(dst, zs);
  src = zw(src, zs);
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

int copy_f64(kdqmc_ctx* c, double* dst, const double* src, size_t n) {
  hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)((n + 255) / 256), 1, c->nch), dim3(256), 0, c->stream, dst,
                     src, n, c->zs);
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

namespace {

// Steps of a stack, counted from its identity end, whose QR re-pivots.
constexpr int kRepivotSteps = 3;

inline dim3 grid_for(kdqmc_ctx* c, size_t count) {
  return dim3((unsigned)((count + 255) / 256), 1, (unsigned)c->nch);
}

double* stackU(kdqmc_ctx* c, bool left, int j) { return (left ? c->LU : c->RU) + (size_t)j * c->N * c->N; }
double* stackT(kdqmc_ctx* c, bool left, int j) { return (left ? c->LT : c->RT) + (size_t)j * c->N * c->N; }
double* stackD(kdqmc_ctx* c, bool left, int j) { return (left ? c->LD : c->RD) + (size_t)j * c->N; }

// One UDT step.  slices: the B's to apply in order (first applied first);
// transposed: apply B^T = exp(V) exp(-dtau (K - mu)) instead of B.
// The columns are ordered by norm before an unpivoted QR.  repivot: the QR is
// then taken a second time with the columns ordered by the first one's
// |R_ii| (the norms left after orthogonalization against the earlier
// columns), which is what column pivoting ranks by.  Ordering by the initial
// norm fails where many columns have similar norms but are close to
// dependent: the first steps from the identity end of a stack, before the
// scales have spread (|R_ij| / |R_ii| reaches about 70 there), where it
// costs a factor of 100 in the accuracy of G between two long stacks.
int udt_step(kdqmc_ctx* c, const double* Uin, const double* Din, const double* Tin,
             const int* slices, int nsl, bool transposed, double* Uout, double* Dout, double* Tout,
             bool repivot) {
  const int n = c->N;
  const size_t nn = (size_t)n * n;
  double* C = c->S[0];
  double* Cp = c->S[1];
  double* Tp = c->S[3];
  double* evs = c->nrm + n;  // second half of the norm buffer holds the slice scale
  KDQMC_TRY(copy_f64(c, C, Uin, nn));
  const size_t zs = c->zs;
  for (int q = 0; q < nsl; ++q) {
    const int l = slices[q];
    hipLaunchKernelGGL(k_ev_slice, grid_for(c, n), dim3(256), 0, c->stream,
                       c->fields + (size_t)(l - 1) * n, n, c->sc, evs, zs);
    if (transposed)
      KDQMC_TRY(launch_kinetic_f64(c, C, n, true, c->tab_mu64, nullptr, nullptr, evs));
    else
      KDQMC_TRY(launch_kinetic_f64(c, C, n, true, c->tab_mu64, evs, nullptr, nullptr));
  }
  hipLaunchKernelGGL(k_scale_cols, grid_for(c, nn), dim3(256), 0, c->stream, C, n, Din, zs);
  hipLaunchKernelGGL(k_colnorm2, dim3((n + 63) / 64, 1, c->nch), dim3(256), 0, c->stream, C, n, c->nrm, zs);
  hipLaunchKernelGGL(k_rank_perm, dim3((n + 255) / 256, 1, c->nch), dim3(256), 0, c->stream, c->nrm, n, c->perm,
                     c->health, zs);
  hipLaunchKernelGGL(k_gather_cols, grid_for(c, nn), dim3(256), 0, c->stream, Cp, C, n, c->perm, zs);
  const int* order = c->perm;
  if (repivot) {
    int* rank2 = c->perm + n;
    int* order2 = c->perm + 2 * n;
    KDQMC_TRY(qr_f64(c, n, n, Cp, nullptr));
    hipLaunchKernelGGL(k_diag_abs, grid_for(c, n), dim3(256), 0, c->stream, Cp, n, c->nrm, zs);
    hipLaunchKernelGGL(k_rank_perm, dim3((n + 255) / 256, 1, c->nch), dim3(256), 0, c->stream, c->nrm, n, rank2,
                       c->health, zs);
    hipLaunchKernelGGL(k_compose_perm, grid_for(c, n), dim3(256), 0, c->stream, order2, c->perm, rank2, n, zs);
    hipLaunchKernelGGL(k_gather_cols, grid_for(c, nn), dim3(256), 0, c->stream, Cp, C, n, order2, zs);
    order = order2;
  }
  KDQMC_TRY(qr_f64(c, n, n, Cp, Uout));
  hipLaunchKernelGGL(k_diag_abs, grid_for(c, n), dim3(256), 0, c->stream, Cp, n, Dout, zs);
  hipLaunchKernelGGL(k_diag_normalize, grid_for(c, nn), dim3(256), 0, c->stream, Cp, n, Dout, zs);
  hipLaunchKernelGGL(k_gather_rows, grid_for(c, nn), dim3(256), 0, c->stream, Tp, Tin, n, order, zs);
  KDQMC_TRY(gemm_f64(c, false, false, n, n, n, 1.0, Cp, n, Tp, n, 0.0, Tout, n));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

// Projector form: one step of a stack of orthonormal panels.  The N x n_occ
// panel Uin (row stride N) is multiplied by the slices' B (or B^T) and
// replaced by the Q factor of its Householder QR: only its span enters G.
int pq_step(kdqmc_ctx* c, const double* Uin, const int* slices, int nsl, bool transposed, double* Uout) {
  const int n = c->N, m = c->nocc;
  double* C = c->S[0];
  double* evs = c->nrm + n;
  KDQMC_TRY(copy_f64(c, C, Uin, (size_t)n * n));
  for (int q = 0; q < nsl; ++q) {
    const int l = slices[q];
    hipLaunchKernelGGL(k_ev_slice, grid_for(c, n), dim3(256), 0, c->stream,
                       c->fields + (size_t)(l - 1) * n, n, c->sc, evs, c->zs);
    if (transposed)
      KDQMC_TRY(launch_kinetic_f64(c, C, n, true, c->tab_mu64, nullptr, nullptr, evs, m));
    else
      KDQMC_TRY(launch_kinetic_f64(c, C, n, true, c->tab_mu64, evs, nullptr, nullptr, m));
  }
  KDQMC_TRY(qr_f64(c, n, m, C, Uout));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

// dst[r][c] = src[c][r] for r < m, c < n (an m x n block from an n x m one; row stride n)
__global__ void k_transpose_panel(double* __restrict__ dst, const double* __restrict__ src, int n, int m,
                                  size_t zs) {
  dst = zw(dst, zs);
  src = zw(src, zs);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)m * n) {
    const int r = idx / n, cc = idx % n;
    dst[(size_t)r * n + cc] = src[(size_t)cc * n + r];
  }
}

__global__ void k_eye(double* __restrict__ X, int n, size_t zs) {
  X = zw(X, zs);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) X[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
}

// Projector G at checkpoint j: I - R (L^T R)^{-1} L^T with the right panel R
// and the left panel L (both N x n_occ, orthonormal): X = L^T R (n_occ^2),
// its QR, Y = L^T (n_occ x N), Y <- Q^T Y, R_X Y' = Y, out = I - R Y'.
int pq_green(kdqmc_ctx* c, int j, double* out) {
  const int n = c->N, m = c->nocc;
  const double* R = stackU(c, false, j);
  const double* Lp = stackU(c, true, j);
  double* X = c->S[0];
  double* Y = c->S[4];
  KDQMC_TRY(gemm_f64(c, true, false, m, m, n, 1.0, Lp, n, R, n, 0.0, X, n));
  KDQMC_TRY(qr_f64(c, m, m, X, nullptr));
  hipLaunchKernelGGL(k_transpose_panel, grid_for(c, (size_t)m * n), dim3(256), 0, c->stream, Y, Lp, n, m, c->zs);
  KDQMC_TRY(apply_qt_f64(c, m, n, Y));
  KDQMC_TRY(trsm_upper_f64(c, m, n, X, Y));
  hipLaunchKernelGGL(k_eye, grid_for(c, (size_t)n * n), dim3(256), 0, c->stream, out, n, c->zs);
  KDQMC_TRY(gemm_f64(c, false, false, n, n, m, -1.0, R, n, Y, n, 1.0, out, n));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

}  // namespace

int stab_identity(kdqmc_ctx* c, bool left, int j) {
  const size_t nn = (size_t)c->N * c->N;
  if (c->proj) return copy_f64(c, stackU(c, left, j), c->Ptrial, nn);  // the trial panel
  hipLaunchKernelGGL(k_identity_udt, grid_for(c, nn), dim3(256), 0, c->stream, stackU(c, left, j),
                     stackD(c, left, j), stackT(c, left, j), c->N, c->zs);
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

int stab_left_step(kdqmc_ctx* c, int j) {
  // L_j^T-chain: B_{c_j+1}^T ... B_{c_{j+1}}^T applied to L_{j+1}: rightmost first
  int sl[1024];
  const int lo = j * c->p.n_stab + 1, hi = (j + 1) * c->p.n_stab;
  int ns = 0;
  for (int l = hi; l >= lo; --l) sl[ns++] = l;
  if (c->proj) return pq_step(c, stackU(c, true, j + 1), sl, ns, true, stackU(c, true, j));
  // the entries nearest the identity end (the first three steps of the stack) re-pivot
  return udt_step(c, stackU(c, true, j + 1), stackD(c, true, j + 1), stackT(c, true, j + 1), sl, ns, true,
                  stackU(c, true, j), stackD(c, true, j), stackT(c, true, j), j >= c->nc - kRepivotSteps);
}

int stab_build_left(kdqmc_ctx* c) {
  KDQMC_TRY(stab_identity(c, true, c->nc));
  for (int j = c->nc - 1; j >= 0; --j) KDQMC_TRY(stab_left_step(c, j));
  return KDQMC_OK;
}

int stab_build_right(kdqmc_ctx* c) {
  KDQMC_TRY(stab_identity(c, false, 0));
  for (int j = 1; j <= c->nc; ++j) KDQMC_TRY(stab_right_step(c, j));
  return KDQMC_OK;
}

int stab_right_step(kdqmc_ctx* c, int j) {
  int sl[1024];
  const int lo = (j - 1) * c->p.n_stab + 1, hi = j * c->p.n_stab;
  int ns = 0;
  for (int l = lo; l <= hi; ++l) sl[ns++] = l;
  if (c->proj) return pq_step(c, stackU(c, false, j - 1), sl, ns, false, stackU(c, false, j));
  return udt_step(c, stackU(c, false, j - 1), stackD(c, false, j - 1), stackT(c, false, j - 1), sl,
                  ns, false, stackU(c, false, j), stackD(c, false, j), stackT(c, false, j), j <= kRepivotSteps);
}

int stab_green(kdqmc_ctx* c, int j, double* out) {
  if (c->proj) return pq_green(c, j, out);
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
  hipLaunchKernelGGL(k_combine_M, grid_for(c, nn), dim3(256), 0, c->stream, X1, X2, n, DR, DL, c->zs);
  KDQMC_TRY(qr_f64(c, n, n, X1, nullptr));
  hipLaunchKernelGGL(k_transpose_scale, grid_for(c, nn), dim3(256), 0, c->stream, Y, UR, n, DR, c->zs);
  KDQMC_TRY(apply_qt_f64(c, n, n, Y));
  KDQMC_TRY(trsm_upper_f64(c, n, n, X1, Y));
  hipLaunchKernelGGL(k_scale_rows_big, grid_for(c, nn), dim3(256), 0, c->stream, Y, n, DL, c->zs);
  KDQMC_TRY(gemm_f64(c, false, false, n, n, n, 1.0, UL, n, Y, n, 0.0, out, n));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

int copy_G_to64(kdqmc_ctx* c, double* out, size_t zn) {
  const size_t nn = (size_t)c->N * c->N;
  const size_t zd = zn ? zn * sizeof(double) : c->zs;
  if (c->fp64)
    hipLaunchKernelGGL((k_convert<double, double>), grid_for(c, nn), dim3(256), 0, c->stream, out,
                       (const double*)c->G, nn, zd, c->zs);
  else
    hipLaunchKernelGGL((k_convert<double, float>), grid_for(c, nn), dim3(256), 0, c->stream, out,
                       (const float*)c->G, nn, zd, c->zs);
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

int copy_64_to_G(kdqmc_ctx* c, const double* in, size_t zn) {
  const size_t nn = (size_t)c->N * c->N;
  const size_t zsrc = zn ? zn * sizeof(double) : c->zs;
  if (c->fp64) {
    if (in != c->G)
      hipLaunchKernelGGL((k_convert<double, double>), grid_for(c, nn), dim3(256), 0, c->stream,
                         (double*)c->G, in, nn, c->zs, zsrc);
  } else {
    hipLaunchKernelGGL((k_convert<float, double>), grid_for(c, nn), dim3(256), 0, c->stream,
                       (float*)c->G, in, nn, c->zs, zsrc);
  }
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

int max_abs_diff(kdqmc_ctx* c, const double* a, int /*n*/, double* out, size_t zn) {
  const size_t nn = (size_t)c->N * c->N;
  const int nblk = 256;
  if (c->fp64)
    hipLaunchKernelGGL((k_maxabs_partial<double>), dim3(nblk, 1, c->nch), dim3(256), 0, c->stream,
                       (const double*)c->G, a, nn, c->err, c->zs);
  else
    hipLaunchKernelGGL((k_maxabs_partial<float>), dim3(nblk, 1, c->nch), dim3(256), 0, c->stream,
                       (const float*)c->G, a, nn, c->err, c->zs);
  hipLaunchKernelGGL(k_max_final, dim3(1, 1, c->nch), dim3(64), 0, c->stream, c->err, nblk, out, c->health,
                     c->wrap_tol, c->zs, zn * sizeof(double));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

}  // namespace kdqmc
