// FP64 dense linear algebra used by the stabilization of the B-chains:
// an MFMA GEMM, a blocked Householder QR (compact WY form, panel factored in
// registers by one workgroup), a blocked upper-triangular solve and small
// elementwise helpers.  All on the context's stream.
#include <algorithm>

#include "common.h"

namespace kdqmc {

typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// GEMM: C = alpha op(A) op(B) + beta C, row-major, TS x TS tile per
// workgroup of 4 waves (each a TS/2 x TS/2 quarter, v_mfma_f64_16x16x4),
// K in slabs of 16 staged through LDS.  The next slab's global loads are in
// flight while the current one is multiplied (clamped addresses, so every
// load is issued unconditionally; out-of-range elements are zeroed after
// the load).  TS = 32 where 64 x 64 tiles would leave most of the chip idle.
// ---------------------------------------------------------------------------
template <bool TA, bool TB, int TS>
__global__ void __launch_bounds__(256)
k_gemm_f64(int M, int N, int K, double alpha, const double* __restrict__ A, int lda,
           const double* __restrict__ B, int ldb, double beta, double* __restrict__ C, int ldc,
           size_t zs) {
  constexpr int LPT = TS / 16;  // elements of each slab per thread
  constexpr int WB = TS / 32;   // 16 x 16 blocks per wave and dimension
  __shared__ double As[16][TS + 2];
  __shared__ double Bs[16][TS + 2];
  A = zw(A, zs);
  B = zw(B, zs);
  C = zw(C, zs);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * TS, n0 = blockIdx.x * TS;
  const int wr = (wave >> 1) * (TS / 2), wc = (wave & 1) * (TS / 2);
  const int lr = lane & 15, lk = lane >> 4;
  // this thread's slab elements: (i, k) of A's tile and (kk, j) of B's
  int ai[LPT], ak[LPT], bk[LPT], bj[LPT];
#pragma unroll
  for (int q = 0; q < LPT; ++q) {
    const int e = tid + 256 * q;
    if (TA) { ai[q] = e % TS; ak[q] = e / TS; } else { ak[q] = e % 16; ai[q] = e / 16; }
    if (TB) { bk[q] = e % 16; bj[q] = e / 16; } else { bj[q] = e % TS; bk[q] = e / TS; }
  }
  double ra[LPT], rb[LPT];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int gi = std::min(m0 + ai[q], M - 1), gk = std::min(k0 + ak[q], K - 1);
      ra[q] = TA ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk];
      const int gj = std::min(n0 + bj[q], N - 1), gkk = std::min(k0 + bk[q], K - 1);
      rb[q] = TB ? B[(size_t)gj * ldb + gkk] : B[(size_t)gkk * ldb + gj];
    }
  };
  v4d acc[WB][WB];
#pragma unroll
  for (int bi = 0; bi < WB; ++bi)
#pragma unroll
    for (int bjj = 0; bjj < WB; ++bjj) acc[bi][bjj] = v4d{0.0, 0.0, 0.0, 0.0};
  if (K > 0) fetch(0);  // (K = 0: no slab, C = beta C)
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      As[ak[q]][ai[q]] = (m0 + ai[q] < M && k0 + ak[q] < K) ? ra[q] : 0.0;
      Bs[bk[q]][bj[q]] = (n0 + bj[q] < N && k0 + bk[q] < K) ? rb[q] : 0.0;
    }
    __syncthreads();
    if (k0 + 16 < K) fetch(k0 + 16);
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
      double a[WB], b[WB];
#pragma unroll
      for (int bi = 0; bi < WB; ++bi) {
        a[bi] = As[k4 + lk][wr + 16 * bi + lr];
        b[bi] = Bs[k4 + lk][wc + 16 * bi + lr];
      }
#pragma unroll
      for (int bi = 0; bi < WB; ++bi)
#pragma unroll
        for (int bjj = 0; bjj < WB; ++bjj)
          acc[bi][bjj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bjj], acc[bi][bjj], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < WB; ++bi)
#pragma unroll
    for (int bjj = 0; bjj < WB; ++bjj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = m0 + wr + 16 * bi + lk + 4 * j, cc = n0 + wc + 16 * bjj + lr;
        if (r < M && cc < N) {
          double v = alpha * acc[bi][bjj][j];
          if (beta != 0.0) v += beta * C[(size_t)r * ldc + cc];
          C[(size_t)r * ldc + cc] = v;
        }
      }
}

int gemm_f64(kdqmc_ctx* c, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
             int lda, const double* B, int ldb, double beta, double* C, int ldc) {
  if (M <= 0 || N <= 0) return KDQMC_OK;
  const int e0 = prof_mark(c);
  // 64 x 64 tiles when they give at least one workgroup per CU, else 32 x 32
  const bool big = (size_t)((N + 63) / 64) * ((M + 63) / 64) * c->nch >= 256;
#define GEMM(TA, TB, TS)                                                                               \
  hipLaunchKernelGGL((k_gemm_f64<TA, TB, TS>), dim3((N + TS - 1) / TS, (M + TS - 1) / TS, c->nch), dim3(256), \
                     0, c->stream, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, c->zs)
  if (big) {
    if (!ta && !tb) GEMM(false, false, 64);
    else if (ta && !tb) GEMM(true, false, 64);
    else if (!ta && tb) GEMM(false, true, 64);
    else GEMM(true, true, 64);
  } else {
    if (!ta && !tb) GEMM(false, false, 32);
    else if (ta && !tb) GEMM(true, false, 32);
    else if (!ta && tb) GEMM(false, true, 32);
    else GEMM(true, true, 32);
  }
#undef GEMM
  prof_pair(c, PH_GEMM, e0, prof_mark(c));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

// ---------------------------------------------------------------------------
// Householder QR, blocked (compact WY form).
//
// Panels of width nbp = 16 are factored by one workgroup of NT = 256 threads
// (512 for panels of more than 1024 rows) holding the panel in registers
// (thread t owns rows j+t, j+t+NT, ..., RPT = 2 or 4 of them).  H_c = I - tau_c v_c v_c^T with
// v_c[jc] = 1 (LAPACK convention); H_0 ... H_{nbp-1} = I - V T V^T.
// Outputs: R in A (zeros below the diagonal), explicit V in Vq (unit diagonal,
// zeros above), T in Tq (row stride 32), tau.
// The block reflector is applied to the trailing columns (and later to the
// identity to form Q, or to a right-hand side) by k_apply_wy, one launch per
// panel, with both products on the FP64 MFMA.
// ---------------------------------------------------------------------------
constexpr int kNBmax = 32;
constexpr int kPanelThreads = 256;

// Lane exchange within a wave (the value of lane ^ mask) without LDS
// traffic: DPP quad permutations for masks 1 and 2; for 4 and 8 a shift
// within the row of 16 lanes whose direction is the lane's bit (lane + mask
// where the bit is clear, lane - mask where it is set); for 16 and 32 the
// permlane swaps, which hand every lane both members of its pair.
__device__ __forceinline__ int xchg_dword(int x, int mask, int lane) {
  switch (mask) {
    case 1:
      return __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
    case 2:
      return __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
    case 4: {
      const int up = __builtin_amdgcn_mov_dpp(x, 0x104, 0xF, 0xF, true);  // row_shl:4
      const int dn = __builtin_amdgcn_mov_dpp(x, 0x114, 0xF, 0xF, true);  // row_shr:4
      return (lane & 4) ? dn : up;
    }
    case 8: {
      const int up = __builtin_amdgcn_mov_dpp(x, 0x108, 0xF, 0xF, true);  // row_shl:8
      const int dn = __builtin_amdgcn_mov_dpp(x, 0x118, 0xF, 0xF, true);  // row_shr:8
      return (lane & 8) ? dn : up;
    }
    case 16: {  // element 0: even rows' values in every row; element 1: odd rows'
      const auto sw = __builtin_amdgcn_permlane16_swap(x, x, false, false);
      return (lane & 16) ? (int)sw[0] : (int)sw[1];
    }
    default: {  // 32; element 0: lanes 0-31's values in both halves; element 1: lanes 32-63's
      const auto sw = __builtin_amdgcn_permlane32_swap(x, x, false, false);
      return (lane & 32) ? (int)sw[0] : (int)sw[1];
    }
  }
}
__device__ __forceinline__ double xchg_xor(double v, int mask, int lane) {
  return __hiloint2double(xchg_dword(__double2hiint(v), mask, lane), xchg_dword(__double2loint(v), mask, lane));
}

// a + (a of lane l ^ M) in the lanes whose bit M is clear, b + (b of lane
// l ^ M) in the others (M = 32: v_permlane32_swap, 16: v_permlane16_swap,
// which exchange a's upper half / odd rows with b's lower half / even rows).
template <int M>
__device__ __forceinline__ double swap_sum(double a, double b) {
  static_assert(M == 16 || M == 32, "permlane swap width");
  const int ah = __double2hiint(a), al = __double2loint(a), bh = __double2hiint(b), bl = __double2loint(b);
  if constexpr (M == 32) {
    const auto h = __builtin_amdgcn_permlane32_swap(ah, bh, false, false);
    const auto l = __builtin_amdgcn_permlane32_swap(al, bl, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
  } else {
    const auto h = __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
    const auto l = __builtin_amdgcn_permlane16_swap(al, bl, false, false);
    return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
  }
}

// a double moved by one DPP control (both halves)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  return __hiloint2double(__builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true),
                          __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true));
}

// One panel of the Householder QR.  Column c (row jc = j + c) needs, over
// the rows r >= jc, the dot products d_t = sum_r a_c[r] a_t[r] with every
// column t of the panel, and the row jc itself.  With alpha = a_c[jc],
// beta = -sign(alpha) sqrt(d_c) and u = a_c - beta e_jc (rows >= jc):
//   v_c = u / (alpha - beta),   tau_c = (beta - alpha) / beta,
//   v_c^T a_t = (d_t - beta a_t[jc]) / (alpha - beta),
// the last being the Householder coefficient of a trailing column t and,
// for an earlier column t (which holds v_t below its diagonal), the entry
// (V^T V)[t][c] of the T factor.  So every column costs one workgroup-wide
// reduction of NB sums and one barrier (the reduction buffers and the
// published row are double-buffered).
//
// The same broadcast coefficients build T: with w_t = -tau_c (V^T V)[t][c]
// for the earlier columns t, column c of T is T[0:c, 0:c] w (and tau_c on
// the diagonal).  Workgroups of 256 threads keep row l of T in lane l's
// registers and add one term per earlier column (no pass over T follows the
// loop); larger ones, with less register room per thread, store V^T V and
// build T after the loop with one wave.
//
// The panel passes through LDS on the way in and out (chunks of up to 1024
// rows), so that global loads and stores run along rows (16 lanes per row
// of 16 columns) rather than one row per lane, which touches 64 cache lines
// per instruction.
//
// All NB columns are unrolled, so register indices and whether a column is
// trailing or factored are compile-time constants (no selects between the
// two updates).
// The panel factorization by threads 0 .. NT-1 of a workgroup (pointers
// already shifted to the chain).
// Rows of a panel staged through LDS at a time.
template <int RPT, int NT>
constexpr int panel_chunk() {
  return RPT * NT < 1024 ? RPT * NT : 1024;
}

// Pst: the caller's staging buffer (panel_chunk x (NB + 1) doubles).  PRE: the
// caller has already written the panel into it (rows j.., one chunk) and
// synchronized, so the global load is skipped.
template <int RPT, int NB, int NT, bool PRE = false>
__device__ __forceinline__ void qr_panel_body(double* __restrict__ A, int lda, int n, int j, int nbp,
                                              double* __restrict__ Vq, double* __restrict__ Tq,
                                              double* __restrict__ tau_out, double (*Pst)[NB + 1]) {
  constexpr int NW = NT / 64;
  static_assert(NB == 16 && NT >= NB, "panel shape (staging assumes 16 columns)");
  constexpr int kRows = RPT * NT;                         // rows the workgroup holds
  constexpr int kChunk = panel_chunk<RPT, NT>();           // rows staged at a time
  static_assert(!PRE || kRows == kChunk, "a pre-staged panel is one chunk");
  constexpr int kQc = kChunk / NT;                        // row slots per thread and chunk
  constexpr int kPass = kChunk / (NT / 16);               // staging rows per thread and chunk
  static_assert(kRows % kChunk == 0 && kChunk % NT == 0, "staging chunks");
  constexpr bool kRegT = NT <= 256;  // T in registers (else built from V^T V in LDS)
  __shared__ double red[2][NW][NB];   // per-wave partial sums d_t
  __shared__ double rowv[2][NB];      // row jc of the panel
  __shared__ double Ts[NB][NB + 1];
  __shared__ double Sv[kRegT ? 1 : NB][NB + 1];  // V^T V, strict upper part
  __shared__ double betas[NB];
  __shared__ double taus[NB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int pl = lane & (NB - 1);     // the sum this lane ends up holding
  double a[RPT][NB];
  double tr[NB];  // row `lane` of T (lanes below NB)
  int row[RPT];
#pragma unroll
  for (int p = 0; p < NB; ++p) tr[p] = 0.0;
#pragma unroll
  for (int q = 0; q < RPT; ++q) row[q] = j + tid + q * NT;
  const int mrows = std::min(n - j, kRows);  // rows of the panel
  const int sc = lane & 15, sr = tid >> 4;   // staging: 16 lanes per row
  // per chunk, all loads issued before the first wait (rows past the panel
  // and columns past nbp read a valid address and store 0); thread t then
  // takes its rows t + q NT of the chunk
#pragma unroll
  for (int h = 0; h < kRows / kChunk; ++h) {
    if constexpr (!PRE) {
      double v[kPass];
#pragma unroll
      for (int k = 0; k < kPass; ++k) {
        const int r = h * kChunk + sr + k * (NT / 16);
        v[k] = A[(size_t)(j + std::min(r, mrows - 1)) * lda + j + (sc < nbp ? sc : 0)];
      }
      if (h > 0) __syncthreads();  // the previous chunk has been read
#pragma unroll
      for (int k = 0; k < kPass; ++k) {
        const int r = h * kChunk + sr + k * (NT / 16);
        Pst[sr + k * (NT / 16)][sc] = (r < mrows && sc < nbp) ? v[k] : 0.0;
      }
      __syncthreads();
    }
#pragma unroll
    for (int qq = 0; qq < kQc; ++qq) {
      const int q = h * kQc + qq;
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) a[q][cc] = (row[q] < n) ? Pst[tid + qq * NT][cc] : 0.0;
    }
  }

  // every column unrolled: register indices and the roles of the positions
  // (factored below c, trailing above) are compile-time constants
#pragma clang loop unroll(full)
  for (int c = 0; c < NB; ++c) {
    if (c < nbp) {
      const int jc = j + c;
      const int buf = c & 1;
      if (tid == c) {  // owner of row jc (its first row)
#pragma unroll
        for (int p = 0; p < NB; ++p) rowv[buf][p] = a[0][p];
      }
      double x[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) x[q] = (row[q] >= jc && row[q] < n) ? a[q][c] : 0.0;
      double part[NB];
#pragma unroll
      for (int p = 0; p < NB; ++p) {
        double sacc = 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) sacc = fma(x[q], a[q][p], sacc);
        part[p] = sacc;
      }
      // reduce-scatter within the wave: halving the sums a lane holds on
      // lane bits 5 and 4 (permlane swaps, which move a pair of sums
      // without selects), then 1 and 0 (quad DPP), and the full sum over
      // bits 2 and 3 (row rotations); lane l then holds sum number
      // 8 b0 + 4 b1 + 2 b4 + b5 (bK = bit K of l)
      {
#pragma unroll
        for (int h = 0; h < NB / 2; ++h) part[h] = swap_sum<32>(part[2 * h], part[2 * h + 1]);
#pragma unroll
        for (int h = 0; h < NB / 4; ++h) part[h] = swap_sum<16>(part[2 * h], part[2 * h + 1]);
#pragma unroll
        for (int b = 1; b >= 0; --b) {
          const int bit = (lane >> b) & 1;
#pragma unroll
          for (int h = 0; h < (1 << b); ++h) {
            const double keep = bit ? part[2 * h + 1] : part[2 * h];
            const double send = bit ? part[2 * h] : part[2 * h + 1];
            part[h] = keep + xchg_xor(send, 1 << b, lane);
          }
        }
        double v = part[0];
        v += dpp_f64<0x124>(v);  // row_ror:4
        v += dpp_f64<0x128>(v);  // row_ror:8
        if ((lane & 12) == 0)
          red[buf][wave][8 * (lane & 1) + 2 * (lane & 2) + 2 * ((lane >> 4) & 1) + (lane >> 5)] = v;
      }
      __syncthreads();
      double tot = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) tot += red[buf][w][pl];
      const double rv = rowv[buf][pl];
      const double ss = lane_value(tot, c);
      const double alpha = lane_value(rv, c);
      double tau_c, beta, scale;
      if (!(ss - alpha * alpha > 0.0)) {  // nothing below the diagonal: H = I
        tau_c = 0.0;
        beta = alpha;
        scale = 0.0;
      } else {
        // alpha - beta = alpha + sign(alpha) nrm (no cancellation) and
        // tau = (beta - alpha) / beta = |alpha - beta| / nrm
        const double y = rsqrt_nr(ss);
        const double nrm = ss * y;
        const double d = (alpha >= 0.0) ? alpha + nrm : alpha - nrm;
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau_c = fabs(d) * y;
        scale = rcp_nr(d);
      }
      const double wv = (tot - beta * rv) * scale;  // v_c^T a_t for t = pl
      const double tw = -tau_c * wv;
      if constexpr (!kRegT) {
        if (wave == 0 && lane < c) Sv[lane][c] = wv;
      }
      if (tid == 0) {
        betas[c] = beta;
        taus[c] = tau_c;
      }
      double vq[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = row[q];
        const double v = (r < jc || r >= n) ? 0.0 : (r == jc ? 1.0 : a[q][c] * scale);
        vq[q] = v;
        if (r >= jc) a[q][c] = v;
      }
      // trailing columns take the rank-1 update; the factored ones add to
      // row `lane` of T's column c
      double tsum = 0.0;
#pragma unroll
      for (int p = 0; p < NB; ++p) {
        if (p > c) {
          const double fp = lane_value(tw, p);
#pragma unroll
          for (int q = 0; q < RPT; ++q) a[q][p] = fma(fp, vq[q], a[q][p]);
        } else if (p < c) {
          if constexpr (kRegT) tsum = fma(tr[p], lane_value(tw, p), tsum);
        }
      }
      if constexpr (kRegT) tr[c] = (lane < c) ? tsum : (lane == c ? tau_c : 0.0);
    }
  }
  if constexpr (kRegT) {
    if (wave == 0 && lane < NB) {
#pragma unroll
      for (int p = 0; p < NB; ++p) Ts[lane][p] = tr[p];
    }
  } else {
    __syncthreads();
    // T[cc][cc] = tau_cc, T[0:cc, cc] = -tau_cc T[0:cc, 0:cc] (V^T V)[0:cc, cc]
    // (one wave, no barriers)
    if (wave == 0) {
      for (int cc = 0; cc < nbp; ++cc) {
        double tv = 0.0;
        if (lane < cc) {
          for (int t = lane; t < cc; ++t) tv += Ts[lane][t] * Sv[t][cc];
          tv *= -taus[cc];
        }
        if (lane < cc) Ts[lane][cc] = tv;
        if (lane == cc) Ts[cc][cc] = taus[cc];
        if (lane > cc && lane < NB) Ts[lane][cc] = 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
  // out through LDS, a chunk at a time: R above the diagonal, beta on it,
  // zeros below; V: zeros above, 1 on the diagonal, v below
#pragma unroll
  for (int h = 0; h < kRows / kChunk; ++h) {
    if (h > 0) __syncthreads();  // the previous chunk has been stored
#pragma unroll
    for (int qq = 0; qq < kQc; ++qq)
#pragma unroll
      for (int p = 0; p < NB; ++p) Pst[tid + qq * NT][p] = a[h * kQc + qq][p];
    __syncthreads();
    const double bsc = betas[sc];
    double x[kPass];
#pragma unroll
    for (int k = 0; k < kPass; ++k) x[k] = Pst[sr + k * (NT / 16)][sc];
#pragma unroll
    for (int k = 0; k < kPass; ++k) {
      const int r = h * kChunk + sr + k * (NT / 16);
      if (r < mrows && sc < nbp) {
        const int gr = j + r, jc = j + sc;
        A[(size_t)gr * lda + jc] = (r < sc) ? x[k] : (r == sc ? bsc : 0.0);
        Vq[(size_t)gr * lda + jc] = (r < sc) ? 0.0 : (r == sc ? 1.0 : x[k]);
      }
    }
  }
  for (int idx = tid; idx < kNBmax * kNBmax; idx += NT) {
    const int r = idx / kNBmax, cc = idx % kNBmax;
    Tq[idx] = (r < nbp && cc < nbp) ? Ts[r][cc] : 0.0;
  }
  if (tid < nbp) tau_out[j + tid] = taus[tid];
}

template <int RPT, int NB, int NT>
__global__ void __launch_bounds__(NT)
k_qr_panel(double* __restrict__ A, int lda, int n, int j, int nbp, double* __restrict__ Vq,
           double* __restrict__ Tq, double* __restrict__ tau_out, size_t zs) {
  __shared__ double Pst[panel_chunk<RPT, NT>()][NB + 1];  // the panel, staged a chunk at a time
  qr_panel_body<RPT, NB, NT>(zw(A, zs), lda, n, j, nbp, zw(Vq, zs), zw(Tq, zs), zw(tau_out, zs), Pst);
}

// C[j:n, s0:s0+SW] -= V op(T) (V^T C[j:n, s0:s0+SW]) for the panel at column
// j (width nbp <= 32): op(T) = T^T applies H^T = H_{nbp-1} ... H_0 (the
// factorization / Q^T direction), op(T) = T applies H = H_0 ... H_{nbp-1}.
// One workgroup (8 waves, or 16 for forming Q) per SW-column stripe (SW = 16
// or 32; narrow stripes give more workgroups for the few-hundred-column
// matrices here).
// W = V^T C: the waves split the rows and their partial 32 x SW products are
// summed in LDS; then C -= V W2 with the waves splitting the rows.
template <int SW, int VB = 2, int NW = 8>
struct WyLds {
  double Wp[NW][16 * VB][SW + 1];
  double W2[16 * VB][SW + 1];
  double Tl[32][33];
};

// One panel applied to the stripe s0 of C (the body of k_apply_wy; NT threads);
// VB = 1 for reflectors of at most 16 columns (half the products of VB = 2).
template <int SW, int VB = 2, int NT = 512>
__device__ __forceinline__ void apply_wy_stripe(WyLds<SW, VB, NT / 64>& sh, double* __restrict__ C, int ldc,
                                                int n, int j, int nbp, int ncols, int s0,
                                                const double* __restrict__ V, int ldv,
                                                const double* __restrict__ T, int trans) {
  constexpr int NW = NT / 64;
  constexpr int BJ = SW / 16;
  constexpr int TH = kNBmax * kNBmax / NT;  // elements of T per thread
  // k-steps of W = V^T C whose loads are issued together (fewer where the
  // registers per thread are fewer: wide stripes, 16-wave workgroups)
  constexpr int U = (SW >= 64 || NT > 512) ? 2 : 4;
  auto& Wp = sh.Wp;
  auto& W2 = sh.W2;
  auto& Tl = sh.Tl;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int m = n - j;
  // Every global load below reads a clamped, in-range address unconditionally
  // and the out-of-range values are zeroed afterwards: a guarded load would
  // be a branch that waits for its data before the next load is issued.
  bool vin[VB], cin[BJ];
  int vcol[VB], ccol[BJ];
#pragma unroll
  for (int bi = 0; bi < VB; ++bi) {
    vin[bi] = bi * 16 + lr < nbp;
    vcol[bi] = j + (vin[bi] ? bi * 16 + lr : 0);
  }
#pragma unroll
  for (int bj = 0; bj < BJ; ++bj) {
    cin[bj] = s0 + bj * 16 + lr < ncols;
    ccol[bj] = cin[bj] ? s0 + bj * 16 + lr : 0;
  }
  // T's two elements per thread are loaded now and stored to LDS after the
  // V^T C loop, so that the loop does not wait for them
  double tv[TH];
#pragma unroll
  for (int h = 0; h < TH; ++h) tv[h] = T[tid + NT * h];
  // W = V^T C (32 x SW), rows split over waves in chunks of 4, U chunks per
  // round of loads
  v4d acc[VB][BJ];
#pragma unroll
  for (int bi = 0; bi < VB; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) acc[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int kb0 = wave * 4; kb0 < m; kb0 += 4 * NW * U) {
    double av[U][VB], bv[U][BJ];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t rc = (size_t)min(j + kb0 + 4 * NW * u + lk, n - 1);
#pragma unroll
      for (int bi = 0; bi < VB; ++bi) av[u][bi] = V[rc * ldv + vcol[bi]];
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj) bv[u][bj] = C[rc * ldc + ccol[bj]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool rin = j + kb0 + 4 * NW * u + lk < n;
#pragma unroll
      for (int bi = 0; bi < VB; ++bi) av[u][bi] = (rin && vin[bi]) ? av[u][bi] : 0.0;
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj) bv[u][bj] = (rin && cin[bj]) ? bv[u][bj] : 0.0;
#pragma unroll
      for (int bi = 0; bi < VB; ++bi)
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][bi], bv[u][bj], acc[bi][bj], 0, 0, 0);
    }
  }
#pragma unroll
  for (int bi = 0; bi < VB; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) Wp[wave][bi * 16 + lk + 4 * e][bj * 16 + lr] = acc[bi][bj][e];
#pragma unroll
  for (int h = 0; h < TH; ++h) {
    const int idx = tid + NT * h, r = idx >> 5, cc = idx & 31;
    Tl[r][cc] = (r < nbp && cc < nbp) ? tv[h] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < 16 * VB * SW; idx += NT) {
    const int r = idx / SW, cc = idx % SW;
    double sacc = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) sacc += Wp[w][r][cc];
    Wp[0][r][cc] = sacc;
  }
  __syncthreads();
  // W2 = op(T) W
  for (int idx = tid; idx < 16 * VB * SW; idx += NT) {
    const int r = idx / SW, cc = idx % SW;
    double sacc = 0.0;
    for (int t = 0; t < 16 * VB; ++t) sacc += (trans ? Tl[t][r] : Tl[r][t]) * Wp[0][t][cc];
    W2[r][cc] = sacc;
  }
  __syncthreads();
  // C -= V W2, 16-row blocks split over waves; the block's rows of V (and,
  // for one-tile stripes, the C elements it updates) are all loaded before
  // the first product.  Wider stripes read C at the update: holding their
  // 16 elements as well runs the whole-QR kernel out of registers.
  for (int rb = wave * 16; rb < m; rb += 16 * NW) {
    const int r = j + rb + lr;
    const size_t rc = (size_t)min(r, n - 1);
    double av[4 * VB], cv[BJ][4];
#pragma unroll
    for (int q = 0; q < 4 * VB; ++q) {
      const int vc = 4 * q + lk;
      av[q] = V[rc * ldv + j + (vc < nbp ? vc : 0)];
    }
    if constexpr (BJ == 1) {
#pragma unroll
      for (int e = 0; e < 4; ++e) cv[0][e] = C[(size_t)min(j + rb + lk + 4 * e, n - 1) * ldc + ccol[0]];
    }
    v4d d[BJ];
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) d[bj] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4 * VB; ++q) {
      const double a = (r < n && 4 * q + lk < nbp) ? av[q] : 0.0;
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj)
        d[bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, W2[4 * q + lk][bj * 16 + lr], d[bj], 0, 0, 0);
    }
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r2 = j + rb + lk + 4 * e;
        if (r2 < n && cin[bj]) {
          double* c = C + (size_t)r2 * ldc + ccol[bj];
          *c = (BJ == 1 ? cv[bj][e] : *c) - d[bj][e];
        }
      }
  }
}

template <int SW>
__global__ void __launch_bounds__(512)
k_apply_wy(double* __restrict__ C, int ldc, int n, int j, int nbp, int ncols,
           const double* __restrict__ V, int ldv, const double* __restrict__ T, int trans,
           size_t zs) {
  __shared__ WyLds<SW> sh;
  apply_wy_stripe<SW>(sh, zw(C, zs), ldc, n, j, nbp, ncols, blockIdx.x * SW, zw(V, zs), ldv, zw(T, zs),
                      trans);
}

// All panels of a factorization applied in turn to each SW-column stripe of C
// (one workgroup per stripe, no launch per panel): forward order with
// H^T (trans, op(T) = T^T) over all columns, as in applying Q^T; or backward
// order with H over the columns right of each panel's start, as in forming Q
// from the identity.  The panel table is the host's.
struct PanelTable {
  int start[160];
  int width[160];
};

// The whole Householder QR of one chain's n x ncol matrix in one workgroup
// (512 threads): panel by panel (the panels of the per-panel launches), each
// panel's reflector then applied to every trailing column in 64-column
// stripes.  For batches of many chains, where one workgroup per chain fills
// the device and the per-panel launches would spread every step of every
// chain over the chip; V, T and tau are those of the per-panel launches.
// The panel staging buffer and the apply's buffers share the LDS (never in
// use at the same time).
template <int RPT>
__global__ void __launch_bounds__(512)
k_qr_chain(double* __restrict__ A, int lda, int n, int ncol, double* __restrict__ Vq,
           double* __restrict__ Tq, double* __restrict__ tau, PanelTable pt, int npan, size_t zs) {
  constexpr size_t kPst = sizeof(double) * panel_chunk<RPT, 512>() * 17;
  constexpr size_t kWy = sizeof(WyLds<64, 1>);
  __shared__ __align__(16) unsigned char smem[kPst > kWy ? kPst : kWy];
  A = zw(A, zs);
  Vq = zw(Vq, zs);
  Tq = zw(Tq, zs);
  tau = zw(tau, zs);
  double(*Pst)[17] = reinterpret_cast<double(*)[17]>(smem);
  WyLds<64, 1>& sh = *reinterpret_cast<WyLds<64, 1>*>(smem);
  for (int p = 0; p < npan; ++p) {
    const int j = pt.start[p], nbp = pt.width[p];
    double* Tp = Tq + (size_t)p * kNBmax * kNBmax;
    qr_panel_body<RPT, 16, 512>(A, lda, n, j, nbp, Vq, Tp, tau, Pst);
    __syncthreads();
    for (int s0 = j + nbp; s0 < ncol; s0 += 64) {
      apply_wy_stripe<64, 1>(sh, A, lda, n, j, nbp, ncol, s0, Vq, lda, Tp, 1);
      __syncthreads();
    }
  }
}

template <int SW, int NT>
__global__ void __launch_bounds__(NT)
k_apply_wy_all(double* __restrict__ C, int ldc, int n, int ncols, const double* __restrict__ V, int ldv,
               const double* __restrict__ Tq, PanelTable pt, int npan, int backward, size_t zs) {
  __shared__ WyLds<SW, 2, NT / 64> sh;
  C = zw(C, zs);
  V = zw(V, zs);
  Tq = zw(Tq, zs);
  const int s0 = blockIdx.x * SW;
  for (int i = 0; i < npan; ++i) {
    const int p = backward ? npan - 1 - i : i;
    const int j = pt.start[p];
    if (backward && j > s0) continue;  // columns left of the panel are untouched
    apply_wy_stripe<SW, 2, NT>(sh, C, ldc, n, j, pt.width[p], ncols, s0, V, ldv,
                               Tq + (size_t)p * kNBmax * kNBmax, backward ? 0 : 1);
    __syncthreads();  // this panel's update is read by the next one
  }
}

// Consecutive panels p, p+1 (columns j1.., width b1; j2 = j1 + b1.., width
// b2) merged into one block reflector: H_p H_{p+1} = I - [V1 V2] T [V1 V2]^T
// with T = [[T1, -T1 (V1^T V2) T2], [0, T2]].  The apply kernels cost the
// same for widths up to 32, so applying the merged pairs halves the passes
// over C.  One workgroup (1024 threads: four row slices of the 16 x 16 sums
// V1^T V2) per pair; a lone last panel is copied.
__global__ void __launch_bounds__(1024)
k_merge_t(const double* __restrict__ V, int ldv, int n, const double* __restrict__ Tq, PanelTable pt,
          int npan, double* __restrict__ Tm, size_t zs) {
  __shared__ double T1[16][17], T2[16][17], S[16][17], X[16][17], Sp[16][16][17];
  V = zw(V, zs);
  Tq = zw(Tq, zs);
  Tm = zw(Tm, zs);
  const int qp = blockIdx.x, p1 = 2 * qp, tid = threadIdx.x;
  const int a = (tid >> 4) & 15, b = tid & 15, slice = tid >> 8;  // (a, b) of the 16 x 16 products
  double* out = Tm + (size_t)qp * kNBmax * kNBmax;
  const double* t1 = Tq + (size_t)p1 * kNBmax * kNBmax;
  if (p1 + 1 >= npan) {
    for (int e = tid; e < kNBmax * kNBmax; e += 1024) out[e] = t1[e];
    return;
  }
  const double* t2 = t1 + kNBmax * kNBmax;
  const int j1 = pt.start[p1], b1 = pt.width[p1], j2 = pt.start[p1 + 1], b2 = pt.width[p1 + 1];
  if (slice == 0) {
    T1[a][b] = (a < b1 && b < b1) ? t1[a * kNBmax + b] : 0.0;
    T2[a][b] = (a < b2 && b < b2) ? t2[a * kNBmax + b] : 0.0;
  }
  // (V1^T V2)[a][b] over the rows from j2 on (V2 is zero above) on the FP64
  // MFMA: wave w takes the 4-row k-steps j2 + 4 w + 64 i, a lane reading one
  // entry of each panel's row (rows contiguous across the lanes); the 16
  // waves' partial products are then summed
  {
    const int wave = tid >> 6, lane = tid & 63, lr = lane & 15, lk = lane >> 4;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int r0 = j2 + 4 * wave; r0 < n; r0 += 64) {
      const int r = r0 + lk;
      const double* row = V + (size_t)min(r, n - 1) * ldv;
      const double x1 = row[j1 + lr], x2 = row[j2 + lr];
      const double va = (r < n && lr < b1) ? x1 : 0.0;
      const double vb = (r < n && lr < b2) ? x2 : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va, vb, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) Sp[wave][lk + 4 * e][lr] = acc[e];
  }
  __syncthreads();
  if (tid >= 256) return;  // the rest is one 16 x 16 product chain
  {
    double s8[8];
#pragma unroll
    for (int w = 0; w < 8; ++w) s8[w] = Sp[w][a][b] + Sp[w + 8][a][b];
    S[a][b] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
  }
  __syncthreads();
  double x = 0.0;
  for (int k = 0; k < 16; ++k) x = fma(S[a][k], T2[k][b], x);
  X[a][b] = x;
  __syncthreads();
  double t12 = 0.0;
  for (int k = 0; k < 16; ++k) t12 = fma(T1[a][k], X[k][b], t12);
  for (int e = tid; e < kNBmax * kNBmax; e += 256) out[e] = 0.0;
  __syncthreads();
  out[a * kNBmax + b] = T1[a][b];
  if (b < b2) {
    out[a * kNBmax + b1 + b] = -t12;
    if (a < b2) out[(b1 + a) * kNBmax + b1 + b] = T2[a][b];
  }
}

// The same apply for one 16-column reflector on a 16-column stripe in the
// look-ahead step (at most 512 rows below the next panel, so at most 528
// from the reflector's first row), with every global load of both products
// issued before the first is used: rows of V and C for W = V^T C (wave w
// takes rows w*4 + 32 i, i < 17) and rows of V for C -= V W2 (16-row blocks
// w*16 + 128 k, k < 5).  512 threads.
__device__ __forceinline__ void apply_wy_short(WyLds<16, 1>& sh, double* __restrict__ C, int ldc, int n,
                                               int j, int nbp, int ncols, int s0,
                                               const double* __restrict__ V, int ldv,
                                               const double* __restrict__ T,
                                               double (*dst)[17] = nullptr, int dst_row0 = 0) {
  constexpr int NW = 8, KI = 17, KB = 5;  // 32 KI >= 528 and 128 KB >= 528
  auto& Wp = sh.Wp;
  auto& W2 = sh.W2;
  auto& Tl = sh.Tl;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int m = n - j;
  const bool vin = lr < nbp, cin = s0 + lr < ncols;
  const int vcol = j + (vin ? lr : 0), ccol = cin ? s0 + lr : 0;
  double tv[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) tv[h] = T[tid + 512 * h];
  double av[KI], bv[KI], vq[KB][4];
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int r = j + min(wave * 4 + 32 * i + lk, m - 1);
    av[i] = V[(size_t)r * ldv + vcol];
    bv[i] = C[(size_t)r * ldc + ccol];
  }
#pragma unroll
  for (int k = 0; k < KB; ++k)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int r = j + min(wave * 16 + 128 * k + lr, m - 1);
      vq[k][kk] = V[(size_t)r * ldv + j + min(4 * kk + lk, nbp - 1)];
    }
  // W = V^T C over the rows (rows past the panel and columns past the
  // reflector / the stripe weigh 0)
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < KI; ++i) {
    const int rr = wave * 4 + 32 * i + lk;
    const bool in = rr < m;
    const double a = (in && vin) ? av[i] : 0.0;
    const double b = (in && cin) ? bv[i] : 0.0;
    if (dst != nullptr && in && j + rr >= dst_row0) dst[j + rr - dst_row0][lr] = b;
    if (wave * 4 + 32 * i < m) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) Wp[wave][lk + 4 * e][lr] = acc[e];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int idx = tid + 512 * h, r = idx >> 5, cc = idx & 31;
    Tl[r][cc] = (r < nbp && cc < nbp) ? tv[h] : 0.0;
  }
  __syncthreads();
  if (tid < 256) {
    const int r = tid >> 4, cc = tid & 15;
    double sacc = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) sacc += Wp[w][r][cc];
    Wp[0][r][cc] = sacc;
  }
  __syncthreads();
  // W2 = T^T W
  if (tid < 256) {
    const int r = tid >> 4, cc = tid & 15;
    double sacc = 0.0;
#pragma unroll
    for (int t = 0; t < 16; ++t) sacc += Tl[t][r] * Wp[0][t][cc];
    W2[r][cc] = sacc;
  }
  __syncthreads();
  // C -= V W2
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int rb = wave * 16 + 128 * k;
    if (rb < m) {
      v4d d = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int vc = 4 * kk + lk;
        const double a = (j + rb + lr < n && vc < nbp) ? vq[k][kk] : 0.0;
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, W2[vc][lr], d, 0, 0, 0);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = j + rb + lk + 4 * e, cc = s0 + lr;
        if (dst != nullptr && r >= dst_row0) {  // in the caller's LDS rows (0 past ncols)
          if (r < n) dst[r - dst_row0][lr] -= d[e];
        } else if (r < n && cc < ncols) {
          C[(size_t)r * ldc + cc] -= d[e];
        }
      }
    }
  }
}

// One step of the factorization with look-ahead (16-column panels of at
// most 512 rows): workgroup 0 applies panel
// p's reflector (columns jp.., width nbp, factor Tp) to the next panel's
// columns and then factors that panel (threads 0 .. NT-1); the other
// workgroups apply panel p's reflector to the 16-column stripes beyond the
// next panel, concurrently.  Both read only panel p's V and T and write
// disjoint columns.
template <int RPT, int NB, int NT>
__global__ void __launch_bounds__(512)
k_qr_step(double* __restrict__ A, int lda, int n, int ncols, int jp, int nbp, const double* __restrict__ Tp,
          int jn, int nbn, double* __restrict__ Vq, double* __restrict__ Tn, double* __restrict__ tau,
          size_t zs) {
  static_assert(NT <= 512, "the panel runs inside a 512-thread workgroup");
  __shared__ WyLds<16, 1> sh;
  A = zw(A, zs);
  Vq = zw(Vq, zs);
  Tp = zw(Tp, zs);
  if (blockIdx.x == 0) {
    // the updated panel rows (from jn on) go straight into the panel's
    // staging buffer; the rows above it (final entries of R) to A
    __shared__ double Pst[panel_chunk<RPT, NT>()][NB + 1];
    static_assert(NB == 16 && RPT * NT == panel_chunk<RPT, NT>(), "one 16-column stripe, one chunk");
    apply_wy_short(sh, A, lda, n, jp, nbp, ncols, jn, Vq, lda, Tp, Pst, jn);
    __syncthreads();
    if (threadIdx.x >= NT) return;  // waves past the panel's leave; barriers count the rest
    qr_panel_body<RPT, NB, NT, true>(A, lda, n, jn, nbn, Vq, zw(Tn, zs), zw(tau, zs), Pst);
  } else {
    apply_wy_short(sh, A, lda, n, jp, nbp, ncols, jn + nbn + (blockIdx.x - 1) * 16, Vq, lda, Tp);
  }
}

// Split-K form of the same apply for tall panels (more than 512 rows), so
// that the whole chip works on it instead of one workgroup per stripe:
// k_wy_partial: workgroup (stripe, q) sums V^T C over rows
//   [j + q rc, j + (q+1) rc) into Wpart[q][32][ncols] (4 waves split the rows);
// k_wy_reduce: workgroup (stripe) adds up the partial products of its columns
//   and writes W2 = op(T) W over chunk 0's partials;
// k_wy_update: workgroup (stripe, 64-row tile) subtracts V W2 from its tile.
constexpr int kWyChunks = 16;

template <int SW>
__global__ void __launch_bounds__(256)
k_wy_partial(const double* __restrict__ C, int ldc, int n, int j, int nbp, int ncols,
             const double* __restrict__ V, int ldv, int rc, double* __restrict__ Wpart, size_t zs) {
  C = zw(C, zs);
  V = zw(V, zs);
  Wpart = zw(Wpart, zs);
  constexpr int NW = 4;
  constexpr int BJ = SW / 16;
  __shared__ double Wp[NW][32][SW + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int s0 = blockIdx.x * SW, q = blockIdx.y;
  const int r0 = j + q * rc, r1 = min(n, r0 + rc);
  v4d acc[2][BJ];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) acc[bi][bj] = v4d{0.0, 0.0, 0.0, 0.0};
  // clamped in-range loads, U k-steps' worth issued together, zeroed
  // afterwards where out of range (a guarded load waits for its data)
  constexpr int U = 4;
  const bool two = nbp > 16;  // reflector columns 16..31 present (same for every lane)
  bool vin[2], cin[BJ];
  int vcol[2], ccol[BJ];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
    vin[bi] = bi * 16 + lr < nbp;
    vcol[bi] = j + (vin[bi] ? bi * 16 + lr : 0);
  }
#pragma unroll
  for (int bj = 0; bj < BJ; ++bj) {
    cin[bj] = s0 + bj * 16 + lr < ncols;
    ccol[bj] = cin[bj] ? s0 + bj * 16 + lr : 0;
  }
  for (int kb0 = r0 + wave * 4; kb0 < r1; kb0 += 4 * NW * U) {
    double av[U][2], bv[U][BJ];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t rcl = (size_t)min(kb0 + 4 * NW * u + lk, r1 - 1);
      av[u][0] = V[rcl * ldv + vcol[0]];
      av[u][1] = two ? V[rcl * ldv + vcol[1]] : 0.0;
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj) bv[u][bj] = C[rcl * ldc + ccol[bj]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool rin = kb0 + 4 * NW * u + lk < r1;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) av[u][bi] = (rin && vin[bi]) ? av[u][bi] : 0.0;
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj) bv[u][bj] = (rin && cin[bj]) ? bv[u][bj] : 0.0;
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj)
        acc[0][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][0], bv[u][bj], acc[0][bj], 0, 0, 0);
      if (two) {
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj)
          acc[1][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][1], bv[u][bj], acc[1][bj], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
      for (int e = 0; e < 4; ++e) Wp[wave][bi * 16 + lk + 4 * e][bj * 16 + lr] = acc[bi][bj][e];
  __syncthreads();
  for (int idx = tid; idx < 32 * SW; idx += 256) {
    const int r = idx / SW, cc = idx % SW;
    if (s0 + cc < ncols)
      Wpart[((size_t)q * 32 + r) * ncols + s0 + cc] = Wp[0][r][cc] + Wp[1][r][cc] + Wp[2][r][cc] + Wp[3][r][cc];
  }
}

template <int SW>
__global__ void __launch_bounds__(256)
k_wy_reduce(int nbp, int ncols, const double* __restrict__ T, int trans, double* __restrict__ Wpart, int nq,
            size_t zs) {
  T = zw(T, zs);
  Wpart = zw(Wpart, zs);
  __shared__ double Tl[32][33];
  __shared__ double Ws[32][SW + 1];
  const int tid = threadIdx.x;
  const int s0 = blockIdx.x * SW;
  for (int idx = tid; idx < 32 * 32; idx += 256) {
    const int r = idx >> 5, cc = idx & 31;
    Tl[r][cc] = (r < nbp && cc < nbp) ? T[r * kNBmax + cc] : 0.0;
  }
  // all kWyChunks partials read at once (clamped chunk and column, the
  // extra ones zeroed), then summed in chunk order
  for (int idx = tid; idx < 32 * SW; idx += 256) {
    const int r = idx / SW, cc = idx % SW;
    const bool in = s0 + cc < ncols;
    const int col = in ? s0 + cc : 0;
    double pv[kWyChunks];
#pragma unroll
    for (int q = 0; q < kWyChunks; ++q) pv[q] = Wpart[((size_t)min(q, nq - 1) * 32 + r) * ncols + col];
    double sacc = 0.0;
#pragma unroll
    for (int q = 0; q < kWyChunks; ++q) sacc += (in && q < nq) ? pv[q] : 0.0;
    Ws[r][cc] = sacc;
  }
  __syncthreads();
  for (int idx = tid; idx < 32 * SW; idx += 256) {
    const int r = idx / SW, cc = idx % SW;
    double sacc = 0.0;
    for (int t = 0; t < 32; ++t) sacc += (trans ? Tl[t][r] : Tl[r][t]) * Ws[t][cc];
    if (s0 + cc < ncols) Wpart[(size_t)r * ncols + s0 + cc] = sacc;
  }
}

template <int SW>
__global__ void __launch_bounds__(256)
k_wy_update(double* __restrict__ C, int ldc, int n, int j, int nbp, int ncols,
            const double* __restrict__ V, int ldv, const double* __restrict__ W2g, size_t zs) {
  C = zw(C, zs);
  V = zw(V, zs);
  W2g = zw(W2g, zs);
  constexpr int BJ = SW / 16;
  __shared__ double W2[32][SW + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int s0 = blockIdx.x * SW;
  for (int idx = tid; idx < 32 * SW; idx += 256) {
    const int r = idx / SW, cc = idx % SW;
    W2[r][cc] = (s0 + cc < ncols) ? W2g[(size_t)r * ncols + s0 + cc] : 0.0;
  }
  __syncthreads();
  // the tile's rows of V (the k-steps that hold reflector columns) and the C
  // elements it updates are read (clamped, in range) before the first
  // product; out-of-range values are zeroed or not stored.  Issued after the
  // barrier, whose fence would wait for them.
  const int rb = j + blockIdx.y * 64 + wave * 16;
  const size_t rv = (size_t)min(rb + lr, n - 1);
  const int nkq = (nbp + 3) / 4;  // 4-column k-steps holding reflector columns (same for every lane)
  double av[8], cv[BJ][4];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int vc = 4 * q + lk;
    av[q] = q < nkq ? V[rv * ldv + j + (vc < nbp ? vc : 0)] : 0.0;
  }
#pragma unroll
  for (int bj = 0; bj < BJ; ++bj) {
    const int cc = s0 + bj * 16 + lr, col = cc < ncols ? cc : 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) cv[bj][e] = C[(size_t)min(rb + lk + 4 * e, n - 1) * ldc + col];
  }
  v4d d[BJ];
#pragma unroll
  for (int bj = 0; bj < BJ; ++bj) d[bj] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    if (q >= nkq) break;
    const double a = (rb + lr < n && 4 * q + lk < nbp) ? av[q] : 0.0;
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj)
      d[bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, W2[4 * q + lk][bj * 16 + lr], d[bj], 0, 0, 0);
  }
#pragma unroll
  for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = rb + lk + 4 * e, cc = s0 + bj * 16 + lr;
      if (r < n && cc < ncols) C[(size_t)r * ldc + cc] = cv[bj][e] - d[bj][e];
    }
}

// Q[0:m, 0:n] = the first n columns of the m x m identity.
__global__ void k_set_identity(double* __restrict__ Q, int m, int n, int ld, size_t zs) {
  Q = zw(Q, zs);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)m * n) {
    const int r = idx / n, cc = idx % n;
    Q[(size_t)r * ld + cc] = (r == cc) ? 1.0 : 0.0;
  }
}

__global__ void k_zero(double* __restrict__ X, size_t count, size_t zs) {
  X = zw(X, zs);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) X[idx] = 0.0;
}

namespace {

// Panel width: 16 columns at every height (the per-column reduction and
// update scale with the width; 32-column panels of up to 1024 rows measured
// 4.6 us per column against 2.0 for 16-column panels with four rows per
// thread).
inline int panel_width(int) { return 16; }

// batches of at least this many chains factor each chain in one workgroup
constexpr int kQrChainMin = 128;

int launch_panel(kdqmc_ctx* c, double* A, int ld, int n, int j, int nbp, double* Tp) {
  const int m = n - j;
  const int e0 = prof_mark(c);
#define PANEL(RPT, NB, NT)                                                                          \
  hipLaunchKernelGGL((k_qr_panel<RPT, NB, NT>), dim3(1, 1, c->nch), dim3(NT), 0, c->stream, A, ld, n, j, \
                     nbp, c->Vq, Tp, c->tau, c->zs)
  // the panel's rows must fit in RPT * NT (lattices up to L = 24: N <= 1728)
  // and its width in NB (panel_width); more rows per thread rather than more
  // waves, whose per-wave reductions would compete for the same SIMDs
  if (m <= 512) PANEL(2, 16, 256);
  else if (m <= 1024) PANEL(4, 16, 256);
  else if (m <= 2048) PANEL(4, 16, 512);
  else return set_error(KDQMC_EUNSUPPORTED, "QR panel of more than 2048 rows");
#undef PANEL
  prof_pair(c, PH_QR_PANEL, e0, prof_mark(c));
  return KDQMC_OK;
}

int launch_apply(kdqmc_ctx* c, double* C, int ld, int n, int j, int nbp, int col0, int ncols,
                 const double* Tp, bool trans) {
  if (ncols <= col0) return KDQMC_OK;
  const int e0 = prof_mark(c);
  // the kernels index columns from C's base: shift the base to col0
  constexpr int SW = 16;
  const int stripes = (ncols - col0 + SW - 1) / SW;
  const int m = n - j;
  if (m <= 512) {
    hipLaunchKernelGGL(k_apply_wy<SW>, dim3(stripes, 1, c->nch), dim3(512), 0, c->stream, C + col0, ld, n, j,
                       nbp, ncols - col0, c->Vq, ld, Tp, trans ? 1 : 0, c->zs);
  } else {
    const int rc = ((m + kWyChunks - 1) / kWyChunks + 15) / 16 * 16;  // rows per chunk
    const int nq = (m + rc - 1) / rc;                                  // <= kWyChunks
    hipLaunchKernelGGL(k_wy_partial<SW>, dim3(stripes, nq, c->nch), dim3(256), 0, c->stream, C + col0, ld, n,
                       j, nbp, ncols - col0, c->Vq, ld, rc, c->Wq, c->zs);
    hipLaunchKernelGGL(k_wy_reduce<SW>, dim3(stripes, 1, c->nch), dim3(256), 0, c->stream, nbp, ncols - col0,
                       Tp, trans ? 1 : 0, c->Wq, nq, c->zs);
    hipLaunchKernelGGL(k_wy_update<SW>, dim3(stripes, (m + 63) / 64, c->nch), dim3(256), 0, c->stream,
                       C + col0, ld, n, j, nbp, ncols - col0, c->Vq, ld, c->Wq, c->zs);
  }
  prof_pair(c, PH_GEMM, e0, prof_mark(c));
  return KDQMC_OK;
}

}  // namespace

// All panels of the last factorization applied to C, one launch: backward
// (forming Q from the identity) or forward with H^T (applying Q^T).
// The merged pairs' table and factors (k_merge_t, run at the end of every QR).
int launch_apply_all(kdqmc_ctx* c, double* C, int ld, int n, int ncols, bool backward) {
  static_assert(sizeof(PanelTable) <= 2048, "kernel argument size");
  PanelTable pt;
  const int nm = (c->qr_npan + 1) / 2;
  for (int q = 0; q < nm; ++q) {
    pt.start[q] = c->qr_panel_start[2 * q];
    pt.width[q] = c->qr_panel_width[2 * q] + (2 * q + 1 < c->qr_npan ? c->qr_panel_width[2 * q + 1] : 0);
  }
  // 16 waves per stripe: at these sizes there are fewer stripes than CUs,
  // and each reflector's row loop is on the critical path of its stripe
  constexpr int SW = 16, NT = 1024;
  const int e0 = prof_mark(c);
  hipLaunchKernelGGL((k_apply_wy_all<SW, NT>), dim3((ncols + SW - 1) / SW, 1, c->nch), dim3(NT), 0, c->stream,
                     C, ld, n, ncols, c->Vq, ld, c->Tm, pt, nm, backward ? 1 : 0, c->zs);
  prof_pair(c, PH_GEMM, e0, prof_mark(c));
  return KDQMC_OK;
}

// Merges consecutive panel pairs of the last QR (k_merge_t).
int launch_merge_t(kdqmc_ctx* c, int n) {
  PanelTable pt;
  for (int p = 0; p < c->qr_npan; ++p) {
    pt.start[p] = c->qr_panel_start[p];
    pt.width[p] = c->qr_panel_width[p];
  }
  const int e0 = prof_mark(c);
  hipLaunchKernelGGL(k_merge_t, dim3((c->qr_npan + 1) / 2, 1, c->nch), dim3(1024), 0, c->stream, c->Vq, c->N, n,
                     c->Tq, pt, c->qr_npan, c->Tm, c->zs);
  prof_pair(c, PH_GEMM, e0, prof_mark(c));
  return KDQMC_OK;
}

// A (n rows x ncol columns, ncol <= n, leading dimension N) = Q R.  With
// Q != nullptr, the first ncol columns of Q are formed explicitly (n x ncol);
// the panels' V and T stay in Vq / Tq for apply_qt_f64.
int qr_f64(kdqmc_ctx* c, int n, int ncol, double* A, double* Q) {
  const int ld = c->N;
  if (n > 2048) return set_error(KDQMC_EUNSUPPORTED, "QR order above 2048");
  if (ncol < 1 || ncol > n) return set_error(KDQMC_EINVAL, "QR: need 1 <= columns <= rows");
  const size_t nn = (size_t)n * ld;
  hipLaunchKernelGGL(k_zero, dim3((nn + 255) / 256, 1, c->nch), dim3(256), 0, c->stream, c->Vq, nn, c->zs);
  // the first panel alone; then per panel one step launch (the previous
  // panel's update of the next panel's columns, that panel's factorization,
  // and concurrently the previous panel's update of the columns beyond) while
  // the next panel has at most 512 rows, else the update (split over the chip
  // for taller panels, which is faster there than one workgroup per stripe)
  // and the panel apart
  if (c->nch >= kQrChainMin && n <= 2048) {
    // one workgroup per chain for the whole factorization
    PanelTable pt;
    int npan = 0;
    for (int j = 0; j < ncol; ++npan) {
      const int nbp = std::min(panel_width(n - j), ncol - j);
      pt.start[npan] = c->qr_panel_start[npan] = j;
      pt.width[npan] = c->qr_panel_width[npan] = nbp;
      j += nbp;
    }
    c->qr_npan = npan;
    const int e0 = prof_mark(c);
    if (n <= 512)
      hipLaunchKernelGGL((k_qr_chain<1>), dim3(1, 1, c->nch), dim3(512), 0, c->stream, A, ld, n, ncol, c->Vq,
                         c->Tq, c->tau, pt, npan, c->zs);
    else if (n <= 1024)
      hipLaunchKernelGGL((k_qr_chain<2>), dim3(1, 1, c->nch), dim3(512), 0, c->stream, A, ld, n, ncol, c->Vq,
                         c->Tq, c->tau, pt, npan, c->zs);
    else
      hipLaunchKernelGGL((k_qr_chain<4>), dim3(1, 1, c->nch), dim3(512), 0, c->stream, A, ld, n, ncol, c->Vq,
                         c->Tq, c->tau, pt, npan, c->zs);
    prof_pair(c, PH_QR_PANEL, e0, prof_mark(c));
    KDQMC_TRY(launch_merge_t(c, n));
    if (Q) {
      hipLaunchKernelGGL(k_set_identity, dim3((n * ncol + 255) / 256, 1, c->nch), dim3(256), 0, c->stream, Q, n,
                         ncol, ld, c->zs);
      KDQMC_TRY(launch_apply_all(c, Q, ld, n, ncol, true));
    }
    KDQMC_HIP(hipGetLastError());
    return KDQMC_OK;
  }
  int npan = 0, j = 0;
  int nbp = std::min(panel_width(n), ncol);
  KDQMC_TRY(launch_panel(c, A, ld, n, 0, nbp, c->Tq));
  for (;;) {
    c->qr_panel_start[npan] = j;
    c->qr_panel_width[npan] = nbp;
    const int jn = j + nbp;
    if (jn >= ncol) {
      ++npan;
      break;
    }
    const int nbn = std::min(panel_width(n - jn), ncol - jn);
    double* Tp = c->Tq + (size_t)npan * kNBmax * kNBmax;
    double* Tn = Tp + kNBmax * kNBmax;
    const int mn = n - jn;
    if (mn <= 512) {  // (the apply inside covers at most mn + 16 <= 528 rows)
      const dim3 grid(1 + (ncol - jn - nbn + 15) / 16, 1, c->nch);
      const int e0 = prof_mark(c);
      hipLaunchKernelGGL((k_qr_step<2, 16, 256>), grid, dim3(512), 0, c->stream, A, ld, n, ncol, j, nbp, Tp, jn,
                         nbn, c->Vq, Tn, c->tau, c->zs);
      prof_pair(c, PH_QR_PANEL, e0, prof_mark(c));
    } else {
      KDQMC_TRY(launch_apply(c, A, ld, n, j, nbp, jn, ncol, Tp, true));
      KDQMC_TRY(launch_panel(c, A, ld, n, jn, nbn, Tn));
    }
    ++npan;
    j = jn;
    nbp = nbn;
  }
  c->qr_npan = npan;
  KDQMC_TRY(launch_merge_t(c, n));
  if (Q) {
    hipLaunchKernelGGL(k_set_identity, dim3((n * ncol + 255) / 256, 1, c->nch), dim3(256), 0, c->stream, Q, n,
                       ncol, ld, c->zs);
    KDQMC_TRY(launch_apply_all(c, Q, ld, n, ncol, true));
  }
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

// X <- Q^T X for the Q of the last qr_f64 call (X: n rows x ncols, ld = N).
int apply_qt_f64(kdqmc_ctx* c, int n, int ncols, double* X) {
  KDQMC_TRY(launch_apply_all(c, X, c->N, n, ncols, false));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

// ---------------------------------------------------------------------------
// Upper-triangular solve R Y = X in place on X (n x n, ld = N).  Columns of
// X are independent: one workgroup owns 16 columns and walks the 32-row
// block rows from the bottom, X_b = R_bb^{-1} (X_b - R[b, b1:] X[b1:]), with
// the 32 x 32 diagonal-block inverses precomputed by k_trinv_blocks.
// ---------------------------------------------------------------------------
constexpr int kTB = 32;

__global__ void k_trinv_blocks(const double* __restrict__ R, int n, int ld, double* __restrict__ Rinv,
                               size_t zs) {
  __shared__ double Rb[kTB][kTB + 1];
  R = zw(R, zs);
  Rinv = zw(Rinv, zs);
  const int b = blockIdx.x;
  const int b0 = b * kTB;
  const int nbp = min(kTB, n - b0);
  for (int idx = threadIdx.x; idx < kTB * kTB; idx += blockDim.x) {
    const int r = idx / kTB, cc = idx % kTB;
    Rb[r][cc] = (r < nbp && cc < nbp) ? R[(size_t)(b0 + r) * ld + b0 + cc] : 0.0;
  }
  __syncthreads();
  const int col = threadIdx.x;
  if (col < kTB) {
    double x[kTB];
#pragma unroll
    for (int r = kTB - 1; r >= 0; --r) {
      double s = (r == col) ? 1.0 : 0.0;
#pragma unroll
      for (int t = r + 1; t < kTB; ++t) s -= Rb[r][t] * x[t];
      x[r] = (r < nbp) ? s / Rb[r][r] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < kTB; ++r) Rinv[(size_t)b * kTB * kTB + r * kTB + col] = x[r];
  }
}

// One workgroup per 16-column stripe of X; for each 32-row block row from the
// bottom: acc = R[b, b1:] X[b1:, stripe] on the FP64 MFMA (8 waves split K,
// clamped unconditional loads, partials summed in LDS), then
// X_b = Rinv_bb (X_b - acc).
__global__ void __launch_bounds__(512)
k_trsm_upper(const double* __restrict__ R, const double* __restrict__ Rinv, double* __restrict__ X,
             int n, int ncols, int ld, size_t zs) {
  constexpr int NW = 8;
  __shared__ double Wp[NW][32][17];
  __shared__ double Rb[32][33];
  R = zw(R, zs);
  Rinv = zw(Rinv, zs);
  X = zw(X, zs);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int s0 = blockIdx.x * 16;
  const int nblk = (n + kTB - 1) / kTB;
  const int xc = std::min(s0 + lr, ncols - 1);  // this lane's column of X (clamped)
  for (int b = nblk - 1; b >= 0; --b) {
    const int b0 = b * kTB;
    const int b1 = min(n, b0 + kTB);
    v4d acc[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) acc[bi] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int k0 = b1 + wave * 4; k0 < n; k0 += 4 * NW) {
      const int k = k0 + lk;
      const int kc = std::min(k, n - 1);
      double av[2];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int r = b0 + bi * 16 + lr;
        const double v = R[(size_t)std::min(r, n - 1) * ld + kc];
        av[bi] = (r < n && k < n) ? v : 0.0;
      }
      const double xv = X[(size_t)kc * ld + xc];
      const double bv = (k < n && s0 + lr < ncols) ? xv : 0.0;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) acc[bi] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], bv, acc[bi], 0, 0, 0);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int e = 0; e < 4; ++e) Wp[wave][bi * 16 + lk + 4 * e][lr] = acc[bi][e];
    for (int idx = tid; idx < 32 * 32; idx += 512) {
      const int r = idx >> 5, cc = idx & 31;
      Rb[r][cc] = Rinv[(size_t)b * kTB * kTB + r * kTB + cc];
    }
    __syncthreads();
    const int r = tid >> 4, cc = tid & 15;  // 32 x 16: one element per thread
    const int gr = b0 + r, gc = s0 + cc;
    {
      const double xv = (gr < n && gc < ncols) ? X[(size_t)gr * ld + gc] : 0.0;
      double sacc = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) sacc += Wp[w][r][cc];
      Wp[0][r][cc] = xv - sacc;  // (the element only this thread reads)
    }
    __syncthreads();
    double y = 0.0;
#pragma unroll 8
    for (int t = 0; t < 32; ++t) y += Rb[r][t] * Wp[0][t][cc];
    if (gr < n && gc < ncols) X[(size_t)gr * ld + gc] = y;
    __syncthreads();
  }
}

int trsm_upper_f64(kdqmc_ctx* c, int n, int ncols, const double* R, double* X) {
  const int ld = c->N;
  const int nblk = (n + kTB - 1) / kTB;
  double* Rinv = c->Tq;  // nblk * 32 * 32 (the QR's T factors are no longer needed)
  const int e0 = prof_mark(c);
  hipLaunchKernelGGL(k_trinv_blocks, dim3(nblk, 1, c->nch), dim3(64), 0, c->stream, R, n, ld, Rinv, c->zs);
  hipLaunchKernelGGL(k_trsm_upper, dim3((ncols + 15) / 16, 1, c->nch), dim3(512), 0, c->stream, R, Rinv, X, n,
                     ncols, ld, c->zs);
  prof_pair(c, PH_GEMM, e0, prof_mark(c));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

}  // namespace kdqmc
