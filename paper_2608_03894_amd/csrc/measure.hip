// Equal-time estimators of one configuration from its G (Secs. IV-V of the
// paper: the pairing structure factor S_Pair(Q) in its symmetric form, and
// the CDW field phi(Q) with the three-sublattice phase), by Wick's theorem
// with G_ab = <c_a c_b^+> for either spin:
//   S_Pair(Q) = (1/N) sum_ab e^{iQ.(r_b - r_a)} [(delta_ab - G_ab)^2 + G_ab^2]
//   D(Q)^2   = (1/N^2) [4 |sum_a c_a (1 - G_aa)|^2
//                       + 2 sum_ab conj(c_a) c_b (delta_ab - G_ba) G_ab],
//   c_a = e^{iQ.R_a} (1, w, w^2)_{s_a}, w = e^{2 pi i/3}, R_a the cell of a.
// One read of G: every 64 x 64 tile is combined with its transposed partner
// (G_ba), each workgroup writes five partial sums, and a one-workgroup pass
// adds them in a fixed order (the result does not depend on scheduling).
#include <cmath>
#include <vector>

#include "common.h"

namespace kdqmc {

namespace {

constexpr int kTile = 64;
constexpr int kParts = 5;  // S(Gamma), Re S(dk1), Re S(dk2), exchange sums at Gamma and K

// Per-site table: p_dk1 (re, im), p_dk2 (re, im), c_Gamma (re, im), c_K (re, im).
template <typename T>
__global__ void __launch_bounds__(256)
k_measure_tiles(const T* __restrict__ G, int N, const double* __restrict__ tab, double* __restrict__ part,
                size_t zs) {
  G = zw(G, zs);
  tab = zw(tab, zs);
  part = zw(part, zs);
  __shared__ double Gt[kTile][kTile + 1];  // G[J rows][I cols], read as G_ba
  __shared__ double ta[kTile][8], tb[kTile][8];
  __shared__ double red[4][kParts];
  const int gt = (N + kTile - 1) / kTile;
  const int I = blockIdx.x / gt, J = blockIdx.x % gt;  // rows a in tile I, columns b in tile J
  const int a0 = I * kTile, b0 = J * kTile;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kTile * kTile; idx += 256) {
    const int r = idx / kTile, c = idx % kTile;  // element (b0 + r, a0 + c)
    const int gb = min(b0 + r, N - 1), ga = min(a0 + c, N - 1);
    Gt[r][c] = double(G[(size_t)gb * N + ga]);
  }
  for (int idx = tid; idx < kTile * 8; idx += 256) {
    const int r = idx / 8, k = idx % 8;
    ta[r][k] = tab[(size_t)min(a0 + r, N - 1) * 8 + k];
    tb[r][k] = tab[(size_t)min(b0 + r, N - 1) * 8 + k];
  }
  __syncthreads();
  double acc[kParts] = {0.0, 0.0, 0.0, 0.0, 0.0};
  // thread: column b = b0 + (tid & 63), rows a = a0 + (tid >> 6) + 4 q
  const int cb = tid & 63, rq = tid >> 6;
  const int b = b0 + cb;
  if (b < N) {
    const double p1r = tb[cb][0], p1i = tb[cb][1], p2r = tb[cb][2], p2i = tb[cb][3];
    const double cgr = tb[cb][4], cgi = tb[cb][5], ckr = tb[cb][6], cki = tb[cb][7];
    for (int q = 0; q < kTile / 4; ++q) {
      const int ra = rq + 4 * q;
      const int a = a0 + ra;
      if (a >= N) break;
      const double gab = double(G[(size_t)a * N + b]);
      const double gba = Gt[cb][ra];
      const double d = (a == b) ? 1.0 : 0.0;
      const double f = (d - gab) * (d - gab) + gab * gab;
      const double e = (d - gba) * gab;
      acc[0] += f;
      acc[1] += f * (p1r * ta[ra][0] + p1i * ta[ra][1]);  // Re(p_b conj(p_a))
      acc[2] += f * (p2r * ta[ra][2] + p2i * ta[ra][3]);
      acc[3] += e * (cgr * ta[ra][4] + cgi * ta[ra][5]);  // Re(conj(c_a) c_b)
      acc[4] += e * (ckr * ta[ra][6] + cki * ta[ra][7]);
    }
  }
  // fixed-order reduction: lanes by DPP-free shuffles, then the four waves
  for (int k = 0; k < kParts; ++k) {
    double v = acc[k];
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if ((tid & 63) == 0) red[tid >> 6][k] = v;
  }
  __syncthreads();
  if (tid < kParts) part[(size_t)blockIdx.x * kParts + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
}

// Sums the tiles' partials in tile order and the diagonal terms, and writes
// the six estimators to the chain's record (zo bytes between records).
template <typename T>
__global__ void __launch_bounds__(256)
k_measure_final(const T* __restrict__ G, int N, const double* __restrict__ tab, const double* __restrict__ part,
                int ntiles, double* __restrict__ out, size_t zs, size_t zo) {
  G = zw(G, zs);
  tab = zw(tab, zs);
  part = zw(part, zs);
  out = zw(out, zo);
  __shared__ double red[4][kParts + 5];
  const int tid = threadIdx.x;
  double acc[kParts + 5];
  for (int k = 0; k < kParts + 5; ++k) acc[k] = 0.0;
  for (int t = tid; t < ntiles; t += 256)
    for (int k = 0; k < kParts; ++k) acc[k] += part[(size_t)t * kParts + k];
  // diagonal: sum_a c_a n_a (Gamma, K; re and im) and sum_a n_a, n_a = 1 - G_aa
  for (int a = tid; a < N; a += 256) {
    const double na = 1.0 - double(G[(size_t)a * N + a]);
    acc[kParts + 0] += tab[(size_t)a * 8 + 4] * na;
    acc[kParts + 1] += tab[(size_t)a * 8 + 5] * na;
    acc[kParts + 2] += tab[(size_t)a * 8 + 6] * na;
    acc[kParts + 3] += tab[(size_t)a * 8 + 7] * na;
    acc[kParts + 4] += na;
  }
  for (int k = 0; k < kParts + 5; ++k) {
    double v = acc[k];
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    if ((tid & 63) == 0) red[tid >> 6][k] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double s[kParts + 5];
    for (int k = 0; k < kParts + 5; ++k) s[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
    const double n = double(N);
    out[KDQMC_OBS_SPAIR_GAMMA] = s[0] / n;
    out[KDQMC_OBS_SPAIR_DK1] = s[1] / n;
    out[KDQMC_OBS_SPAIR_DK2] = s[2] / n;
    out[KDQMC_OBS_CDW2_GAMMA] = (4.0 * (s[5] * s[5] + s[6] * s[6]) + 2.0 * s[3]) / (n * n);
    out[KDQMC_OBS_CDW2_K] = (4.0 * (s[7] * s[7] + s[8] * s[8]) + 2.0 * s[4]) / (n * n);
    out[KDQMC_OBS_DENSITY] = 2.0 * s[9] / n;
  }
}

}  // namespace

// The per-site table of the estimators' phases (host, written into tab[N*8]):
// sites sit at (x1 + f1_s) a1 + (x2 + f2_s) a2 with f = (0, 0), (0, -1/2),
// (-1/2, 0) for A, B, C (so that every bond of Eq. (3) has the same length
// on the 60-degree lattice); dk1, dk2 = 2 pi/L b1, 2 pi/L b2; K = the Dirac
// point (2 pi/3, -2 pi/3) of the cell coordinates.
void measure_table(int L, double* tab) {
  const double f1[3] = {0.0, 0.0, -0.5}, f2[3] = {0.0, -0.5, 0.0};
  for (int x1 = 0; x1 < L; ++x1)
    for (int x2 = 0; x2 < L; ++x2)
      for (int s = 0; s < 3; ++s) {
        double* t = tab + (size_t)((x1 * L + x2) * 3 + s) * 8;
        const double X1 = x1 + f1[s], X2 = x2 + f2[s];
        const double ph1 = 2.0 * kPi * X1 / L, ph2 = 2.0 * kPi * X2 / L;
        const double w = 2.0 * kPi * s / 3.0;                       // (1, w, w^2)
        const double k = 2.0 * kPi * (double(x1) + 2.0 * x2) / 3.0;  // K . R
        t[0] = std::cos(ph1);
        t[1] = std::sin(ph1);
        t[2] = std::cos(ph2);
        t[3] = std::sin(ph2);
        t[4] = std::cos(w);
        t[5] = std::sin(w);
        t[6] = std::cos(k + w);
        t[7] = std::sin(k + w);
      }
}

int launch_measure(kdqmc_ctx* c, double* out, size_t zn) {
  const int N = c->N;
  const int gt = (N + kTile - 1) / kTile;
  const int ntiles = gt * gt;
  double* part = c->S[7];  // ntiles * kParts <= N * N
  const size_t zo = zn * sizeof(double);
  const int e0 = prof_mark(c);
  if (c->fp64) {
    hipLaunchKernelGGL(k_measure_tiles<double>, dim3(ntiles, 1, c->nch), dim3(256), 0, c->stream,
                       (const double*)c->G, N, c->obs_tab, part, c->zs);
    hipLaunchKernelGGL(k_measure_final<double>, dim3(1, 1, c->nch), dim3(256), 0, c->stream,
                       (const double*)c->G, N, c->obs_tab, part, ntiles, out, c->zs, zo);
  } else {
    hipLaunchKernelGGL(k_measure_tiles<float>, dim3(ntiles, 1, c->nch), dim3(256), 0, c->stream,
                       (const float*)c->G, N, c->obs_tab, part, c->zs);
    hipLaunchKernelGGL(k_measure_final<float>, dim3(1, 1, c->nch), dim3(256), 0, c->stream,
                       (const float*)c->G, N, c->obs_tab, part, ntiles, out, c->zs, zo);
  }
  prof_pair(c, PH_MEASURE, e0, prof_mark(c));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

}  // namespace kdqmc
