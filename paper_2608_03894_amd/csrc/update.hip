// Delayed Ising-field updates of one time slice (the delay-update algorithm
// cited in Sec. II of the paper), organised for one GPU:
//
//   * sites are visited in order in windows S of w consecutive sites;
//   * k_decide (one workgroup) holds G~cur[S,S] in LDS and runs the
//     sequential Metropolis tests of the window; each accepted flip updates
//     the window submatrix by a rank-one Sherman-Morrison step, and two small
//     triangular factors Z, Z' are grown so that the window's accepted flips
//     together add  G~cur[:,A] Z Z' (I - G~cur)[A,:]  to G~ (A = accepted
//     sites of the window);
//   * k_extend turns that into a := |A| new columns of the pending factors
//     U (N x k) and W (k x N), G~cur = G~ + U W;
//   * k_flush adds U W to G as one rank-(<= delay_k) MFMA product once the
//     pending rank could exceed delay_k, and at the end of the slice.
//
// Frames: G holds D^{-1} G~ D with D = diag(exp(alpha s_l)) taken from the
// fields at the start of the slice (ev, evinv); the pending factors are
// stored in the same frame (U_store = D^{-1} U, W_store = W D), so the flush
// is a plain G += U_store W_store and the column pass of the wrap applies D.
#include "common.h"

namespace kdqmc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// ev = exp(alpha s), evinv = exp(-alpha s) for the fields of one slice.
__global__ void k_frame_scale(const int8_t* __restrict__ s, int n, const double* __restrict__ sc,
                              double* __restrict__ ev, double* __restrict__ evinv, size_t zs) {
  s = zw(s, zs);
  ev = zw(ev, zs);
  evinv = zw(evinv, zs);
  const double ea = zw(sc, zs)[SC_EA], eainv = zw(sc, zs)[SC_EAINV];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const bool up = s[i] > 0;
    ev[i] = up ? ea : eainv;
    evinv[i] = up ? eainv : ea;
  }
}

// Downward pass: G <- F G F^{-1}, F_i = exp(alpha s_old,i) exp(-alpha s_new,i)
// (1 where the site was not flipped), element by element.
template <typename T>
__global__ void k_down_reframe(T* __restrict__ G, int n, const double* __restrict__ ev,
                               const double* __restrict__ evinv, const int8_t* __restrict__ s,
                               const double* __restrict__ sc, size_t zs) {
  G = zw(G, zs);
  ev = zw(ev, zs);
  evinv = zw(evinv, zs);
  s = zw(s, zs);
  const double ea = zw(sc, zs)[SC_EA], eainv = zw(sc, zs)[SC_EAINV];
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)n * n) {
    const int r = (int)(idx / n), cc = (int)(idx % n);
    const double fr = ev[r] * (s[r] > 0 ? eainv : ea);
    const double fci = evinv[cc] * (s[cc] > 0 ? ea : eainv);
    if (fr != 1.0 || fci != 1.0) G[idx] = T(double(G[idx]) * fr * fci);
  }
}

// ---------------------------------------------------------------------------
// Sequential decisions of one window (single workgroup of 256 threads).
// Three wn x wn blocks are kept: the window submatrix Gs (tilde frame) and two
// coefficient blocks Cf, Cr.  After the accepts so far,
//   G~cur[:, y] = G0[:, y] + sum_q G0[:, i_q] Cf[q][y]   (columns y of the window)
//   G~cur[x, :] = G0[x, :] + sum_q Cr[x][q] h_q           (rows x of the window)
// with G0 the window-start matrix and h_q = e_{i_q} - G0[i_q, :].  The accept
// number n at window position p (c = Delta/R) therefore has the factors
//   u_n = sum_q G0[:, i_q] Z[q][n],  Z[q][n] = -c (delta_qn + Cf[q][p]),
//   w_n = sum_q Z'[n][q] h_q,        Z'[n][q] = delta_nq - Cr[p][q],
// and Gs, Cf, Cr receive rank-one updates on their live part (indices > p);
// row p and column p of all three are never written again.
// Register layout: the NT threads form a GR x GR grid (GR = 8 for one wave,
// 16 for four); thread t owns the WS x WS entries (x, y) with
// x = t/GR + GR i, y = t%GR + GR k of each block.  Per accept the owners
// publish row p / column p through LDS (one barrier), everyone updates its
// registers and the diagonal owners publish the new diagonal for the
// decisions after the next accept.  A decision reads three LDS words (the
// diagonal entry and the latest accept's row/column entries) and needs no
// barrier.  Four waves are used
// for every window size: the per-accept updates are VALU bound and spread
// better over four SIMDs than the barriers cost.
// ---------------------------------------------------------------------------
template <typename T, int WS, int NT>
__global__ void __launch_bounds__(NT)
k_decide(const T* __restrict__ G, int N, const double* __restrict__ ev,
         const double* __restrict__ evinv, int8_t* __restrict__ s_l,
         const double* __restrict__ u, const uint8_t* __restrict__ forced,
         uint8_t* __restrict__ acc_out, double* __restrict__ ratio_out, int w0, int wn, int W,
         const double* __restrict__ Gs_in, const double* __restrict__ sc, int win,
         int* __restrict__ win_a, int* __restrict__ win_p, double* __restrict__ Zg,
         double* __restrict__ Zpg, size_t zs, size_t zn) {
  constexpr int GR = (NT == 64) ? 8 : 16;
  G = zw(G, zs);
  ev = zw(ev, zs);
  evinv = zw(evinv, zs);
  s_l = zw(s_l, zs);
  u = zc(u, zn);
  forced = zc(forced, zn);
  acc_out = zc(acc_out, zn);
  ratio_out = zc(ratio_out, zn);
  Gs_in = zw(Gs_in, zs);
  win_a = zw(win_a, zs);
  win_p = zw(win_p, zs);
  Zg = zw(Zg, zs);
  Zpg = zw(Zpg, zs);
  const double em2a = zw(sc, zs)[SC_EM2A], ep2a = zw(sc, zs)[SC_EP2A];
  constexpr int WM = GR * WS;  // largest window this instance handles
  // Everything the loop produces stays in LDS until the end: a barrier also
  // waits for outstanding global stores, so none are issued inside the loop.
  // The published row / column of the latest accept and the diagonal of G~cur
  // are double-buffered by accept parity, so one barrier per accept suffices:
  // buffer n & 1 is written by accept n before its barrier and read until the
  // barrier of accept n + 1, after which nobody reads it before accept n + 2
  // overwrites it.  diagB[k & 1] holds the diagonal after k accepts (entries
  // past the k-th accepted site); a decision after accept n adds accept n's
  // rank-one term to diagB[n & 1] itself, exactly as the owners do.
  __shared__ double rowp[2][WM], colp[2][WM], cfp[2][WM], crp[2][WM], diagB[2][WM];
  __shared__ double ul[WM], rl[WM];
  __shared__ double Zs[WM][WM + 1], Zps[WM][WM + 1];
  __shared__ int pl[WM], posq[WM];
  __shared__ int8_t sl[WM];
  __shared__ uint8_t fl[WM], al[WM];
  const int tid = threadIdx.x;
  const int rx = tid / GR, cy = tid % GR;
  double gs[WS][WS], cf[WS][WS], cr[WS][WS];
#pragma unroll
  for (int i = 0; i < WS; ++i)
#pragma unroll
    for (int k = 0; k < WS; ++k) {
      const int x = rx + GR * i, y = cy + GR * k;
      double g = 0.0;
      if (x < wn && y < wn) {
        if (Gs_in) {
          g = Gs_in[x * W + y];
        } else {
          const int gx = w0 + x, gy = w0 + y;
          g = double(G[(size_t)gx * N + gy]) * ev[gx] * evinv[gy];
        }
      }
      gs[i][k] = g;
      cf[i][k] = 0.0;
      cr[i][k] = 0.0;
      if (x == y && x < wn) diagB[0][x] = g;
    }
  for (int p = tid; p < wn; p += NT) {
    sl[p] = s_l[w0 + p];
    ul[p] = u ? u[w0 + p] : 0.0;
    fl[p] = forced ? forced[w0 + p] : 0;
  }
  __syncthreads();

  // A rejected proposal leaves G~cur unchanged, so every proposal between two
  // accepts sees the same matrix: lane x of each wave tests site x of the
  // window against the state after the latest accept, and the lowest
  // accepting site past the previous accept (a ballot) is the next accept;
  // the sites before it are rejections with exactly the ratios the one by one
  // scan computes.  Every wave evaluates the same tests, so all agree on the
  // accept without a barrier.
  const int lane = tid & 63;
  const bool xin = lane < wn;
  const int sx = xin ? sl[lane] : 1;
  const double ux = xin ? ul[lane] : 0.0;
  const bool fx = xin && fl[lane] != 0;
  const double delta_x = (sx > 0 ? em2a : ep2a) - 1.0;
  const double e2as_x = sx > 0 ? ep2a : em2a;
  int na = 0;
  int p0 = 0;           // first site not yet decided
  double c_last = 0.0;  // c of the latest accept (the same in every thread)
  while (p0 < wn) {
    double gxx;
    if (na == 0) {
      gxx = xin ? diagB[0][lane] : 0.0;
    } else {
      const int bl = (na - 1) & 1;
      gxx = xin ? fma(c_last * colp[bl][lane], rowp[bl][lane], diagB[bl][lane]) : 0.0;
    }
    const double Rx = 1.0 + delta_x * (1.0 - gxx);
    const double ratio_x = e2as_x * Rx * Rx;
    const bool ax = forced ? fx : (ux < ratio_x);
    const unsigned long long hits = __ballot(xin && lane >= p0 && ax);
    const int p = hits ? __builtin_ctzll(hits) : wn;
    if (tid < 64 && lane >= p0 && lane <= p && xin) {
      rl[lane] = ratio_x;
      al[lane] = lane == p ? 1 : 0;
    }
    if (p >= wn) break;
    p0 = p + 1;
    const double R = lane_value(Rx, p);
    const double delta = lane_value(delta_x, p);
    const double c = delta * rcp_nr(R);
    const int n = na;
    const int b = n & 1;
    const int ip = p / GR, pr = p % GR;
    // phase A: publish row p of Gs and Cr, column p of Gs and Cf
    if (rx == pr) {
#pragma unroll
      for (int k = 0; k < WS; ++k) {
        double g = 0.0, r = 0.0;
#pragma unroll
        for (int i = 0; i < WS; ++i)
          if (i == ip) {
            g = gs[i][k];
            r = cr[i][k];
          }
        rowp[b][cy + GR * k] = g;
        crp[b][cy + GR * k] = r;
      }
    }
    if (cy == pr) {
#pragma unroll
      for (int i = 0; i < WS; ++i) {
        double g = 0.0, f = 0.0;
#pragma unroll
        for (int k = 0; k < WS; ++k)
          if (k == ip) {
            g = gs[i][k];
            f = cf[i][k];
          }
        colp[b][rx + GR * i] = g;
        cfp[b][rx + GR * i] = f;
      }
    }
    if (tid == 0) pl[n] = p;
    __syncthreads();
    // phase B: rank-one updates of the live parts; publish the accept's factors
    double cx[WS], qx[WS], ry[WS], zpy[WS];
#pragma unroll
    for (int i = 0; i < WS; ++i) {
      const int x = rx + GR * i;
      cx[i] = colp[b][x];
      qx[i] = -c * ((x == n ? 1.0 : 0.0) + cfp[b][x]);   // Z[x][n] (rows q = x of Cf)
    }
#pragma unroll
    for (int k = 0; k < WS; ++k) {
      const int y = cy + GR * k;
      ry[k] = rowp[b][y];
      zpy[k] = (y == n ? 1.0 : 0.0) - crp[b][y];        // Z'[n][y] (columns q = y of Cr)
    }
#pragma unroll
    for (int i = 0; i < WS; ++i)
#pragma unroll
      for (int k = 0; k < WS; ++k) {
        const int x = rx + GR * i, y = cy + GR * k;
        if (x > p && y > p) gs[i][k] = fma(c * cx[i], ry[k], gs[i][k]);
        if (x <= n && y > p) cf[i][k] -= qx[i] * ry[k];
        if (x > p && y <= n) cr[i][k] -= c * cx[i] * zpy[k];
      }
    if (tid <= n) {
      Zs[tid][n] = -c * ((tid == n ? 1.0 : 0.0) + cfp[b][tid]);
      Zps[n][tid] = (tid == n ? 1.0 : 0.0) - crp[b][tid];
    }
    if (rx == cy) {
#pragma unroll
      for (int i = 0; i < WS; ++i) {
        const int x = rx + GR * i;
        if (x > p && x < wn) diagB[b ^ 1][x] = gs[i][i];
      }
    }
    c_last = c;
    ++na;
  }
  __syncthreads();
  if (tid == 0) win_a[win] = na;
  for (int n = tid; n < na; n += NT) win_p[win * W + n] = pl[n];
  for (int p = tid; p < wn; p += NT) {
    s_l[w0 + p] = al[p] ? int8_t(-sl[p]) : sl[p];   // the loop never writes sl: other waves read it
    if (ratio_out) ratio_out[w0 + p] = rl[p];
    if (acc_out) acc_out[w0 + p] = al[p];
  }
  // Z and Z' by window position, n-major with stride WM and the frame scales
  // folded in (as written by decide_window):
  //   Zh[n][p] = evinv[w0+p] Z[q_p][n],  Zph[n][p] = ev[w0+p] Z'[n][q_p]
  for (int p = tid; p < WM; p += NT) posq[p] = -1;
  __syncthreads();
  for (int n = tid; n < na; n += NT) posq[pl[n]] = n;
  __syncthreads();
  for (int idx = tid; idx < WM * WM; idx += NT) {
    const int n = idx / WM, p = idx % WM;
    const int q = posq[p];
    const bool live = q >= 0 && q <= n && n < na;
    const int pc = w0 + min(p, wn - 1);
    Zg[idx] = live ? Zs[q][n] * evinv[pc] : 0.0;
    Zpg[idx] = live ? Zps[n][q] * ev[pc] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Sequential decisions of one window of at most 32 sites in a single wave
// (no barriers).  Accept n at site p adds u_n w_n^T to the window, with
//   u_n = -c G~cur[:, p] = -c (G0[:, p] + sum_{r<n} u_r w_r[p]),
//   w_n = e_p - G~cur[p, :] = e_p - G0[p, :] - sum_{r<n} u_r[p] w_r,
// so lane x (site x of the window) rebuilds column and row p from G0 (LDS)
// and the factors of the earlier accepts (its own in registers, lane p's
// read back from LDS), and keeps only its own diagonal entry current.  Rejections leave G~cur
// unchanged: all sites past the latest accept are tested at once against
// that state and a ballot names the next accept (the sites before it are
// rejections with the ratios a one-by-one scan computes).  Lanes 32 + q run
// the same recursion for the coefficient row q of Z and column q of Z'
// (u_n = sum_q G0[:, i_q] Z[q][n], w_n = sum_q Z'[n][q] h_q with
// h_q = e_{i_q} - G0[i_q, :]):
//   Z[q][n]  = -c (delta_qn + sum_{r<n} Z[q][r] w_r[p]),
//   Z'[n][q] = delta_nq - sum_{r<n} u_r[p] Z'[r][q],
// with the same remote values w_r[p], u_r[p] as the sites use.
// ---------------------------------------------------------------------------
// The decisions of one window whose submatrix G0 (tilde frame, zero outside
// wn x wn) is in g0s, run by the calling wave alone.  sx, ux, fx: field,
// uniform and forced flag of site `lane` (lanes < wn).  Writes the flipped
// fields, the accept flags and ratios, win_a[win], win_p and Z, Z'.
template <int WM>
__device__ __forceinline__ void decide_window(int lane, int wn, int w0, int W, int win,
                                              double (*g0s)[WM + 1], double2 (*hist)[64], int sx,
                                              double ux, bool fx, bool use_forced, double em2a,
                                              double ep2a,
                                              int8_t* __restrict__ s_l, uint8_t* __restrict__ acc_out,
                                              double* __restrict__ ratio_out, int* __restrict__ win_a,
                                              int* __restrict__ win_p, double* __restrict__ Zg,
                                              double* __restrict__ Zpg, const double* __restrict__ ev,
                                              const double* __restrict__ evinv) {
  static_assert(WM <= 32, "one wave holds the sites in lanes 0..31 and Z in lanes 32..63");
  const bool site = lane < WM;
  const bool xin = lane < wn;
  const bool zlane = lane >= 32;  // coefficient lanes (q = lane - 32)
  const int q = lane - 32;
  const double delta_x = (sx > 0 ? em2a : ep2a) - 1.0;
  const double e2as_x = sx > 0 ? ep2a : em2a;
  double diag = xin ? g0s[lane][lane] : 0.0;
  // the ratio of site `lane` stays in a register until the end; the accepted
  // positions are a wave-uniform bit mask
  double my_ratio = 0.0;
  unsigned long long accm = 0;
  int na = 0, p0 = 0;
  // per-lane constants: the accept step is branch-free apart from the exit
  // (divergent updates are selects, the window entries read by the
  // coefficient lanes are weighted by 0).  With replayed decisions a forced
  // accept compares -1 < ratio (always true, the ratio being positive) and a
  // forced reject +inf < ratio (always false).
  const double sitef = site ? 1.0 : 0.0;
  const int lx = lane & (WM - 1);
  const double ucmp = use_forced ? (fx ? -1.0 : __builtin_inf()) : ux;
  const unsigned long long live = __ballot(xin);
  // The accept loop is unrolled, so that the accept index n is a
  // compile-time constant: the lane's own factor history (u_r[x], w_r[x])
  // lives in registers hu[r], hw[r]; the rows also go to LDS (hist[r][lane]),
  // from where every lane reads the accepted site's row r < n (one broadcast
  // read per row, all issued together).
  double hu[WM], hw[WM];
#pragma unroll
  for (int n = 0; n < WM; ++n) {
    const double Rx = 1.0 + delta_x * (1.0 - diag);
    double cx = delta_x * rcp_nr(Rx);  // c of every candidate, off the ballot's path
    const double ratio_x = e2as_x * Rx * Rx;
    const unsigned long long hits = __ballot(ucmp < ratio_x) & live & ~((1ull << p0) - 1ull);
    asm volatile("" : "+v"(cx));  // (the division is issued before the branch below)
    const int p = hits ? __builtin_ctzll(hits) : wn;
    // (a site's last update is at its own decision: p0 passes it afterwards)
    my_ratio = (lane >= p0) ? ratio_x : my_ratio;
    if (p >= wn) break;
    p0 = p + 1;
    accm |= 1ull << p;
    const double c = lane_value(cx, p);
    // window entries G0[x][p], G0[p][x], and row r < n of lane p's history
    // (u_r[p], w_r[p]); four partial sums per product
    const double gA = g0s[lx][p], gB = g0s[p][lx];
    double2 rem[WM > 1 ? WM - 1 : 1];
#pragma unroll
    for (int r = 0; r < n; ++r) rem[r] = hist[r][p];
    double A[4] = {0.0, 0.0, 0.0, 0.0}, B[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < n; ++r) {
      A[r & 3] = fma(hu[r], rem[r].y, A[r & 3]);
      B[r & 3] = fma(rem[r].x, hw[r], B[r & 3]);
    }
    const double As = fma(gA, sitef, (!site && q == n) ? 1.0 : 0.0) + ((A[0] + A[1]) + (A[2] + A[3]));
    const double Bs = fma(gB, sitef, (B[0] + B[1]) + (B[2] + B[3]));
    const double Xn = -c * As;
    const double Yn = ((site ? lane == p : q == n) ? 1.0 : 0.0) - Bs;
    hu[n] = Xn;
    hw[n] = Yn;
    hist[n][lane] = make_double2(Xn, Yn);
    diag = fma(Xn * sitef, Yn, diag);
    na = n + 1;
  }
  wave_sync();
  const bool my_acc = xin && ((accm >> lane) & 1ull);
  if (lane == 0) win_a[win] = na;
  if (my_acc) win_p[win * W + __popcll(accm & ((1ull << lane) - 1ull))] = lane;
  if (xin) {
    s_l[w0 + lane] = my_acc ? int8_t(-sx) : int8_t(sx);
    if (ratio_out) ratio_out[w0 + lane] = my_ratio;
    if (acc_out) acc_out[w0 + lane] = my_acc ? 1 : 0;
  }
  // Z and Z' by window position, n-major with stride WM and the frame scales
  // folded in, so that the factors in the store frame of G are
  // U = G[:, S] Zh^T and W = Zph (E_S - G[S, :]):
  //   Zh[n][p] = evinv[w0+p] Z[q_p][n],  Zph[n][p] = ev[w0+p] Z'[n][q_p]
  // with q_p the accept at position p (q_p <= n < na), zero elsewhere
  // (also past the window up to WM).  Lanes 0..31 write Zh, lanes 32..63
  // Zph, the lane's position p = lane % 32.  Every history row is read
  // (qp < 32 always indexes a coefficient lane) and the unused ones are
  // selected away, so the reads and the stores each go out together rather
  // than one branch and round trip per row.
  {
    const int p = lane & 31;
    if (p < WM) {
      const bool acc_p = (accm >> p) & 1ull;
      const int qp = __popcll(accm & ((1ull << p) - 1ull));
      const int pc = w0 + min(p, wn - 1);
      const double f = zlane ? ev[pc] : evinv[pc];
      double* __restrict__ dst = zlane ? Zpg : Zg;
      double2 h[WM];
#pragma unroll
      for (int n = 0; n < WM; ++n) h[n] = hist[n][32 + qp];
      __builtin_amdgcn_sched_barrier(0);  // (all reads issued before the first use)
#pragma unroll
      for (int n = 0; n < WM; ++n)
        dst[n * WM + p] = (acc_p && n >= qp && n < na) ? (zlane ? h[n].y : h[n].x) * f : 0.0;
    }
  }
}

// Field, uniform and forced flag of site `lane` of the window at w0 (loads
// clamped into the window; lanes >= wn get neutral values).
// (absent inputs are read from stand-ins -- any double array `dfl` and the
// field array -- and discarded, so that no branch separates these loads from
// the caller's)
__device__ __forceinline__ void site_inputs(int lane, int w0, int wn, const int8_t* __restrict__ s_l,
                                            const double* __restrict__ u,
                                            const uint8_t* __restrict__ forced,
                                            const double* __restrict__ dfl, int& sx, double& ux,
                                            bool& fx) {
  const int xs = w0 + min(lane, wn - 1);
  const int s_raw = s_l[xs];
  const double* ud = u ? u : dfl;
  const double u_ld = ud[u ? xs : 0];
  const uint8_t* fd = forced ? forced : reinterpret_cast<const uint8_t*>(s_l);
  const uint8_t f_ld = fd[xs];
  const double u_raw = u ? u_ld : 0.0;
  const bool f_raw = forced ? f_ld != 0 : false;
  const bool xin = lane < wn;
  sx = xin ? s_raw : 1;
  ux = xin ? u_raw : 0.0;
  fx = xin && f_raw;
}

// Loads the window submatrix (from G, or from the prepared Gs_in) and runs
// its decisions in the calling wave (64 threads).
template <typename T, int WM>
__device__ __forceinline__ void
decide_wave_body(const T* __restrict__ G, int N, const double* __restrict__ ev,
                 const double* __restrict__ evinv, int8_t* __restrict__ s_l,
                 const double* __restrict__ u, const uint8_t* __restrict__ forced,
                 uint8_t* __restrict__ acc_out, double* __restrict__ ratio_out, int w0, int wn, int W,
                 const double* __restrict__ Gs_in, const double* __restrict__ sc, int win,
                 int* __restrict__ win_a, int* __restrict__ win_p, double* __restrict__ Zg,
                 double* __restrict__ Zpg, size_t zs, size_t zn) {
  G = zw(G, zs);
  ev = zw(ev, zs);
  evinv = zw(evinv, zs);
  s_l = zw(s_l, zs);
  u = zc(u, zn);
  forced = zc(forced, zn);
  acc_out = zc(acc_out, zn);
  ratio_out = zc(ratio_out, zn);
  Gs_in = zw(Gs_in, zs);
  win_a = zw(win_a, zs);
  win_p = zw(win_p, zs);
  Zg = zw(Zg, zs);
  Zpg = zw(Zpg, zs);
  const double em2a = zw(sc, zs)[SC_EM2A], ep2a = zw(sc, zs)[SC_EP2A];
  __shared__ double g0s[WM][WM + 1];
  __shared__ double2 hist[WM][64];  // hist[r][lane]: (u_r[x], w_r[x]) or (Z[q][r], Z'[r][q])
  const int lane = threadIdx.x;
  int sx;
  double ux;
  bool fx;
  site_inputs(lane, w0, wn, s_l, u, forced, ev, sx, ux, fx);
  // window submatrix G0 (tilde frame): all loads issued before any is used
  // (addresses clamped into the window instead of branches)
  constexpr int PER = (WM * WM + 63) / 64;
  double gv[PER];
  if (Gs_in) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int idx = lane + 64 * j;
      const int x = min(idx / WM, wn - 1), y = min(idx % WM, wn - 1);
      gv[j] = Gs_in[x * W + y];
    }
  } else {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int idx = lane + 64 * j;
      const int gx = w0 + min(idx / WM, wn - 1), gy = w0 + min(idx % WM, wn - 1);
      gv[j] = double(G[(size_t)gx * N + gy]) * ev[gx] * evinv[gy];
    }
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int idx = lane + 64 * j;
    const bool ok = idx / WM < wn && idx % WM < wn;
    if (idx < WM * WM) g0s[idx / WM][idx % WM] = ok ? gv[j] : 0.0;
  }
  wave_sync();
  decide_window<WM>(lane, wn, w0, W, win, g0s, hist, sx, ux, fx, forced != nullptr, em2a, ep2a, s_l,
                    acc_out, ratio_out, win_a, win_p, Zg, Zpg, ev, evinv);
}

template <typename T, int WM>
__global__ void __launch_bounds__(64)
k_decide_wave(const T* __restrict__ G, int N, const double* __restrict__ ev,
              const double* __restrict__ evinv, int8_t* __restrict__ s_l,
              const double* __restrict__ u, const uint8_t* __restrict__ forced,
              uint8_t* __restrict__ acc_out, double* __restrict__ ratio_out, int w0, int wn, int W,
              const double* __restrict__ Gs_in, const double* __restrict__ sc, int win,
              int* __restrict__ win_a, int* __restrict__ win_p, double* __restrict__ Zg,
              double* __restrict__ Zpg, size_t zs, size_t zn) {
  decide_wave_body<T, WM>(G, N, ev, evinv, s_l, u, forced, acc_out, ratio_out, w0, wn, W, Gs_in, sc,
                          win, win_a, win_p, Zg, Zpg, zs, zn);
}

// ---------------------------------------------------------------------------
// Fused schedule (FP64, a flush after every window, windows of at most 32
// sites that never straddle a 64 x 64 tile).  Per slice: k_window_start runs
// the decisions of window 0 (workgroup 0) and copies window 0's columns
// G[:, S] and rows G[S, :] into the snapshot buffers (the other workgroups);
// then per window one k_flush_decide:
//   * every 64 x 64 tile (R, C) forms its own rows of the window's new
//     factors, U[R, n] = sum_{q<=n} G~[R, i_q] Z[q][n] and
//     W[n, C] = sum_{q<=n} Z'[n][q] (e_{i_q} - G~[i_q, C]), from the
//     snapshots (other tiles update G[R, S] and G[S, C] in the same launch)
//     in the same arithmetic as k_extend, and adds U W to its tile in the
//     MFMA order of k_flush_f64;
//   * the tiles crossing the next window's columns / rows copy them into the
//     other snapshot buffer;
//   * the tile holding the next window's diagonal block runs that window's
//     decisions on its freshly updated block (one wave), writing Z, Z' to
//     the other coefficient buffer.
// Snapshots and coefficients alternate between two buffers by window parity.
// ---------------------------------------------------------------------------
template <int WM>
__global__ void __launch_bounds__(64)
k_window_start(const double* __restrict__ G, int N, const double* __restrict__ ev,
               const double* __restrict__ evinv, int8_t* __restrict__ s_l,
               const double* __restrict__ u, const uint8_t* __restrict__ forced,
               uint8_t* __restrict__ acc_out, double* __restrict__ ratio_out, int wn, int W,
               const double* __restrict__ sc, int* __restrict__ win_a, int* __restrict__ win_p,
               double* __restrict__ Zg, double* __restrict__ Zpg, double* __restrict__ csn,
               double* __restrict__ rsn, double* __restrict__ bk1, size_t zs, size_t zn) {
  if (blockIdx.x == 0) {
    decide_wave_body<double, WM>(G, N, ev, evinv, s_l, u, forced, acc_out, ratio_out, 0, wn, W,
                                 nullptr, sc, 0, win_a, win_p, Zg, Zpg, zs, zn);
    return;
  }
  G = zw(G, zs);
  csn = zw(csn, zs);
  rsn = zw(rsn, zs);
  bk1 = zw(bk1, zs);
  // column snapshot csn[r][y] = G[r][y] (row stride WM), row snapshot stored
  // transposed, rsn[c][x] = G[x][c] (stride WM), for x, y < wn, and window
  // 1's diagonal block bk1[x][y] = G[W + x][W + y] (x, y < wn1): 8 elements
  // per thread, loads before stores
  constexpr int B = 8;
  const int wn1 = max(min(W, N - W), 0);
  const int nc = N * wn, total = 2 * nc + wn1 * wn1;
  const int base = (blockIdx.x - 1) * 64 * B + threadIdx.x;
  double v[B];
#pragma unroll
  for (int k = 0; k < B; ++k) {
    const int e = min(base + 64 * k, total - 1);
    size_t off;
    if (e < nc)
      off = (size_t)(e / wn) * N + e % wn;
    else if (e < 2 * nc)
      off = (size_t)((e - nc) / N) * N + (e - nc) % N;
    else
      off = (size_t)(W + (e - 2 * nc) / wn1) * N + W + (e - 2 * nc) % wn1;
    v[k] = G[off];
  }
#pragma unroll
  for (int k = 0; k < B; ++k) {
    const int e = base + 64 * k;
    if (e < nc)
      csn[(size_t)(e / wn) * WM + e % wn] = v[k];
    else if (e < 2 * nc)
      rsn[(size_t)((e - nc) % N) * WM + (e - nc) / N] = v[k];
    else if (e < total)
      bk1[(size_t)((e - 2 * nc) / wn1) * W + (e - 2 * nc) % wn1] = v[k];
  }
}

// PS consecutive doubles from a 16-byte aligned address, two per load.
template <int PS>
__device__ __forceinline__ void load_run(double (&v)[PS], const double* __restrict__ src) {
  static_assert(PS % 2 == 0, "runs of pairs");
  const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
  for (int i = 0; i < PS / 2; ++i) {
    const double2 t = s2[i];
    v[2 * i] = t.x;
    v[2 * i + 1] = t.y;
  }
}

// The window's factor products on the FP64 MFMA (16x16x4; lane l holds
// A[l%16][l/16] and B[l/16][l%16], and element j of the result is
// D[l/16 + 4j][l%16]).  In the store frame of G the window's factors are
//   U[r][n] = sum_p G~cur[r, w0+p] Zh[n][p],
//   W[n][c] = sum_p Zph[n][p] (delta(c, w0+p) - G~cur[w0+p, c])
// (Zh, Zph n-major with the frame scales folded in, zero past the accepts).
// U is formed transposed: block (nb, rows) of U^T holds in its element j
// exactly the A operand of k-step 16 nb + 4 j of the flush G += U W, and
// block (nb, cols) of W the B operand of the same step, so neither goes
// through LDS.  p-step s takes position p = PS (l/16) + s, so that every
// lane reads PS consecutive positions (two per load); steps s >= wn are
// skipped (all their positions lie past the window).
template <int WM>
struct WinOps {
  static constexpr int PS = WM / 4;   // p-steps
  static constexpr int NB = WM / 16;  // n blocks
  double za[NB][PS], zpa[NB][PS];     // A operands: Zh, Zph

  __device__ __forceinline__ void load_z(const double* __restrict__ Zh, const double* __restrict__ Zph,
                                         int lr, int lk) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      load_run<PS>(za[nb], Zh + (16 * nb + lr) * WM + PS * lk);
      load_run<PS>(zpa[nb], Zph + (16 * nb + lr) * WM + PS * lk);
    }
  }
};

// The pieces of the fused window step, shared by the per-window launch
// (k_flush_decide) and the persistent slice launch (k_slice_persist), which
// therefore compute the same values bit for bit.
//
// decider_block: the next window's block (window w1, wn1 sites) on the four
// waves of the calling workgroup, wave (bi, bj) the 16 x 16 block (bi, bj) of
// the 32 x 32 quadrant holding it, in the arithmetic of the tiles (the same
// operands and MFMA steps in the same order, so the block equals the one the
// tiles write to G bit for bit), written in the tilde frame to Zs (zero
// outside wn1 x wn1).  Inputs: the window's accepts a and Z, Z' (Zc, Zpc),
// the snapshots of its columns and rows (csc, rsc) and the copy of the next
// window's block before this window's flush (bkc).  The caller synchronizes
// the workgroup before Zs is read.
template <int WM>
__device__ __forceinline__ void decider_block(int tid, int N, int W, int w0, int wn, int a, int w1, int wn1,
                                              const double* __restrict__ ev, const double* __restrict__ evinv,
                                              const double* __restrict__ Zc, const double* __restrict__ Zpc,
                                              const double* __restrict__ csc, const double* __restrict__ rsc,
                                              const double* __restrict__ bkc, double (*Zs)[WM + 1]) {
  typedef WinOps<WM> Ops;
  constexpr int PS = Ops::PS, NB = Ops::NB;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nbl = (a + 15) >> 4;
  const int Q0 = w1 & ~31;
  const int bi = wave >> 1, bj = wave & 1;
  const int rq = Q0 + 16 * bi, cq = Q0 + 16 * bj;
  // (entries outside the window block are computed but never used); the
  // frame scales of the block's rows and column are read up front
  v4d blk;
  double evr[4];
  const double evic = evinv[min(cq + lr, N - 1)];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = rq + lk + 4 * j, cc = cq + lr;
    blk[j] = bkc[(size_t)min(max(r - w1, 0), W - 1) * W + min(max(cc - w1, 0), W - 1)];
    evr[j] = ev[min(r, N - 1)];
  }
  if (a > 0) {
    // operands: Zh, Zph rows, the snapshot row rq + l%16 (g) and the
    // transposed row snapshot at column cq + l%16 (h), PS positions each
    Ops ops;
    double gb[PS], hb[PS];
    ops.load_z(Zc, Zpc, lr, lk);
    load_run<PS>(gb, csc + (size_t)min(rq + lr, N - 1) * WM + PS * lk);
    const int ch = min(cq + lr, N - 1);
    load_run<PS>(hb, rsc + (size_t)ch * WM + PS * lk);
#pragma unroll
    for (int s = 0; s < PS; ++s) hb[s] = ((ch == w0 + PS * lk + s) ? 1.0 : 0.0) - hb[s];
    v4d ut[NB], wt[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) ut[nb] = wt[nb] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < PS; ++s)
      if (s < wn) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          if (nb < nbl) {
            ut[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ops.za[nb][s], gb[s], ut[nb], 0, 0, 0);
            wt[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ops.zpa[nb][s], hb[s], wt[nb], 0, 0, 0);
          }
      }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (16 * nb + 4 * j < a) blk = __builtin_amdgcn_mfma_f64_16x16x4f64(ut[nb][j], wt[nb][j], blk, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = rq + lk + 4 * j, cc = cq + lr;
    const double v = blk[j] * evr[j] * evic;
    if (r >= w1 && r < w1 + wn1 && cc >= w1 && cc < w1 + wn1) Zs[r - w1][cc - w1] = v;
  }
  // (the decisions read rows and columns below WM only: nothing to clear
  // for a full window)
  if (wave == 0 && wn1 < WM)
    for (int idx = lane; idx < WM * WM; idx += 64) {
      const int x = idx / WM, y = idx % WM;
      if (x >= wn1 || y >= wn1) Zs[x][y] = 0.0;
    }
}

// The tile quarter's operands of the factor products: G~cur[rows, w0..]
// (from the column snapshot) and G~cur[w0.., cols] (from the row snapshot).
template <int PS>
struct TileEdges {
  double gb[2][PS], hb[2][PS];
};

template <int WM>
__device__ __forceinline__ void tile_edges(TileEdges<WM / 4>& e, int lane, int N, int row0, int col0,
                                           const double* __restrict__ csc, const double* __restrict__ rsc) {
  constexpr int PS = WM / 4;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    load_run<PS>(e.gb[b], csc + (size_t)min(row0 + 16 * b + lr, N - 1) * WM + PS * lk);
    load_run<PS>(e.hb[b], rsc + (size_t)min(col0 + 16 * b + lr, N - 1) * WM + PS * lk);
  }
}

// The two parts of the edges: the column snapshot at the quarter's rows
// (U^T's operands) and the row snapshot at its columns (W's).
template <int WM>
__device__ __forceinline__ void tile_edges_g(double (&gb)[2][WM / 4], int lane, int N, int row0,
                                             const double* __restrict__ csc) {
  constexpr int PS = WM / 4;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int b = 0; b < 2; ++b) load_run<PS>(gb[b], csc + (size_t)min(row0 + 16 * b + lr, N - 1) * WM + PS * lk);
}

template <int WM>
__device__ __forceinline__ void tile_edges_h(double (&hb)[2][WM / 4], int lane, int N, int col0,
                                             const double* __restrict__ rsc) {
  constexpr int PS = WM / 4;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int b = 0; b < 2; ++b) load_run<PS>(hb[b], rsc + (size_t)min(col0 + 16 * b + lr, N - 1) * WM + PS * lk);
}

// tile_apply: a 64 x 64 tile's quarter (wave (wave >> 1, wave & 1), rows
// row0.., columns col0..) in registers takes the window's rank-a update
// G += U W, U^T and W formed from Z, Z' (ops) and the tile's edges on the
// MFMA: in one piece (tile_apply), or in two parts for several tiles of a
// tile row, tile_ut (U^T of the quarter's rows, shared) and tile_wuw (W of
// its columns and the product).  All compute the same values.
template <int WM>
__device__ __forceinline__ void tile_ut(v4d (&ut)[WM / 16][2], const WinOps<WM>& ops,
                                        const double (&gb)[2][WM / 4], int wn, int a) {
  constexpr int PS = WM / 4, NB = WM / 16;
  const int nbl = (a + 15) >> 4;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int b = 0; b < 2; ++b) ut[nb][b] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < PS; ++s)
    if (s < wn) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        if (nb < nbl) {
#pragma unroll
          for (int b = 0; b < 2; ++b)
            ut[nb][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ops.za[nb][s], gb[b][s], ut[nb][b], 0, 0, 0);
        }
    }
}

template <int WM>
__device__ __forceinline__ void tile_wuw(v4d (&acc)[2][2], const WinOps<WM>& ops, double (&hb)[2][WM / 4],
                                         const v4d (&ut)[WM / 16][2], int lane, int N, int w0, int wn, int a,
                                         int col0) {
  constexpr int PS = WM / 4, NB = WM / 16;
  const int lr = lane & 15, lk = lane >> 4;
  const int nbl = (a + 15) >> 4;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int ch = min(col0 + 16 * b + lr, N - 1);
#pragma unroll
    for (int s = 0; s < PS; ++s) hb[b][s] = ((ch == w0 + PS * lk + s) ? 1.0 : 0.0) - hb[b][s];
  }
  v4d wt[NB][2];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int b = 0; b < 2; ++b) wt[nb][b] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < PS; ++s)
    if (s < wn) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        if (nb < nbl) {
#pragma unroll
          for (int b = 0; b < 2; ++b)
            wt[nb][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ops.zpa[nb][s], hb[b][s], wt[nb][b], 0, 0, 0);
        }
    }
  // G += U W, k-steps 16 nb + 4 j in increasing order (the order of k_flush_f64)
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (16 * nb + 4 * j < a) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ut[nb][bi][j], wt[nb][bj][j], acc[bi][bj], 0, 0, 0);
      }
}

// (One tile: U^T and W formed together, eight independent MFMA chains.)
template <int WM>
__device__ __forceinline__ void tile_apply(v4d (&acc)[2][2], const WinOps<WM>& ops, TileEdges<WM / 4>& e,
                                           int lane, int N, int w0, int wn, int a, int col0) {
  typedef WinOps<WM> Ops;
  constexpr int PS = Ops::PS, NB = Ops::NB;
  const int lr = lane & 15, lk = lane >> 4;
  const int nbl = (a + 15) >> 4;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int ch = min(col0 + 16 * b + lr, N - 1);
#pragma unroll
    for (int s = 0; s < PS; ++s) e.hb[b][s] = ((ch == w0 + PS * lk + s) ? 1.0 : 0.0) - e.hb[b][s];
  }
  v4d ut[NB][2], wt[NB][2];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int b = 0; b < 2; ++b) ut[nb][b] = wt[nb][b] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < PS; ++s)
    if (s < wn) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        if (nb < nbl) {
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            ut[nb][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ops.za[nb][s], e.gb[b][s], ut[nb][b], 0, 0, 0);
            wt[nb][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ops.zpa[nb][s], e.hb[b][s], wt[nb][b], 0, 0, 0);
          }
        }
    }
  // G += U W, k-steps 16 nb + 4 j in increasing order (the order of k_flush_f64)
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (16 * nb + 4 * j < a) {
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
            acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ut[nb][bi][j], wt[nb][bj][j], acc[bi][bj], 0, 0, 0);
      }
}

// tile_flush: the window's update of one tile quarter, Z and the edges
// loaded here.
template <int WM>
__device__ __forceinline__ void tile_flush(v4d (&acc)[2][2], int lane, int N, int w0, int wn, int a, int row0,
                                           int col0, const double* __restrict__ Zc,
                                           const double* __restrict__ Zpc, const double* __restrict__ csc,
                                           const double* __restrict__ rsc) {
  WinOps<WM> ops;
  ops.load_z(Zc, Zpc, lane & 15, lane >> 4);
  TileEdges<WM / 4> e;
  tile_edges<WM>(e, lane, N, row0, col0, csc, rsc);
  tile_apply<WM>(acc, ops, e, lane, N, w0, wn, a, col0);
}

// tile_snapshots: the tile quarter's part of the next window's columns and
// rows (csn, rsn) and of the diagonal block of the window after next (bkn).
__device__ __forceinline__ void tile_snapshots(const v4d (&acc)[2][2], int lane, int N, int W, int WMs, int row0,
                                               int col0, int w1, int wn1, int w2, int wn2,
                                               double* __restrict__ csn, double* __restrict__ rsn,
                                               double* __restrict__ bkn) {
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + 16 * bi + lk + 4 * j, cc = col0 + 16 * bj + lr;
        if (r < N && cc < N) {
          if (cc >= w1 && cc < w1 + wn1) csn[(size_t)r * WMs + (cc - w1)] = acc[bi][bj][j];
          if (r >= w1 && r < w1 + wn1) rsn[(size_t)cc * WMs + (r - w1)] = acc[bi][bj][j];
          if (r >= w2 && r < w2 + wn2 && cc >= w2 && cc < w2 + wn2)
            bkn[(size_t)(r - w2) * W + (cc - w2)] = acc[bi][bj][j];
        }
      }
}

__device__ __forceinline__ void tile_load(v4d (&acc)[2][2], const double* __restrict__ G, int N, int lane,
                                          int row0, int col0) {
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + 16 * bi + lk + 4 * j, cc = col0 + 16 * bj + lr;
        acc[bi][bj][j] = G[(size_t)min(r, N - 1) * N + min(cc, N - 1)];
      }
}

__device__ __forceinline__ void tile_store(const v4d (&acc)[2][2], double* __restrict__ G, int N, int lane,
                                           int row0, int col0) {
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + 16 * bi + lk + 4 * j, cc = col0 + 16 * bj + lr;
        if (r < N && cc < N) G[(size_t)r * N + cc] = acc[bi][bj][j];
      }
}

template <int WM>
__global__ void __launch_bounds__(256)
k_flush_decide(double* __restrict__ G, int N, int gxt, const double* __restrict__ ev,
               const double* __restrict__ evinv, int8_t* __restrict__ s_l,
               const double* __restrict__ u, const uint8_t* __restrict__ forced,
               uint8_t* __restrict__ acc_out, double* __restrict__ ratio_out,
               const double* __restrict__ sc, int win, int W, int nw, int* __restrict__ win_a,
               int* __restrict__ win_p, const double* __restrict__ Zc, const double* __restrict__ Zpc,
               double* __restrict__ Zn, double* __restrict__ Zpn, const double* __restrict__ csc,
               const double* __restrict__ rsc, double* __restrict__ csn, double* __restrict__ rsn,
               const double* __restrict__ bkc, double* __restrict__ bkn, size_t zs, size_t zn) {
  // Roles: with a next window, workgroup z < nch (the first dispatched)
  // decides chain z's next window; the others take the gxt x gxt tiles.
  const int w1 = (win + 1) * W, w2 = (win + 2) * W;
  const bool has_next = win + 1 < nw;
  const int T = gxt * gxt, nz = gridDim.z;
  const int lin = blockIdx.x + gridDim.x * blockIdx.z;
  const bool decider = has_next && lin < nz;
  int z, t;
  if (decider) {
    z = lin;
    t = 0;
  } else {
    const int j = lin - (has_next ? nz : 0);
    z = j / T;
    t = j % T;
  }
  const int bx = t % gxt, by = t / gxt;
  G = zw_at(G, zs, z);
  ev = zw_at(ev, zs, z);
  evinv = zw_at(evinv, zs, z);
  s_l = zw_at(s_l, zs, z);
  u = zc_at(u, zn, z);
  forced = zc_at(forced, zn, z);
  acc_out = zc_at(acc_out, zn, z);
  ratio_out = zc_at(ratio_out, zn, z);
  win_a = zw_at(win_a, zs, z);
  win_p = zw_at(win_p, zs, z);
  Zc = zw_at(Zc, zs, z);
  Zpc = zw_at(Zpc, zs, z);
  Zn = zw_at(Zn, zs, z);
  Zpn = zw_at(Zpn, zs, z);
  csc = zw_at(csc, zs, z);
  rsc = zw_at(rsc, zs, z);
  csn = zw_at(csn, zs, z);
  rsn = zw_at(rsn, zs, z);
  bkc = zw_at(bkc, zs, z);
  bkn = zw_at(bkn, zs, z);
  sc = zw_at(sc, zs, z);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int w0 = win * W;
  const int wn = min(W, N - w0);
  const int a = win_a[win];
  const int wn1 = has_next ? min(W, N - w1) : 0;
  const int wn2 = win + 2 < nw ? min(W, N - w2) : 0;
  if (decider) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double(*Zs)[WM + 1] = reinterpret_cast<double(*)[WM + 1]>(smem_raw);
    double2(*hist)[64] = reinterpret_cast<double2(*)[64]>(smem_raw + sizeof(double) * WM * (WM + 1));
    int sx;
    double ux;
    bool fx;
    site_inputs(lane, min(w1, N - 1), max(wn1, 1), s_l, u, forced, ev, sx, ux, fx);
    decider_block<WM>(tid, N, W, w0, wn, a, w1, wn1, ev, evinv, Zc, Zpc, csc, rsc, bkc, Zs);
    __syncthreads();
    if (wave != 0) return;
    const double em2a = sc[SC_EM2A], ep2a = sc[SC_EP2A];
    decide_window<WM>(lane, wn1, w1, W, win + 1, Zs, hist, sx, ux, fx, forced != nullptr, em2a, ep2a,
                      s_l, acc_out, ratio_out, win_a, win_p, Zn, Zpn, ev, evinv);
    return;
  }
  // a tile: wave (wave >> 1, wave & 1) takes the 32 x 32 quarter at (row0, col0)
  const int row0 = by * 64 + (wave >> 1) * 32, col0 = bx * 64 + (wave & 1) * 32;
  v4d acc[2][2];
  tile_load(acc, G, N, lane, row0, col0);
  if (a > 0) {
    tile_flush<WM>(acc, lane, N, w0, wn, a, row0, col0, Zc, Zpc, csc, rsc);
    tile_store(acc, G, N, lane, row0, col0);
  }
  // copies for the next launches: the next window's columns and rows, and
  // the diagonal block of the window after next
  tile_snapshots(acc, lane, N, W, WM, row0, col0, w1, wn1, w2, wn2, csn, rsn, bkn);
}

// the decider's LDS: the window block and the decision history
template <int WM>
constexpr size_t flush_decide_lds() {
  return size_t(WM * (WM + 1)) * 8 + size_t(WM) * 64 * 16;
}

// ---------------------------------------------------------------------------
// Persistent slice launch (one chain, FP64, every workgroup resident): the
// window steps of the per-window launches in one launch per slice.
// Workgroup 0 decides the windows in turn; workgroups 1..T own one 64 x 64
// tile of G each, held in registers for the whole slice.  They hand over
// through counters in the chain's workspace: ctl[1 + k] counts the tiles done
// with the snapshots of window k (the flush of window k - 1, or for k = 0 the
// initial copies); ctl[0] = k + 1 is window k's go, set by the decider once
// window k's Z, Z' are written and ctl[1 + k] = T; ctl[2 + nw] is set by a
// workgroup whose wait ran out.  Producer: its stores, a device-scope release,
// then the counter; consumer: a bounded spin on the counter, then a
// device-scope acquire before its loads.  A wait that runs out (a workgroup
// not resident, or a fault) sets the abort flag, after which every wait
// returns at once and the tiles write NaN into G, which the next
// stabilization reports (KDQMC_ENUMERIC); nothing spins without bound.
// Order of the data (buffers by window parity): window k's Z, Z' are written
// by the decider before go k and read by flush k; the decider rewrites their
// buffer with window k + 2 after go k + 1, i.e. after every tile is done with
// flush k.  Window k's snapshots are written during flush k - 1 (complete at
// go k) and read by flush k and the decider's block of window k + 1; flush
// k + 1 rewrites them after go k + 1, which the decider gives after that
// block.  Window k's block copy is written during flush k - 2 and read for
// the block of window k (before go k), and rewritten during flush k.
// ---------------------------------------------------------------------------
constexpr int kSpinLimit = 1 << 22;

// One thread spins and takes the device-scope acquire (the cache
// invalidations act for the whole compute unit); the workgroup barrier then
// orders the other waves' loads after it.
__device__ __forceinline__ bool wait_count(int* __restrict__ ctr, int target, int* __restrict__ abort_flag) {
  int good = 1;
  if (threadIdx.x == 0) {
    int spins = 0;
    for (;;) {
      if (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          ++spins > kSpinLimit) {
        good = 0;
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  return __syncthreads_and(good) != 0;
}

// Every wave's stores complete (workgroup-scope release), the barrier, then
// one thread's device-scope release (the write-back acts for the whole
// cache) and the counter.
__device__ __forceinline__ void signal_count(int* __restrict__ ctr) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// The end of a workgroup of the slice launch: the last of the grid to get
// here clears every counter (ctl[0 .. n), the exit count at ctl[n - 1]
// included) for the next launch on the stream; the others have made their
// last counter update before their own increment.
__device__ __forceinline__ void slice_exit(int* __restrict__ ctl, int n) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const int prev = __hip_atomic_fetch_add(ctl + n - 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == (int)gridDim.x - 1)
      for (int i = 0; i < n; ++i) __hip_atomic_store(ctl + i, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int WM, int TPW>
__global__ void __launch_bounds__(256)
k_slice_persist(double* __restrict__ G, int N, int gxt, const double* __restrict__ ev,
                const double* __restrict__ evinv, int8_t* __restrict__ s_l,
                const double* __restrict__ u, const uint8_t* __restrict__ forced,
                uint8_t* __restrict__ acc_out, double* __restrict__ ratio_out,
                const double* __restrict__ sc, int W, int nw, int* __restrict__ win_a,
                int* __restrict__ win_p, double* __restrict__ Zb, double* __restrict__ Zpb,
                double* __restrict__ csb, double* __restrict__ rsb, double* __restrict__ bkb,
                int* __restrict__ ctl) {
  const int T = gxt * gxt;
  const int nwg = gridDim.x - 1;  // tile workgroups, TPW tiles each at most
  const size_t zz = (size_t)WM * WM, nwv = (size_t)N * WM, ww = (size_t)W * W;
  int* zflag = ctl;
  int* cnt = ctl + 1;          // cnt[k], k = 0 .. nw
  int* abort_flag = ctl + 2 + nw;
  const int nctl = nw + 4;     // (and the exit count)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double Zs[WM][WM + 1];
  __shared__ double2 hist[WM][64];
  if (blockIdx.x == 0) {
    // ---- the decider
    const double em2a = sc[SC_EM2A], ep2a = sc[SC_EP2A];
    if (wave == 0) {
      // window 0 straight from G (nothing flushed yet)
      const int wn0 = min(W, N);
      int sx;
      double ux;
      bool fx;
      site_inputs(lane, 0, wn0, s_l, u, forced, ev, sx, ux, fx);
      constexpr int PER = (WM * WM + 63) / 64;
      double gv[PER];
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int idx = lane + 64 * j;
        const int gx = min(idx / WM, wn0 - 1), gy = min(idx % WM, wn0 - 1);
        gv[j] = G[(size_t)gx * N + gy] * ev[gx] * evinv[gy];
      }
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int idx = lane + 64 * j;
        const bool ok = idx / WM < wn0 && idx % WM < wn0;
        if (idx < WM * WM) Zs[idx / WM][idx % WM] = ok ? gv[j] : 0.0;
      }
      wave_sync();
      decide_window<WM>(lane, wn0, 0, W, 0, Zs, hist, sx, ux, fx, forced != nullptr, em2a, ep2a, s_l, acc_out,
                        ratio_out, win_a, win_p, Zb, Zpb, ev, evinv);
    }
    // window 0's Z is out and the tiles' initial copies are complete: go
    bool ok = wait_count(cnt + 0, nwg, abort_flag);
    signal_count(zflag);
    for (int k = 0; k + 1 < nw; ++k) {
      const int w0 = k * W, wn = min(W, N - w0);
      const int w1 = w0 + W, wn1 = min(W, N - w1);
      int sx = 1;
      double ux = 0.0;
      bool fx = false;
      if (wave == 0) site_inputs(lane, w1, wn1, s_l, u, forced, ev, sx, ux, fx);
      // (window k's snapshots and window k + 1's block copy are complete:
      // the wait before window k's go)
      if (ok) {
        const int a = win_a[k];
        decider_block<WM>(tid, N, W, w0, wn, a, w1, wn1, ev, evinv, Zb + (k & 1) * zz, Zpb + (k & 1) * zz,
                          csb + (k & 1) * nwv, rsb + (k & 1) * nwv, bkb + ((k + 1) & 1) * ww, Zs);
      }
      __syncthreads();
      if (ok && wave == 0)
        decide_window<WM>(lane, wn1, w1, W, k + 1, Zs, hist, sx, ux, fx, forced != nullptr, em2a, ep2a, s_l,
                          acc_out, ratio_out, win_a, win_p, Zb + ((k + 1) & 1) * zz, Zpb + ((k + 1) & 1) * zz,
                          ev, evinv);
      // window k + 1's go once every tile is done with flush k (whose
      // snapshots window k + 1's flush and the next block read)
      ok = ok && wait_count(cnt + k + 1, nwg, abort_flag);
      signal_count(zflag);
    }
    slice_exit(ctl, nctl);
    return;
  }
  // ---- TPW consecutive tiles (t = (blockIdx.x - 1) TPW + i), held in
  // registers for the whole slice; where they share a tile row (always when
  // TPW divides the tiles per row) they share the window's U^T
  v4d acc[TPW][2][2];
  int row0[TPW], col0[TPW];
  bool live[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = (blockIdx.x - 1) * TPW + i;
    live[i] = t < T;
    const int tc = live[i] ? t : 0;
    row0[i] = (tc / gxt) * 64 + (wave >> 1) * 32;
    col0[i] = (tc % gxt) * 64 + (wave & 1) * 32;
    tile_load(acc[i], G, N, lane, row0[i], col0[i]);
  }
  {
    // window 0's columns and rows, window 1's block
    const int wn0 = min(W, N), w1 = W, wn1 = nw > 1 ? min(W, N - W) : 0;
#pragma unroll
    for (int i = 0; i < TPW; ++i)
      if (live[i]) tile_snapshots(acc[i], lane, N, W, WM, row0[i], col0[i], 0, wn0, w1, wn1, csb, rsb, bkb + ww);
  }
  signal_count(cnt + 0);
  bool ok = true;
  for (int k = 0; k < nw; ++k) {
    const int w0 = k * W, wn = min(W, N - w0);
    const int w1 = w0 + W, wn1 = k + 1 < nw ? min(W, N - w1) : 0;
    const int w2 = w1 + W, wn2 = k + 2 < nw ? min(W, N - w2) : 0;
    // window k's go: its Z is published and every tile is done with the
    // snapshots it reads
    ok = ok && wait_count(zflag, k + 1, abort_flag);
    if (ok) {
      const int a = win_a[k];
      const double* csc = csb + (k & 1) * nwv;
      const double* rsc = rsb + (k & 1) * nwv;
      if (a > 0) {
        WinOps<WM> ops;
        ops.load_z(Zb + (k & 1) * zz, Zpb + (k & 1) * zz, lane & 15, lane >> 4);
        if constexpr (TPW == 1) {
          TileEdges<WM / 4> e;
          tile_edges<WM>(e, lane, N, row0[0], col0[0], csc, rsc);
          if (live[0]) tile_apply<WM>(acc[0], ops, e, lane, N, w0, wn, a, col0[0]);
        } else {
          // Z once for the window; U^T once per tile row (the tiles of a
          // workgroup share one unless they straddle two rows); each tile's
          // column operands, the next tile's in flight while the current
          // one is on the MFMA
          v4d ut[WM / 16][2];
          double gb[2][WM / 4], hb[2][2][WM / 4];
          tile_edges_g<WM>(gb, lane, N, row0[0], csc);
          tile_edges_h<WM>(hb[0], lane, N, col0[0], rsc);
#pragma unroll
          for (int i = 0; i < TPW; ++i) {
            if (i + 1 < TPW) tile_edges_h<WM>(hb[(i + 1) & 1], lane, N, col0[i + 1], rsc);
            const bool new_row = i == 0 || (live[i] && row0[i] != row0[i - 1]);
            if (i > 0 && new_row) tile_edges_g<WM>(gb, lane, N, row0[i], csc);
            if (new_row) tile_ut<WM>(ut, ops, gb, wn, a);
            if (live[i]) tile_wuw<WM>(acc[i], ops, hb[i & 1], ut, lane, N, w0, wn, a, col0[i]);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < TPW; ++i)
        if (live[i])
          tile_snapshots(acc[i], lane, N, W, WM, row0[i], col0[i], w1, wn1, w2, wn2, csb + ((k + 1) & 1) * nwv,
                         rsb + ((k + 1) & 1) * nwv, bkb + (k & 1) * ww);
    }
    signal_count(cnt + k + 1);
  }
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    if (!live[i]) continue;
    if (!ok) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
          acc[i][bi][bj] = v4d{__builtin_nan(""), __builtin_nan(""), __builtin_nan(""), __builtin_nan("")};
    }
    tile_store(acc[i], G, N, lane, row0[i], col0[i]);
  }
  slice_exit(ctl, nctl);
}

// ---------------------------------------------------------------------------
// New pending factors of the window (store frame), with G~cur = G + U_pend
// W_pend (the m pending factors of this flush group):
//   U[:, m+n] = sum_p G~cur[:, w0+p] Zh[n][p],
//   W[m+n, :] = sum_p Zph[n][p] (e_{w0+p} - G~cur[w0+p, :]).
// One wave per 16 rows r (which are also the columns of W): the columns
// G~cur[r, S] and rows G~cur[S, r] start from G and take the pending products
// on the MFMA, laid out so that element j of block pb is the operand of p-step
// 4 pb + j; then U^T and W on the MFMA with the operands and steps of the
// fused window launch (both schedules produce the same factors bit for bit).
// ---------------------------------------------------------------------------
template <typename T, int WM>
__global__ void __launch_bounds__(256)
k_extend(const T* __restrict__ G, int N, T* __restrict__ Up, T* __restrict__ Wp,
         const int* __restrict__ win_a, int win, int grp0, const double* __restrict__ Zg,
         const double* __restrict__ Zpg, int W, int w0, size_t zs) {
  typedef WinOps<WM> Ops;
  constexpr int PS = Ops::PS, NB = Ops::NB, PB = PS / 4;
  G = zw(G, zs);
  Up = zw(Up, zs);
  Wp = zw(Wp, zs);
  win_a = zw(win_a, zs);
  Zg = zw(Zg, zs);
  Zpg = zw(Zpg, zs);
  const int a = win_a[win];
  if (a == 0) return;
  int m = 0;
  for (int j = grp0; j < win; ++j) m += win_a[j];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int r0 = blockIdx.x * 64 + 16 * wave;
  if (r0 >= N) return;  // (no barriers below)
  const int wn = min(W, N - w0);
  const int nbl = (a + 15) >> 4;
  const int r = r0 + lr, rc = min(r, N - 1);
  Ops ops;
  ops.load_z(Zg, Zpg, lr, lk);
  // element j of block pb: position PS (l/16) + 4 pb + j; the A operands of
  // the pending products take row i = l%16 at position PS (i%4) + 4 pb + i/4
  v4d gT[PB], hT[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = min(w0 + PS * lk + 4 * pb + j, N - 1);
      gT[pb][j] = double(G[(size_t)rc * N + col]);
      hT[pb][j] = double(G[(size_t)col * N + rc]);
    }
  for (int j0 = 0; j0 < m; j0 += 4) {
    const int jj = min(j0 + lk, m - 1);
    const bool jin = j0 + lk < m;
    const double ub = jin ? double(Up[(size_t)jj * N + rc]) : 0.0;
    const double wb = jin ? double(Wp[(size_t)jj * N + rc]) : 0.0;
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const int col = min(w0 + PS * (lr & 3) + 4 * pb + (lr >> 2), N - 1);
      const double wa = jin ? double(Wp[(size_t)jj * N + col]) : 0.0;
      const double ua = jin ? double(Up[(size_t)jj * N + col]) : 0.0;
      gT[pb] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa, ub, gT[pb], 0, 0, 0);
      hT[pb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ua, wb, hT[pb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int j = 0; j < 4; ++j) hT[pb][j] = ((rc == w0 + PS * lk + 4 * pb + j) ? 1.0 : 0.0) - hT[pb][j];
  v4d ut[NB], wt[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) ut[nb] = wt[nb] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < PS; ++s)
    if (s < wn) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        if (nb < nbl) {
          ut[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ops.za[nb][s], gT[s >> 2][s & 3], ut[nb], 0, 0, 0);
          wt[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ops.zpa[nb][s], hT[s >> 2][s & 3], wt[nb], 0, 0, 0);
        }
    }
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = 16 * nb + lk + 4 * j;
      if (n < a && r < N) {
        Up[(size_t)(m + n) * N + r] = T(ut[nb][j]);
        Wp[(size_t)(m + n) * N + r] = T(wt[nb][j]);
      }
    }
}

// Window submatrix of the next window from G and the pending factors:
// Gs[x][y] = ev_x evinv_y (G[x,y] + sum_{j<m} U[j][x] W[j][y]), the sum on the
// MFMA; one wave per 16 x 16 block of the (at most 64 x 64) window.
template <typename T>
__global__ void __launch_bounds__(256)
k_prep(const T* __restrict__ G, int N, const double* __restrict__ ev,
       const double* __restrict__ evinv, const T* __restrict__ Up, const T* __restrict__ Wp,
       const int* __restrict__ win_a, int grp0, int upto, int w0, int wn, int W,
       double* __restrict__ Gs, size_t zs) {
  G = zw(G, zs);
  ev = zw(ev, zs);
  evinv = zw(evinv, zs);
  Up = zw(Up, zs);
  Wp = zw(Wp, zs);
  win_a = zw(win_a, zs);
  Gs = zw(Gs, zs);
  int m = 0;
  for (int j = grp0; j <= upto; ++j) m += win_a[j];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nbk = (wn + 15) >> 4;
  for (int blk = wave; blk < nbk * nbk; blk += 4) {
    const int x0 = (blk / nbk) * 16, y0 = (blk % nbk) * 16;
    v4d d;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = min(x0 + lk + 4 * j, wn - 1), y = min(y0 + lr, wn - 1);
      d[j] = double(G[(size_t)(w0 + x) * N + w0 + y]);
    }
    for (int j0 = 0; j0 < m; j0 += 4) {
      const int jj = min(j0 + lk, m - 1);
      const bool jin = j0 + lk < m;
      const double ua = jin ? double(Up[(size_t)jj * N + w0 + min(x0 + lr, wn - 1)]) : 0.0;
      const double wb = jin ? double(Wp[(size_t)jj * N + w0 + min(y0 + lr, wn - 1)]) : 0.0;
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(ua, wb, d, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = x0 + lk + 4 * j, y = y0 + lr;
      if (x < wn && y < wn) Gs[x * W + y] = d[j] * ev[w0 + x] * evinv[w0 + y];
    }
  }
}

// ---------------------------------------------------------------------------
// Rank-K flush G += U^T W (U, W stored K x N), K = accepted flips of the
// flush group (read on the device).  FP64: v_mfma_f64_16x16x4.
// Tile 64 x 64 per workgroup (4 waves, each 32 x 32 = 2 x 2 MFMA blocks).
// MFMA 16x16x4 f64 operand layout (lane l): A[l%16][l/16], B[l/16][l%16];
// result element j of lane l is D[l/16 + 4j][l%16] (checked on gfx950).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_flush_f64(double* __restrict__ G, int N, const double* __restrict__ Up,
            const double* __restrict__ Wp, const int* __restrict__ win_a, int grp0, int grp1,
            size_t zs) {
  G = zw(G, zs);
  Up = zw(Up, zs);
  Wp = zw(Wp, zs);
  win_a = zw(win_a, zs);
  int K = 0;
  for (int j = grp0; j < grp1; ++j) K += win_a[j];
  if (K == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int col0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  v4d acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + 16 * bi + lk + 4 * j, cc = col0 + 16 * bj + lr;
        acc[bi][bj][j] = (r < N && cc < N) ? G[(size_t)r * N + cc] : 0.0;
      }
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + lk;
    double a[2], b[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int r = row0 + 16 * bi + lr;
      a[bi] = (k < K && r < N) ? Up[(size_t)k * N + r] : 0.0;
      const int cc = col0 + 16 * bi + lr;
      b[bi] = (k < K && cc < N) ? Wp[(size_t)k * N + cc] : 0.0;
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + 16 * bi + lk + 4 * j, cc = col0 + 16 * bj + lr;
        if (r < N && cc < N) G[(size_t)r * N + cc] = acc[bi][bj][j];
      }
}

// Split-precision flush for FP32 G: x = hi + lo * 2^-S with hi, lo in H
// (FP16 or BF16); U W ~= hi_u hi_w + 2^-S (hi_u lo_w + lo_u hi_w), the two
// parts accumulated in FP32 by v_mfma_f32_16x16x32_{f16,bf16}.
// MFMA 16x16x32 operand layout (lane l): A row l%16, k = 8*(l/16) .. +7;
// B column l%16, same k; result element j of lane l is D[4*(l/16)+j][l%16]
// (checked on gfx950; note the different row order from the f64 MFMA).
template <typename H>
struct SplitTraits;
template <>
struct SplitTraits<_Float16> {
  typedef v8h vec;
  static constexpr float kScale = 4096.0f;  // 2^12 keeps the low part normal in FP16
  __device__ static v4f mfma(vec a, vec b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct SplitTraits<__bf16> {
  typedef v8bf vec;
  static constexpr float kScale = 256.0f;
  __device__ static v4f mfma(vec a, vec b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <typename H>
__global__ void __launch_bounds__(256)
k_flush_split(float* __restrict__ G, int N, const float* __restrict__ Up,
              const float* __restrict__ Wp, const int* __restrict__ win_a, int grp0, int grp1,
              size_t zs) {
  G = zw(G, zs);
  Up = zw(Up, zs);
  Wp = zw(Wp, zs);
  win_a = zw(win_a, zs);
  typedef SplitTraits<H> Tr;
  typedef typename Tr::vec vec;
  int K = 0;
  for (int j = grp0; j < grp1; ++j) K += win_a[j];
  if (K == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int col0 = blockIdx.x * 64 + (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  v4f hh[2][2], cr[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + 16 * bi + 4 * lk + j, cc = col0 + 16 * bj + lr;
        hh[bi][bj][j] = (r < N && cc < N) ? G[(size_t)r * N + cc] : 0.0f;
        cr[bi][bj][j] = 0.0f;
      }
  for (int k0 = 0; k0 < K; k0 += 32) {
    vec ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int r = row0 + 16 * bi + lr;
      const int cc = col0 + 16 * bi + lr;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int k = k0 + 8 * lk + t;
        const float xa = (k < K && r < N) ? Up[(size_t)k * N + r] : 0.0f;
        const float xb = (k < K && cc < N) ? Wp[(size_t)k * N + cc] : 0.0f;
        const H ha = H(xa), hb = H(xb);
        ah[bi][t] = ha;
        bh[bi][t] = hb;
        al[bi][t] = H((xa - float(ha)) * Tr::kScale);
        bl[bi][t] = H((xb - float(hb)) * Tr::kScale);
      }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        hh[bi][bj] = Tr::mfma(ah[bi], bh[bj], hh[bi][bj]);
        cr[bi][bj] = Tr::mfma(ah[bi], bl[bj], cr[bi][bj]);
        cr[bi][bj] = Tr::mfma(al[bi], bh[bj], cr[bi][bj]);
      }
  }
  const float inv = 1.0f / Tr::kScale;
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = row0 + 16 * bi + 4 * lk + j, cc = col0 + 16 * bj + lr;
        if (r < N && cc < N) G[(size_t)r * N + cc] = hh[bi][bj][j] + cr[bi][bj][j] * inv;
      }
}

// ---------------------------------------------------------------------------
// Host orchestration of one slice's updates.
// ---------------------------------------------------------------------------
namespace {


// The fused schedule of one slice (see k_flush_decide): 1 + nw launches.
template <int WM>
int fused_updates(kdqmc_ctx* c, int l, const double* u, const uint8_t* forced, uint8_t* acc,
                  double* ratio, size_t zn) {
  const int N = c->N, W = c->w;
  double* G = static_cast<double*>(c->G);
  int8_t* s_l = c->fields + (size_t)(l - 1) * N;
  const unsigned Z = (unsigned)c->nch;
  const size_t zs = c->zs;
  // Z, Z' and the snapshots have the padded stride WM (= c->wm), the block
  // copies the window's own W
  const size_t zz = (size_t)WM * WM, nwv = (size_t)N * WM, ww = (size_t)W * W;
  const int wn0 = std::min(W, N), wn1 = std::max(std::min(W, N - W), 0);
  const int nsnap = (2 * N * wn0 + wn1 * wn1 + 64 * 8 - 1) / (64 * 8);
  const int gxt = (N + 63) / 64;
  if (c->persist) {
    // one resident launch for the slice (the context checked that the
    // decider and ceil(gxt^2 / tpw) tile workgroups fit on the device)
    const int e0 = prof_mark(c);
    // (the counters start at zero: cleared when the context is made and
    // by the last workgroup of every launch)
    const int T = gxt * gxt, tpw = c->persist_tpw, nwg = (T + tpw - 1) / tpw;
#define PERSIST(TPW)                                                                                    \
  hipLaunchKernelGGL((k_slice_persist<WM, TPW>), dim3(1 + nwg), dim3(256), 0, c->stream, G, N, gxt, c->ev,   \
                     c->evinv, s_l, u, forced, acc, ratio, c->sc, W, c->nw, c->win_a, c->win_p, c->Xw, c->Yw, \
                     c->snapc, c->snapr, c->snapb, c->ctl)
    if (tpw == 1) PERSIST(1);
    else if (tpw == 2) PERSIST(2);
    else PERSIST(3);
#undef PERSIST
    prof_pair(c, PH_FLUSH_DECIDE, e0, prof_mark(c));
    KDQMC_HIP(hipGetLastError());
    return KDQMC_OK;
  }
  const int e0 = prof_mark(c);
  hipLaunchKernelGGL((k_window_start<WM>), dim3(1 + nsnap, 1, Z), dim3(64), 0, c->stream, G, N, c->ev,
                     c->evinv, s_l, u, forced, acc, ratio, wn0, W, c->sc, c->win_a, c->win_p, c->Xw,
                     c->Yw, c->snapc, c->snapr, c->snapb + ww, zs, zn);
  int e1 = prof_mark(c);
  prof_pair(c, PH_DECIDE, e0, e1);
  for (int win = 0; win < c->nw; ++win) {
    const size_t cur = win & 1, nxt = cur ^ 1;
    // the tiles, and with a next window one deciding workgroup per chain
    const dim3 grid(gxt * gxt + (win + 1 < c->nw ? 1 : 0), 1, Z);
    hipLaunchKernelGGL((k_flush_decide<WM>), grid, dim3(256), flush_decide_lds<WM>(), c->stream, G, N,
                       gxt, c->ev, c->evinv, s_l, u, forced, acc, ratio, c->sc, win, W, c->nw, c->win_a,
                       c->win_p, c->Xw + cur * zz, c->Yw + cur * zz, c->Xw + nxt * zz, c->Yw + nxt * zz,
                       c->snapc + cur * nwv, c->snapr + cur * nwv, c->snapc + nxt * nwv,
                       c->snapr + nxt * nwv, c->snapb + nxt * ww, c->snapb + cur * ww, zs, zn);
    const int e2 = prof_mark(c);
    prof_pair(c, PH_FLUSH_DECIDE, e1, e2);
    e1 = e2;
  }
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

template <typename T>
int slice_updates(kdqmc_ctx* c, int l, const double* u, const uint8_t* forced, uint8_t* acc,
                  double* ratio, size_t zn) {
  if constexpr (sizeof(T) == 8) {
    if (c->fused)
      return c->w <= 16 ? fused_updates<16>(c, l, u, forced, acc, ratio, zn)
                        : fused_updates<32>(c, l, u, forced, acc, ratio, zn);
  }
  const int N = c->N, W = c->w;
  T* G = static_cast<T*>(c->G);
  T* Up = static_cast<T*>(c->Upend);
  T* Wp = static_cast<T*>(c->Wpend);
  int8_t* s_l = c->fields + (size_t)(l - 1) * N;
  const unsigned Z = (unsigned)c->nch;
  const size_t zs = c->zs;
  for (int win = 0; win < c->nw; ++win) {
    const int w0 = win * W;
    const int wn = std::min(W, N - w0);
    const int grp0 = (win / c->F) * c->F;
    const bool first_in_group = (win == grp0);
    // decide
    const int e_d = prof_mark(c);
    // (the template's window size is the padded size of Z and Z': chosen by
    // the window size W, not by this window's own wn)
    if (c->wm == 16)
      hipLaunchKernelGGL((k_decide_wave<T, 16>), dim3(1, 1, Z), dim3(64), 0, c->stream, G, N, c->ev,
                         c->evinv, s_l, u, forced, acc, ratio, w0, wn, W,
                         first_in_group ? nullptr : c->Gs, c->sc, win, c->win_a, c->win_p, c->Xw,
                         c->Yw, zs, zn);
    else if (c->wm == 32)
      hipLaunchKernelGGL((k_decide_wave<T, 32>), dim3(1, 1, Z), dim3(64), 0, c->stream, G, N, c->ev,
                         c->evinv, s_l, u, forced, acc, ratio, w0, wn, W,
                         first_in_group ? nullptr : c->Gs, c->sc, win, c->win_a, c->win_p, c->Xw,
                         c->Yw, zs, zn);
    else
      hipLaunchKernelGGL((k_decide<T, 4, 256>), dim3(1, 1, Z), dim3(256), 0, c->stream, G, N, c->ev,
                         c->evinv, s_l, u, forced, acc, ratio, w0, wn, W,
                         first_in_group ? nullptr : c->Gs, c->sc, win, c->win_a, c->win_p, c->Xw,
                         c->Yw, zs, zn);
    const int e_e = prof_mark(c);
    prof_pair(c, PH_DECIDE, e_d, e_e);
    // extend
    const dim3 ge((N + 63) / 64, 1, Z);
    if (W <= 16)
      hipLaunchKernelGGL((k_extend<T, 16>), ge, dim3(256), 0, c->stream, G, N, Up, Wp, c->win_a, win,
                         grp0, c->Xw, c->Yw, W, w0, zs);
    else if (W <= 32)
      hipLaunchKernelGGL((k_extend<T, 32>), ge, dim3(256), 0, c->stream, G, N, Up, Wp, c->win_a, win,
                         grp0, c->Xw, c->Yw, W, w0, zs);
    else
      hipLaunchKernelGGL((k_extend<T, 64>), ge, dim3(256), 0, c->stream, G, N, Up, Wp, c->win_a, win,
                         grp0, c->Xw, c->Yw, W, w0, zs);
    const int e_x = prof_mark(c);
    prof_pair(c, PH_EXTEND, e_e, e_x);
    const bool last_in_group = (win - grp0 == c->F - 1) || (win == c->nw - 1);
    if (last_in_group) {
      dim3 grid((N + 63) / 64, (N + 63) / 64, Z);
      if constexpr (sizeof(T) == 8) {
        hipLaunchKernelGGL(k_flush_f64, grid, dim3(256), 0, c->stream, (double*)G, N,
                           (const double*)Up, (const double*)Wp, c->win_a, grp0, win + 1, zs);
      } else {
        if (c->p.prec == KDQMC_MIXED_BF16)
          hipLaunchKernelGGL(k_flush_split<__bf16>, grid, dim3(256), 0, c->stream, (float*)G, N,
                             (const float*)Up, (const float*)Wp, c->win_a, grp0, win + 1, zs);
        else
          hipLaunchKernelGGL(k_flush_split<_Float16>, grid, dim3(256), 0, c->stream, (float*)G, N,
                             (const float*)Up, (const float*)Wp, c->win_a, grp0, win + 1, zs);
      }
      prof_pair(c, PH_FLUSH, e_x, prof_mark(c));
    } else {
      const int nx = win + 1;
      const int nw0 = nx * W;
      const int nwn = std::min(W, N - nw0);
      hipLaunchKernelGGL(k_prep<T>, dim3(1, 1, Z), dim3(256), 0, c->stream, G, N, c->ev, c->evinv,
                         Up, Wp, c->win_a, grp0, win, nw0, nwn, W, c->Gs, zs);
      prof_pair(c, PH_PREP, e_x, prof_mark(c));
    }
  }
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

}  // namespace

int prepare_updates() { return KDQMC_OK; }

int launch_frame_scale(kdqmc_ctx* c, int l) {
  hipLaunchKernelGGL(k_frame_scale, dim3((c->N + 255) / 256, 1, (unsigned)c->nch), dim3(256), 0,
                     c->stream, c->fields + (size_t)(l - 1) * c->N, c->N, c->sc, c->ev, c->evinv,
                     c->zs);
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

int launch_down_reframe(kdqmc_ctx* c, int l) {
  const size_t nn = (size_t)c->N * c->N;
  const dim3 grid((unsigned)((nn + 255) / 256), 1, (unsigned)c->nch);
  const int8_t* s = c->fields + (size_t)(l - 1) * c->N;
  if (c->fp64)
    hipLaunchKernelGGL(k_down_reframe<double>, grid, dim3(256), 0, c->stream, (double*)c->G, c->N, c->ev,
                       c->evinv, s, c->sc, c->zs);
  else
    hipLaunchKernelGGL(k_down_reframe<float>, grid, dim3(256), 0, c->stream, (float*)c->G, c->N, c->ev,
                       c->evinv, s, c->sc, c->zs);
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

int run_slice_updates(kdqmc_ctx* c, int l, const double* u, const uint8_t* forced, uint8_t* acc,
                      double* ratio, size_t zn) {
  if (c->fp64) return slice_updates<double>(c, l, u, forced, acc, ratio, zn);
  return slice_updates<float>(c, l, u, forced, acc, ratio, zn);
}

}  // namespace kdqmc
