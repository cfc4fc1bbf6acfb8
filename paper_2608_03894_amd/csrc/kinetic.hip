// Kinetic propagator applied to every column (or row) of a dense N x N
// matrix through the momentum-space block form (Eq. (6)): per vector, a 2D
// L x L FFT of each sublattice component, an n x n complex block multiply per
// momentum (n = S sublattices: 3 kagome, 1 triangular, 2 honeycomb; Eq. (4)
// and App. A), and the inverse 2D FFT.  Two real vectors travel as one
// complex vector (the operator is real, so the real and imaginary parts do
// not mix).
//
// One workgroup owns P complex vectors (2P real columns or rows), staged in
// LDS as separate real/imaginary planes [slot][vector]; the FFT lines are
// processed in registers, one line per thread.  Element e = (x1 L + x2) S + s
// sits in slot e + x1: every x1 row of S L elements is padded by one slot, so
// that the lanes of an x2-direction stage (one x1 row each, S L + 1 slots
// apart) spread over the LDS banks instead of sharing one.
#include "common.h"

namespace kdqmc {

// ---------------------------------------------------------------------------
// In-register mixed-radix FFT (decimation in time), twiddles from the
// compile-time table kTw<N>.  SIGN = -1: forward exp(-2 pi i nk/N); +1: inverse
// (both unnormalized).
// ---------------------------------------------------------------------------
template <typename T, int R, int SIGN>
struct SmallDFT;

template <typename T, int SIGN>
struct SmallDFT<T, 2, SIGN> {
  __device__ __forceinline__ static void run(T* re, T* im) {
    const T r0 = re[0] + re[1], i0 = im[0] + im[1];
    re[1] = re[0] - re[1];
    im[1] = im[0] - im[1];
    re[0] = r0;
    im[0] = i0;
  }
};

template <typename T, int SIGN>
struct SmallDFT<T, 3, SIGN> {
  __device__ __forceinline__ static void run(T* re, T* im) {
    const T h = T(SIGN * 0.86602540378443864676372317075293618);  // SIGN sin(2 pi/3)
    const T tr = re[1] + re[2], ti = im[1] + im[2];
    const T dr = re[1] - re[2], di = im[1] - im[2];
    const T mr = re[0] - T(0.5) * tr, mi = im[0] - T(0.5) * ti;
    re[0] += tr;
    im[0] += ti;
    re[1] = mr - h * di;
    im[1] = mi + h * dr;
    re[2] = mr + h * di;
    im[2] = mi - h * dr;
  }
};

template <typename T, int SIGN>
struct SmallDFT<T, 4, SIGN> {
  __device__ __forceinline__ static void run(T* re, T* im) {
    const T t0r = re[0] + re[2], t0i = im[0] + im[2];
    const T t1r = re[0] - re[2], t1i = im[0] - im[2];
    const T t2r = re[1] + re[3], t2i = im[1] + im[3];
    const T t3r = re[1] - re[3], t3i = im[1] - im[3];
    re[0] = t0r + t2r;
    im[0] = t0i + t2i;
    re[2] = t0r - t2r;
    im[2] = t0i - t2i;
    // X1 = t1 + SIGN i t3, X3 = t1 - SIGN i t3
    re[1] = t1r - T(SIGN) * t3i;
    im[1] = t1i + T(SIGN) * t3r;
    re[3] = t1r + T(SIGN) * t3i;
    im[3] = t1i - T(SIGN) * t3r;
  }
};

template <typename T, int SIGN>
struct SmallDFT<T, 5, SIGN> {
  __device__ __forceinline__ static void run(T* re, T* im) {
    const T c1 = T(kTw<5>.c[1]), c2 = T(kTw<5>.c[2]);
    const T s1 = T(SIGN * kTw<5>.s[1]), s2 = T(SIGN * kTw<5>.s[2]);
    const T t1r = re[1] + re[4], t1i = im[1] + im[4];
    const T t2r = re[2] + re[3], t2i = im[2] + im[3];
    const T t3r = re[1] - re[4], t3i = im[1] - im[4];
    const T t4r = re[2] - re[3], t4i = im[2] - im[3];
    const T ar = re[0] + c1 * t1r + c2 * t2r, ai = im[0] + c1 * t1i + c2 * t2i;
    const T br = re[0] + c2 * t1r + c1 * t2r, bi = im[0] + c2 * t1i + c1 * t2i;
    // i * (s1 t3 + s2 t4) and i * (s2 t3 - s1 t4)
    const T pr = s1 * t3r + s2 * t4r, pi = s1 * t3i + s2 * t4i;
    const T qr = s2 * t3r - s1 * t4r, qi = s2 * t3i - s1 * t4i;
    re[0] = re[0] + t1r + t2r;
    im[0] = im[0] + t1i + t2i;
    re[1] = ar - pi;
    im[1] = ai + pr;
    re[4] = ar + pi;
    im[4] = ai - pr;
    re[2] = br - qi;
    im[2] = bi + qr;
    re[3] = br + qi;
    im[3] = bi - qr;
  }
};

constexpr int pick_radix(int n) {
  return (n % 4 == 0) ? 4 : (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : (n % 5 == 0) ? 5 : 0;
}

template <typename T, int N, int SIGN>
struct FFT {
  static constexpr int R = pick_radix(N);
  static_assert(R != 0, "FFT length must factor into 2, 3 and 5");
  static constexpr int M = N / R;
  __device__ __forceinline__ static void run(T* re, T* im) {
    if constexpr (M == 1) {
      SmallDFT<T, R, SIGN>::run(re, im);
    } else {
      T yr[R][M], yi[R][M];
#pragma unroll
      for (int n1 = 0; n1 < R; ++n1)
#pragma unroll
        for (int n2 = 0; n2 < M; ++n2) {
          yr[n1][n2] = re[R * n2 + n1];
          yi[n1][n2] = im[R * n2 + n1];
        }
#pragma unroll
      for (int n1 = 0; n1 < R; ++n1) FFT<T, M, SIGN>::run(yr[n1], yi[n1]);
#pragma unroll
      for (int k2 = 0; k2 < M; ++k2) {
        T tr[R], ti[R];
#pragma unroll
        for (int n1 = 0; n1 < R; ++n1) {
          const int e = (n1 * k2) % N;
          if (e == 0) {
            tr[n1] = yr[n1][k2];
            ti[n1] = yi[n1][k2];
          } else {
            const T cw = T(kTw<N>.c[e]);
            const T sw = T(SIGN * kTw<N>.s[e]);
            tr[n1] = yr[n1][k2] * cw - yi[n1][k2] * sw;
            ti[n1] = yr[n1][k2] * sw + yi[n1][k2] * cw;
          }
        }
        SmallDFT<T, R, SIGN>::run(tr, ti);
#pragma unroll
        for (int k1 = 0; k1 < R; ++k1) {
          re[k2 + M * k1] = tr[k1];
          im[k2 + M * k1] = ti[k1];
        }
      }
    }
  }
};

// LDS slot of element e (row x1 = e / (S L) padded by one slot).
template <int L, int S>
__device__ __forceinline__ int slot_of(int e) {
  return e + e / (S * L);
}

// One FFT stage over all lines of the tile: line (a, s, c) for a in [0, L),
// s in [0, S), c in [0, P): slots base(a, s) + m * stride, m in [0, L).
// AXIS == 2: lines along x2 (a = x1, stride S); AXIS == 1: along x1 (a = x2,
// stride S L + 1, the padded row).
template <typename T, int L, int S, int AXIS, int SIGN>
__device__ __forceinline__ void fft_stage(T* sre, T* sim, int P) {
  const int nlines = S * L * P;
  for (int idx = threadIdx.x; idx < nlines; idx += blockDim.x) {
    const int c = idx % P;
    const int q = idx / P;  // q = a*S + s
    const int s = q % S;
    const int a = q / S;
    const int base = (AXIS == 2) ? (a * (S * L + 1) + s) : (a * S + s);
    constexpr int stride = (AXIS == 2) ? S : S * L + 1;
    T re[L], im[L];
#pragma unroll
    for (int m = 0; m < L; ++m) {
      re[m] = sre[(base + m * stride) * P + c];
      im[m] = sim[(base + m * stride) * P + c];
    }
    FFT<T, L, SIGN>::run(re, im);
#pragma unroll
    for (int m = 0; m < L; ++m) {
      sre[(base + m * stride) * P + c] = re[m];
      sim[(base + m * stride) * P + c] = im[m];
    }
  }
}

// Per momentum k and vector c: (x_0 .. x_{S-1}) <- T(k) (x_0 .. x_{S-1}).
template <typename T, int L, int S>
__device__ __forceinline__ void mix_stage(T* sre, T* sim, int P, const T* __restrict__ tab) {
  const int nitems = L * L * P;
  for (int idx = threadIdx.x; idx < nitems; idx += blockDim.x) {
    const int c = idx % P;
    const int k = idx / P;
    const T* tk = tab + 2 * S * S * k;
    const int b = (k / L) * (S * L + 1) + S * (k % L);  // slot of (k, s = 0)
    T xr[S], xi[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      xr[s] = sre[(b + s) * P + c];
      xi[s] = sim[(b + s) * P + c];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      T yr = T(0), yi = T(0);
#pragma unroll
      for (int t = 0; t < S; ++t) {
        const T ar = tk[2 * (S * s + t)], ai = tk[2 * (S * s + t) + 1];
        yr += ar * xr[t] - ai * xi[t];
        yi += ar * xi[t] + ai * xr[t];
      }
      sre[(b + s) * P + c] = yr;
      sim[(b + s) * P + c] = yi;
    }
  }
}

// Loads of the tile, B items per thread in flight at a time: item indices
// are clamped into range (an item past the end repeats the last item, whose
// value it writes again to the same slot) and values of vectors past the
// ragged tail replaced by zeros, so no branch separates one load from the next.  HE / HV: scale by pre_e[e] (element)
// and pre_v[v] (vector) on the way in.
constexpr int kWrapBatch = 16;

template <typename T, int L, int S, bool COLS, bool HE, bool HV>
__device__ __forceinline__ void load_tile(const T* __restrict__ A, int lda, int P, int vbase,
                                          int nreal, const double* __restrict__ pre_e,
                                          const double* __restrict__ pre_v, T* sre, T* sim) {
  constexpr int NS = S * L * L;
  constexpr int B = kWrapBatch;
  const int nt = blockDim.x;
  if constexpr (COLS) {
    // item (e, j): column vbase + j of row e; the 2P columns of a row are
    // read by consecutive lanes (one contiguous segment per row)
    const int w = 2 * P;
    const int total = NS * w;
    for (int base = threadIdx.x; base < total; base += B * nt) {
      T x[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int idx = min(base + k * nt, total - 1);
        const int j = idx % w, e = idx / w;
        const int v = vbase + min(j, nreal - 1);
        const T a = A[(size_t)e * lda + v];
        T y = a;
        if constexpr (HE || HV)
          y = T(double(a) * (HE ? pre_e[e] : 1.0) * (HV ? pre_v[v] : 1.0));
        x[k] = j < nreal ? y : T(0);
      }
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int idx = min(base + k * nt, total - 1);
        const int j = idx % w, e = idx / w;
        ((j & 1) ? sim : sre)[slot_of<L, S>(e) * P + (j >> 1)] = x[k];
      }
    }
  } else {
    // item (r, e): element e of real vector r (contiguous in e)
    const int total = NS * 2 * P;
    for (int base = threadIdx.x; base < total; base += B * nt) {
      T x[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int idx = min(base + k * nt, total - 1);
        const int e = idx % NS, r = idx / NS;
        const int v = vbase + min(r, nreal - 1);
        const T a = A[(size_t)v * lda + e];
        T y = a;
        if constexpr (HE || HV)
          y = T(double(a) * (HE ? pre_e[e] : 1.0) * (HV ? pre_v[v] : 1.0));
        x[k] = r < nreal ? y : T(0);
      }
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int idx = min(base + k * nt, total - 1);
        const int e = idx % NS, r = idx / NS;
        ((r & 1) ? sim : sre)[slot_of<L, S>(e) * P + (r >> 1)] = x[k];
      }
    }
  }
}

// Stores of the tile (LDS reads batched ahead of the stores, clamped item
// indices as in load_tile: a repeated last item stores the same value again);
// HP: scale by post_e[e] on the way out.
template <typename T, int L, int S, bool COLS, bool HP>
__device__ __forceinline__ void store_tile(T* __restrict__ A, int lda, int P, int vbase, int nreal,
                                           const double* __restrict__ post_e, const T* sre,
                                           const T* sim) {
  constexpr int NS = S * L * L;
  constexpr int B = kWrapBatch;
  const int nt = blockDim.x;
  if constexpr (COLS) {
    const int w = 2 * P;
    const int total = NS * w;
    for (int base = threadIdx.x; base < total; base += B * nt) {
      T x[B];
      double se[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int idx = min(base + k * nt, total - 1);
        const int j = idx % w, e = idx / w, so = slot_of<L, S>(e);
        x[k] = (j & 1) ? sim[so * P + (j >> 1)] : sre[so * P + (j >> 1)];
        se[k] = HP ? post_e[e] : 1.0;
      }
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int idx = min(base + k * nt, total - 1);
        const int j = idx % w, e = idx / w;
        if (j < nreal) A[(size_t)e * lda + vbase + j] = HP ? T(double(x[k]) * se[k]) : x[k];
      }
    }
  } else {
    const int total = NS * 2 * P;
    for (int base = threadIdx.x; base < total; base += B * nt) {
      T x[B];
      double se[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int idx = min(base + k * nt, total - 1);
        const int e = idx % NS, r = idx / NS, so = slot_of<L, S>(e);
        x[k] = (r & 1) ? sim[so * P + (r >> 1)] : sre[so * P + (r >> 1)];
        se[k] = HP ? post_e[e] : 1.0;
      }
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int idx = min(base + k * nt, total - 1);
        const int e = idx % NS, r = idx / NS;
        if (r < nreal) A[(size_t)(vbase + r) * lda + e] = HP ? T(double(x[k]) * se[k]) : x[k];
      }
    }
  }
}

template <typename T, int L, int S, bool COLS>
__global__ void __launch_bounds__(512)
k_kinetic(T* __restrict__ A, int lda, int P, int nvec, const T* __restrict__ tab,
          const double* __restrict__ pre_e, const double* __restrict__ pre_v,
          const double* __restrict__ post_e, size_t zs) {
  constexpr int NS = S * L * L;
  A = zw(A, zs);
  tab = zw(tab, zs);
  pre_e = zw(pre_e, zs);
  pre_v = zw(pre_v, zs);
  post_e = zw(post_e, zs);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sre = reinterpret_cast<T*>(smem_raw);
  constexpr int NSP = NS + L;  // padded slots
  T* sim = sre + NSP * P;
  // Workgroups are dealt to the 8 XCDs in turn (by linear id, so by
  // blockIdx.x % 8 within every chain); tile t is renumbered so that each XCD
  // owns a contiguous range of vectors and the column pass's short row
  // segments of neighbouring tiles meet in the same L2.
  const int gx = gridDim.x, xk = blockIdx.x % 8, xq = gx / 8, xr = gx % 8;
  const int tile = xk * xq + min(xk, xr) + blockIdx.x / 8;
  const int vbase = 2 * tile * P;              // first real vector of this workgroup
  const int nreal = min(2 * P, nvec - vbase);  // real vectors present (ragged tail)

  if (pre_e) {
    if (pre_v)
      load_tile<T, L, S, COLS, true, true>(A, lda, P, vbase, nreal, pre_e, pre_v, sre, sim);
    else
      load_tile<T, L, S, COLS, true, false>(A, lda, P, vbase, nreal, pre_e, pre_v, sre, sim);
  } else {
    if (pre_v)
      load_tile<T, L, S, COLS, false, true>(A, lda, P, vbase, nreal, pre_e, pre_v, sre, sim);
    else
      load_tile<T, L, S, COLS, false, false>(A, lda, P, vbase, nreal, pre_e, pre_v, sre, sim);
  }
  __syncthreads();
  fft_stage<T, L, S, 2, -1>(sre, sim, P);
  __syncthreads();
  fft_stage<T, L, S, 1, -1>(sre, sim, P);
  __syncthreads();
  mix_stage<T, L, S>(sre, sim, P, tab);
  __syncthreads();
  fft_stage<T, L, S, 1, +1>(sre, sim, P);
  __syncthreads();
  fft_stage<T, L, S, 2, +1>(sre, sim, P);
  __syncthreads();
  if (post_e)
    store_tile<T, L, S, COLS, true>(A, lda, P, vbase, nreal, post_e, sre, sim);
  else
    store_tile<T, L, S, COLS, false>(A, lda, P, vbase, nreal, post_e, sre, sim);
}

namespace {

template <typename T, int L, int S>
int launch_L(kdqmc_ctx* c, T* A, int lda, bool cols, const T* tab, const double* pre_e,
             const double* pre_v, const double* post_e, int nvec) {
  constexpr int NS = S * L * L;
  if (nvec <= 0 || nvec > NS) nvec = NS;
  int P = (sizeof(T) == 8) ? c->P64 : c->P;
  if (P <= 0) P = 1;
  const size_t lds = size_t(2) * (NS + L) * P * sizeof(T);
  if (lds > 160 * 1024)
    return set_error(KDQMC_EINVAL, "fft_tile too large for LDS");
  const int ncomplex = (nvec + 1) / 2;
  const int grid = (ncomplex + P - 1) / P;
  int threads = S * L * P;
  threads = ((threads + 63) / 64) * 64;
  if (threads > 512) threads = 512;
  if (threads < 64) threads = 64;
  const int e0 = prof_mark(c);
  if (cols)
    hipLaunchKernelGGL((k_kinetic<T, L, S, true>), dim3(grid, 1, c->nch), dim3(threads), lds, c->stream, A, lda,
                       P, nvec, tab, pre_e, pre_v, post_e, c->zs);
  else
    hipLaunchKernelGGL((k_kinetic<T, L, S, false>), dim3(grid, 1, c->nch), dim3(threads), lds, c->stream, A, lda,
                       P, nvec, tab, pre_e, pre_v, post_e, c->zs);
  prof_pair(c, (sizeof(T) == 8 && tab == (const T*)c->tab_mu64) ? PH_BMUL : (cols ? PH_WRAP_COLS : PH_WRAP_ROWS), e0, prof_mark(c));
  KDQMC_HIP(hipGetLastError());
  return KDQMC_OK;
}

template <typename T, int L, int S>
int prepare_L() {
  KDQMC_HIP(hipFuncSetAttribute((const void*)k_kinetic<T, L, S, true>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  KDQMC_HIP(hipFuncSetAttribute((const void*)k_kinetic<T, L, S, false>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  return KDQMC_OK;
}

// The lattice sizes compiled in (FFT lengths of radices 2, 3, 4, 5), for S
// sublattices.
#define KDQMC_FOR_L(MACRO, S) \
  case 3: MACRO(3, S); case 6: MACRO(6, S); case 9: MACRO(9, S); case 12: MACRO(12, S); \
  case 15: MACRO(15, S); case 18: MACRO(18, S); case 24: MACRO(24, S);

template <typename T, int S>
int prepare_s(int L) {
#define PREP(LL, SS) return prepare_L<T, LL, SS>()
  switch (L) {
    KDQMC_FOR_L(PREP, S)
    default: return set_error(KDQMC_EUNSUPPORTED, "lattice size not compiled in");
  }
#undef PREP
}

template <typename T>
int prepare_any(int L, int S) {
  if (S == 1) return prepare_s<T, 1>(L);
  if (S == 2) return prepare_s<T, 2>(L);
  return prepare_s<T, 3>(L);
}

template <typename T, int S>
int launch_s(kdqmc_ctx* c, T* A, int lda, bool cols, const T* tab, const double* pre_e,
             const double* pre_v, const double* post_e, int nvec) {
#define LAUNCH(LL, SS) return launch_L<T, LL, SS>(c, A, lda, cols, tab, pre_e, pre_v, post_e, nvec)
  switch (c->L) {
    KDQMC_FOR_L(LAUNCH, S)
    default: return set_error(KDQMC_EUNSUPPORTED, "lattice size not compiled in");
  }
#undef LAUNCH
}

template <typename T>
int launch_any(kdqmc_ctx* c, T* A, int lda, bool cols, const T* tab, const double* pre_e,
               const double* pre_v, const double* post_e, int nvec) {
  if (c->nsub == 1) return launch_s<T, 1>(c, A, lda, cols, tab, pre_e, pre_v, post_e, nvec);
  if (c->nsub == 2) return launch_s<T, 2>(c, A, lda, cols, tab, pre_e, pre_v, post_e, nvec);
  return launch_s<T, 3>(c, A, lda, cols, tab, pre_e, pre_v, post_e, nvec);
}

}  // namespace

// Raises the dynamic-LDS limit of the kinetic kernels of this lattice size
// and sublattice count (done once at context creation, outside any graph
// capture).
int prepare_kinetic(int L, int nsub) {
  KDQMC_TRY(prepare_any<double>(L, nsub));
  return prepare_any<float>(L, nsub);
}

int launch_kinetic_f64(kdqmc_ctx* c, double* A, int lda, bool cols, const double* tab,
                       const double* pre_e, const double* pre_v, const double* post_e, int nvec) {
  return launch_any<double>(c, A, lda, cols, tab, pre_e, pre_v, post_e, nvec);
}

int launch_kinetic_f32(kdqmc_ctx* c, float* A, int lda, bool cols, const float* tab,
                       const double* pre_e, const double* pre_v, const double* post_e, int nvec) {
  return launch_any<float>(c, A, lda, cols, tab, pre_e, pre_v, post_e, nvec);
}

}  // namespace kdqmc
