// Shared declarations of the kdqmc HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/kdqmc.h"

namespace kdqmc {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
int set_error(int code, const std::string& msg);
void clear_error();

#define KDQMC_HIP(call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::kdqmc::set_error(KDQMC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define KDQMC_TRY(call)        \
  do {                         \
    int r_ = (call);           \
    if (r_ != KDQMC_OK) return r_; \
  } while (0)

// ---------------------------------------------------------------------------
// Compile-time trigonometry for FFT twiddles: cos/sin(2 pi e / n) by exact
// quadrant reduction of the rational angle and a Taylor series on
// |phi| <= pi/4 (error below 1 ulp of double after rounding).
// ---------------------------------------------------------------------------
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 16; ++k) {
    term *= -x2 / double((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}

constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 16; ++k) {
    term *= -x2 / double((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}

// returns {cos, sin} of 2 pi e / n as a pair via two functions
constexpr long mod_pos(long a, long n) { return ((a % n) + n) % n; }

// The padded window size of the decision kernels (16, 32 or 64): Z, Z' and the
// window snapshots are stored with this stride, zero past the window.
constexpr int window_pad(int w) { return w <= 16 ? 16 : (w <= 32 ? 32 : 64); }

constexpr double cos2pi(long e, long n) {
  const long ee = mod_pos(e, n);
  const long q = (4 * ee + n / 2) / n;  // nearest quarter turn
  const long r = 4 * ee - q * n;        // |r| <= n/2
  const double phi = (kPi / 2) * double(r) / double(n);
  const double c = taylor_cos(phi), s = taylor_sin(phi);
  switch (q & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
  }
}

constexpr double sin2pi(long e, long n) {
  const long ee = mod_pos(e, n);
  const long q = (4 * ee + n / 2) / n;
  const long r = 4 * ee - q * n;
  const double phi = (kPi / 2) * double(r) / double(n);
  const double c = taylor_cos(phi), s = taylor_sin(phi);
  switch (q & 3) {
    case 0: return s;
    case 1: return c;
    case 2: return -s;
    default: return -c;
  }
}

template <int N>
struct TwiddleTable {
  double c[N];
  double s[N];
  constexpr TwiddleTable() : c(), s() {
    for (int e = 0; e < N; ++e) {
      c[e] = cos2pi(e, N);
      s[e] = sin2pi(e, N);
    }
  }
};

template <int N>
inline constexpr TwiddleTable<N> kTw{};

// ---------------------------------------------------------------------------
// Batched chains.  A context may hold nch chains of one shape (same L, L_tau
// and schedule; U may differ).  Every launch then has gridDim.z = nch and
// chain z = blockIdx.z works on its own copy of the workspace, zs bytes after
// chain z-1's: kernels receive chain 0's workspace pointers and shift them
// with zw().  Caller arrays hold one record per chain, zn elements apart,
// shifted with zc().  Null pointers stay null.
// ---------------------------------------------------------------------------
// (byte arithmetic on a char pointer, not on an integer: the compiler then
// still knows the result points to global memory and emits global loads)
template <typename T>
__device__ __forceinline__ T* zw(T* p, size_t zs) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p ? reinterpret_cast<T*>(reinterpret_cast<B*>(p) + (size_t)blockIdx.z * zs) : p;
}
template <typename T>
__device__ __forceinline__ T* zc(T* p, size_t zn) {
  return p ? p + (size_t)blockIdx.z * zn : p;
}
// The same for an explicit chain z (kernels that number their workgroups themselves).
template <typename T>
__device__ __forceinline__ T* zw_at(T* p, size_t zs, int z) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p ? reinterpret_cast<T*>(reinterpret_cast<B*>(p) + (size_t)z * zs) : p;
}
template <typename T>
__device__ __forceinline__ T* zc_at(T* p, size_t zn, int z) {
  return p ? p + (size_t)z * zn : p;
}

// 1/sqrt(x) and 1/x for normal positive (resp. nonzero) x: the hardware
// estimates refined by two Newton steps each (the estimates are good to about 2^-24
// and the error squares per step).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Wave-level ordering of LDS accesses (LDS writes and reads within one wave;
// a wave's LDS operations complete in order, the fences keep the compiler
// from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Lane `src` (wave-uniform) of a double held in a vector register; the value
// is wave-uniform afterwards (scalar registers).
__device__ __forceinline__ double lane_value(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Per-chain scalars kept in the workspace (the decoupling constant differs
// between chains of a batch): exp(alpha), exp(-alpha), exp(-2 alpha), exp(2 alpha).
enum { SC_EA = 0, SC_EAINV, SC_EM2A, SC_EP2A, SC_COUNT };

// Per-chain numeric-health record (doubles in the workspace): the largest
// wrap error since the record was cleared (NaN once any was not finite), the
// number of stabilizations whose wrap error was not finite or above the
// tolerance, 1 once a column norm of a stabilization product was not finite,
// and the wrap error of the latest stabilization.
enum { HL_WORST = 0, HL_NVIOL, HL_NONFINITE, HL_LAST, HL_COUNT };

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct Layout;  // workspace carving, see api.hip

}  // namespace kdqmc

namespace kdqmc {
// Phases timed by the optional HIP-event profiler (kdqmc_profile_*).
enum Phase {
  PH_WRAP_COLS = 0, PH_WRAP_ROWS, PH_DECIDE, PH_EXTEND, PH_PREP, PH_FLUSH, PH_BMUL, PH_QR_PANEL,
  PH_GEMM, PH_STABILIZE, PH_FLUSH_DECIDE, PH_MEASURE, PH_COUNT
};
}  // namespace kdqmc

struct kdqmc_ctx {
  kdqmc_params p;
  // profiler: event pool and recorded (phase, begin, end) triples
  bool prof_on = false;
  std::vector<hipEvent_t> prof_events;
  int prof_next = 0;
  std::vector<int> prof_triples;
  // hipGraph of a whole sweep: captured on cap_stream, replayed on stream
  bool use_graphs = true;
  bool capturing = false;
  hipStream_t cap_stream = nullptr;
  // captured passes, [0] upward and [1] downward: one graph per segment
  std::vector<hipGraphExec_t> sweep_exec[2];
  const void* sweep_key[2][7] = {{nullptr}};
  std::vector<hipEvent_t> graph_events;   // events that are nodes of the captured graph
  int graph_next = 0;
  std::vector<int> graph_triples;
  double prof_acc_ms[16] = {0};
  int prof_acc_n[16] = {0};
  int N = 0, L = 0, Ltau = 0, nc = 0;     // sites, cells/side, slices, stack checkpoints
  int lattice = 0, nsub = 3;              // kdqmc_lattice, sublattices per cell
  int w = 0, nw = 0, F = 0;               // window size, windows per slice, windows per flush
  int wm = 0;                             // window_pad(w): the padded size of Z, Z' and the snapshots
  int P = 0;                              // complex vectors per wrap workgroup (storage type)
  int P64 = 0;                            // same for the FP64 stack products
  int kmax = 0;                           // columns of the pending factors (F * w)
  int nb = 32;                            // QR panel width
  double alpha = 0.0;                     // decoupling constant of chain 0
  int nch = 1;                            // chains in this context
  size_t zs = 0;                          // workspace bytes per chain
  double* sc = nullptr;                   // SC_COUNT per-chain scalars
  hipStream_t stream = nullptr;
  int l_cur = -1;
  bool stacks_valid = false;
  int stab_next = 1;        // index j of the next stabilization due (at slice j * n_stab)
  int dir = 0;              // pass in progress: +1 upward, -1 downward, 0 none (at slice 0)
  bool left_valid = false;  // left stack entries match the current fields
  bool right_valid = false; // right stack entries match the current fields
  bool fp64 = true;
  // projector form: n_occ trial orbitals, stacks of N x nocc panels
  bool proj = false;
  int nocc = 0;
  bool trial_set = false;
  double* Ptrial = nullptr;    // N x nocc trial orbitals (row stride N)
  double* obs_tab = nullptr;   // N x 8: phases of the measurement estimators

  // device buffers (carved from the caller's workspace)
  void* G = nullptr;           // N*N, double (FP64) or float (mixed)
  double* G64 = nullptr;       // N*N FP64: fresh G from stabilization / measure staging
  int8_t* fields = nullptr;    // Ltau*N
  double* ev = nullptr;        // N: exp(alpha s) frame scale of the current slice
  double* evinv = nullptr;     // N: exp(-alpha s)
  void* tab_m = nullptr;       // L*L*9 complex (T): exp(-dtau H(k)) / L^2
  void* tab_p = nullptr;       // L*L*9 complex (T): exp(+dtau H(k)) / L^2
  double* tab_mu64 = nullptr;  // L*L*9 complex FP64: exp(-dtau (H(k) - mu)) / L^2
  double* tab_mu64t = nullptr; // unused placeholder for symmetry
  double* tab_m64 = nullptr;   // FP64 copies (wrap tables) for FP64 helpers
  double* tab_p64 = nullptr;
  void* Upend = nullptr;       // kmax*N (T), store frame, column j contiguous over rows
  void* Wpend = nullptr;       // kmax*N (T)
  int* win_a = nullptr;        // nw: accepted count per window
  int* win_p = nullptr;        // nw*w: window-local positions of the accepts
  double* win_c = nullptr;     // nw*w: Delta/R of the accepts
  double* Xw = nullptr;        // 2*wm*wm: Z of a window by position, n-major (two buffers by parity)
  double* Yw = nullptr;        // 2*wm*wm: Z' of a window by position, n-major
  double* snapc = nullptr;     // 2*N*wm: G[:, S] of a window, row stride wm (fused schedule, by parity)
  double* snapr = nullptr;     // 2*N*wm: G[S, :] of a window stored transposed, G[s][c] at c*wm + s
  double* snapb = nullptr;     // 2*w*w: G[S, S] of the window after next
  int* ctl = nullptr;          // nw + 4 counters of the persistent slice launch
  bool persist = false;        // one resident launch per slice (single FP64 chain, small N)
  bool persist_ok = false;     // the shape allows it (1 + ceil(tiles / persist_tpw) <= compute units)
  int persist_tpw = 1;         // tiles per workgroup of the persistent launch (1..3)
  bool fused = false;          // FP64, one window per flush, windows inside 64 x 64 tiles
  double* Gs = nullptr;        // w*w: G~cur[S,S] of the next window
  int* flag = nullptr;         // small device status words
  double* err = nullptr;       // reduction scratch
  // numeric-health record (HL_* slots), cleared by set_fields / set_G / kdqmc_health
  double* health = nullptr;
  double wrap_tol = 1e-6;      // largest wrap error a stabilization accepts
  // stabilization stacks: entry j holds the UDT form of the chain up to checkpoint j
  double* RU = nullptr; double* RT = nullptr; double* RD = nullptr;
  double* LU = nullptr; double* LT = nullptr; double* LD = nullptr;
  // linear-algebra scratch (N*N each unless noted)
  double* S[8] = {nullptr};
  double* Vq = nullptr;        // N*N explicit Householder vectors
  double* Tq = nullptr;        // per-panel 32 x 32 block-reflector factors
  double* Tm = nullptr;        // the same for consecutive panel pairs merged into one
  int qr_npan = 0;             // panels of the last QR (start column, width)
  int qr_panel_start[160] = {0};
  int qr_panel_width[160] = {0};
  double* Wq = nullptr;        // 16 * 32 * N: partial V^T C products of the split WY apply
  double* tau = nullptr;       // N
  double* nrm = nullptr;       // N
  int* perm = nullptr;         // N
};

namespace kdqmc {

// ---------------------------------------------------------------------------
// Host helpers implemented in lattice.hip
// ---------------------------------------------------------------------------
bool lattice_supported(int L);
// Sublattices per cell: 3 (kagome), 1 (triangular), 2 (honeycomb).
int lattice_nsub(int lattice);
// Fills tab[L*L*S*S] complex (interleaved re, im) with exp(scale * (H(k) - shift)) / L^2.
void bloch_table(int lattice, int L, double t, double scale, double shift, double* tab);
double dirac_mu(int L, double t);
// Per-site phase table of the measurement estimators (host, tab[N * 8]).
void measure_table(int L, double* tab);
// The KDQMC_NOBS estimators of the current G into out (records zn doubles apart).
int launch_measure(kdqmc_ctx* c, double* out, size_t zn);
// Trial orbitals of the projector form into P[N * n_occ] (row-major, host).
int trial_orbitals(int L, double t, int n_occ, double eps, double* P);

// ---------------------------------------------------------------------------
// Launchers (all enqueue on c->stream)
// ---------------------------------------------------------------------------
// Vector-batched kinetic operator: for every column (cols=true) or row of the
// N x N matrix A (row stride lda): x <- post_e .* Op( pre_e .* x .* pre_v[v] ),
// with Op the table operator.  Pointers pre_e/pre_v/post_e may be null.
// nvec (> 0): only the first nvec columns (rows) are vectors.
int launch_kinetic_f64(kdqmc_ctx* c, double* A, int lda, bool cols, const double* tab,
                       const double* pre_e, const double* pre_v, const double* post_e, int nvec = 0);
int launch_kinetic_f32(kdqmc_ctx* c, float* A, int lda, bool cols, const float* tab,
                       const double* pre_e, const double* pre_v, const double* post_e, int nvec = 0);

int prepare_kinetic(int L, int nsub);
int prepare_updates();
int launch_frame_scale(kdqmc_ctx* c, int l);
// Downward pass: after the flips of slice l, G <- F G F^{-1} with
// F = diag(exp(alpha (s_old - s_new))) (ev holds exp(alpha s_old)).
int launch_down_reframe(kdqmc_ctx* c, int l);
// Caller arrays u, forced, acc, ratio: one record per chain, zn elements apart.
int run_slice_updates(kdqmc_ctx* c, int l, const double* u, const uint8_t* forced, uint8_t* acc,
                      double* ratio, size_t zn);

int gemm_f64(kdqmc_ctx* c, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
             int lda, const double* B, int ldb, double beta, double* C, int ldc);
// QR of the n x ncol matrix A (ncol <= n, row stride N); Q (n x ncol) formed
// when non-null.
int qr_f64(kdqmc_ctx* c, int n, int ncol, double* A, double* Q);
// X (n rows x ncols, row stride N) <- Q^T X for the last qr_f64.
int apply_qt_f64(kdqmc_ctx* c, int n, int ncols, double* X);
// R Y = X for upper-triangular R (n x n) and X (n x ncols), in place on X.
int trsm_upper_f64(kdqmc_ctx* c, int n, int ncols, const double* R, double* X);

int stab_identity(kdqmc_ctx* c, bool left, int j);
int stab_build_left(kdqmc_ctx* c);                  // all left entries from the current fields
int stab_build_right(kdqmc_ctx* c);                 // all right entries from the current fields
int stab_left_step(kdqmc_ctx* c, int j);            // left stack entry j from j+1
int stab_green(kdqmc_ctx* c, int j, double* out);   // G at checkpoint j into out (FP64)
int stab_right_step(kdqmc_ctx* c, int j);           // right stack entry j from j-1
// in / out may be workspace arrays (zn = 0: shifted by the workspace stride)
// or caller arrays (zn > 0: one N x N record per chain, zn elements apart).
int copy_G_to64(kdqmc_ctx* c, double* out, size_t zn = 0);
int copy_64_to_G(kdqmc_ctx* c, const double* in, size_t zn = 0);
// max |G - a| (a in the workspace) into out[0] of each chain's record (zn
// apart; out == nullptr: only into the health record), and the health record
// updated with it against c->wrap_tol.
int max_abs_diff(kdqmc_ctx* c, const double* a, int n, double* out, size_t zn);
// Zeroes every chain's health record.
int clear_health(kdqmc_ctx* c);

// Device-to-device copy of n doubles as a kernel (graph-capture friendly).
int copy_f64(kdqmc_ctx* c, double* dst, const double* src, size_t n);

// Profiler: prof_mark records an event on the stream (returns its index, or
// -1 when profiling is off); prof_pair attributes the interval to a phase.
int prof_mark(kdqmc_ctx* c);
void prof_pair(kdqmc_ctx* c, int phase, int e0, int e1);

}  // namespace kdqmc
