// C ABI of the library: parameter checks, workspace carving, slice order,
// and the composition of the kernels into the calls declared in kdqmc.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"

namespace kdqmc {

namespace {
thread_local std::string g_last_error;

struct Derived {
  int N = 0, S = 3, Ltau = 0, nc = 0, w = 0, wm = 0, nw = 0, F = 0, kmax = 0, P = 0, P64 = 0;
  bool fp64 = true, proj = false;
};

// Complex vectors per wrap workgroup: at least one workgroup per compute
// unit (256) over all chains of the context where the matrices allow, at most
// 4 (wider tiles coalesce the column pass but leave fewer workgroups), within
// 64 KB of LDS and 512 threads.
int auto_tile(int L, int S, size_t elem, int requested, int nch) {
  if (requested > 0) return requested;
  const int N = S * L * L;
  const int ncomplex = (N + 1) / 2;
  int P = std::max(1, std::min(4, (int)((size_t)nch * ncomplex / 256)));
  while (P > 1 && (2 * (size_t)(N + L) * P * elem > 64 * 1024 || S * L * P > 512)) --P;
  return P;
}

int derive(const kdqmc_params* p, Derived* d, int nch = 1) {
  if (!p) return set_error(KDQMC_EINVAL, "params is NULL");
  if (!lattice_supported(p->L))
    return set_error(KDQMC_EUNSUPPORTED, "L must be one of 3, 6, 9, 12, 15, 18, 24");
  if (p->lattice < KDQMC_KAGOME || p->lattice > KDQMC_HONEYCOMB)
    return set_error(KDQMC_EINVAL, "lattice must be KDQMC_KAGOME, KDQMC_TRIANGULAR or KDQMC_HONEYCOMB");
  if (!(std::isfinite(p->t) && std::isfinite(p->U) && std::isfinite(p->mu)))
    return set_error(KDQMC_EINVAL, "t, U, mu must be finite");
  if (p->U > 0.0)
    return set_error(KDQMC_EUNSUPPORTED, "only the attractive (U <= 0) charge-channel decoupling is built");
  if (!(p->dtau > 0.0) || !(p->beta > 0.0)) return set_error(KDQMC_EINVAL, "beta and dtau must be > 0");
  const double lt = p->beta / p->dtau;
  const int Ltau = (int)std::lround(lt);
  if (Ltau < 1 || std::fabs(Ltau - lt) > 1e-9 * lt)
    return set_error(KDQMC_EINVAL, "beta must be an integer multiple of dtau");
  if (p->n_stab < 1 || Ltau % p->n_stab != 0)
    return set_error(KDQMC_EINVAL, "n_stab must divide L_tau");
  if (Ltau / p->n_stab > 1024) return set_error(KDQMC_EINVAL, "too many stabilization checkpoints");
  if (p->n_stab > 1024) return set_error(KDQMC_EINVAL, "n_stab above 1024");
  if (p->delay_k < 1 || p->delay_k > 512) return set_error(KDQMC_EINVAL, "delay_k must be in 1..512");
  if (p->prec != KDQMC_FP64 && p->prec != KDQMC_MIXED_F16 && p->prec != KDQMC_MIXED_BF16)
    return set_error(KDQMC_EINVAL, "unknown precision");
  int w = p->window > 0 ? p->window : std::min(p->delay_k, 32);
  if (w > 64) return set_error(KDQMC_EINVAL, "window above 64");
  if (w > p->delay_k) return set_error(KDQMC_EINVAL, "window larger than delay_k");
  d->S = lattice_nsub(p->lattice);
  d->N = d->S * p->L * p->L;
  d->Ltau = Ltau;
  d->nc = Ltau / p->n_stab;
  d->w = std::min(w, d->N);
  d->wm = window_pad(d->w);
  d->nw = (d->N + d->w - 1) / d->w;
  d->F = std::max(1, p->delay_k / d->w);
  d->kmax = d->F * d->w;
  d->fp64 = (p->prec == KDQMC_FP64);
  if (p->n_occ < 0 || p->n_occ > d->N) return set_error(KDQMC_EINVAL, "n_occ must be in 0..N");
  d->proj = p->n_occ > 0;
  const size_t es = d->fp64 ? 8 : 4;
  d->P = auto_tile(p->L, d->S, es, p->fft_tile, nch);
  d->P64 = d->fp64 ? d->P : auto_tile(p->L, d->S, 8, 0, nch);
  if (2 * (size_t)(d->N + p->L) * d->P * es > 160 * 1024 || d->S * p->L * d->P > 512)
    return set_error(KDQMC_EINVAL, "fft_tile exceeds LDS or thread limits");
  return KDQMC_OK;
}

// Carves one chain's block of the workspace; with c == nullptr only
// measures.  Returns the block size (a multiple of 256 bytes).
size_t carve(const kdqmc_params* p, const Derived& d, kdqmc_ctx* c, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) & ~size_t(255);
    char* ptr = base ? base + off : nullptr;
    off += bytes;
    return ptr;
  };
  const size_t N = d.N, nn = N * N, L2 = (size_t)p->L * p->L;
  const size_t es = d.fp64 ? 8 : 4;
  const size_t nb = 16;
  char* G = take(nn * es);
  char* G64 = take(nn * 8);
  char* fields = take((size_t)d.Ltau * N);
  char* ev = take(N * 8);
  char* evinv = take(N * 8);
  char* tab_m = take(L2 * 18 * es);
  char* tab_p = take(L2 * 18 * es);
  char* tab_mu64 = take(L2 * 18 * 8);
  char* Up = take((size_t)d.kmax * N * es);
  char* Wp = take((size_t)d.kmax * N * es);
  char* win_a = take((size_t)d.nw * 4);
  char* win_p = take((size_t)d.nw * d.w * 4);
  char* Zg = take(2 * (size_t)d.wm * d.wm * 8);
  char* Zpg = take(2 * (size_t)d.wm * d.wm * 8);
  char* snapc = take(2 * N * d.wm * 8);
  char* snapr = take(2 * N * d.wm * 8);
  char* snapb = take(2 * (size_t)d.w * d.w * 8);
  char* Gs = take((size_t)d.w * d.w * 8);
  char* ctl = take((size_t)(d.nw + 4) * 4);
  char* flag = take(64);
  char* err = take(1024 * 8);
  char* health = take(HL_COUNT * 8);
  // stacks: U (and T, D) entries of N x N; the projector form keeps only the
  // panels (N x n_occ, row stride N) in U
  const size_t tmat = d.proj ? 0 : (d.nc + 1) * nn * 8;
  char* RU = take((d.nc + 1) * nn * 8);
  char* RT = take(tmat);
  char* RD = take((d.nc + 1) * N * 8);
  char* LU = take((d.nc + 1) * nn * 8);
  char* LT = take(tmat);
  char* LD = take((d.nc + 1) * N * 8);
  char* Ptr = take(d.proj ? nn * 8 : 0);
  char* obs = take(N * 8 * 8);
  char* S[8];
  for (int i = 0; i < 8; ++i) S[i] = take(nn * 8);
  char* Vq = take(nn * 8);
  // per-panel factors, then those of the merged panel pairs
  char* Tq = take((N / nb + 2 + N / (2 * nb) + 2) * 32 * 32 * 8);
  char* Wq = take((size_t)16 * 32 * N * 8);  // split WY apply: 16 row chunks of 32 x N partials
  char* tau = take(N * 8);
  char* nrm = take(2 * N * 8);
  char* perm = take(3 * N * 4);  // the pivot order, a second ranking and their composition
  char* sc = take(SC_COUNT * 8);
  if (c) {
    c->G = G;
    c->G64 = (double*)G64;
    c->fields = (int8_t*)fields;
    c->ev = (double*)ev;
    c->evinv = (double*)evinv;
    c->tab_m = tab_m;
    c->tab_p = tab_p;
    c->tab_mu64 = (double*)tab_mu64;
    c->Upend = Up;
    c->Wpend = Wp;
    c->win_a = (int*)win_a;
    c->win_p = (int*)win_p;
    c->Xw = (double*)Zg;
    c->Yw = (double*)Zpg;
    c->snapc = (double*)snapc;
    c->snapr = (double*)snapr;
    c->snapb = (double*)snapb;
    c->Gs = (double*)Gs;
    c->ctl = (int*)ctl;
    c->flag = (int*)flag;
    c->err = (double*)err;
    c->health = (double*)health;
    c->RU = (double*)RU; c->RT = (double*)RT; c->RD = (double*)RD;
    c->LU = (double*)LU; c->LT = (double*)LT; c->LD = (double*)LD;
    c->Ptrial = d.proj ? (double*)Ptr : nullptr;
    c->obs_tab = (double*)obs;
    for (int i = 0; i < 8; ++i) c->S[i] = (double*)S[i];
    c->Vq = (double*)Vq;
    c->Tq = (double*)Tq;
    c->Tm = c->Tq + (N / nb + 2) * 32 * 32;
    c->Wq = (double*)Wq;
    c->tau = (double*)tau;
    c->nrm = (double*)nrm;
    c->perm = (int*)perm;
    c->sc = (double*)sc;
  }
  return (off + 255) & ~size_t(255);
}

// Bytes for nch chains of one shape: nch blocks plus slack for aligning the base.
size_t batch_bytes(const kdqmc_params* p, const Derived& d, int nch) {
  return (size_t)nch * carve(p, d, nullptr, nullptr) + 256;
}

__global__ void k_check_fields(const int8_t* __restrict__ s, size_t n, int* __restrict__ bad) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && s[i] != 1 && s[i] != -1) atomicOr(bad, 1);
}

__global__ void k_zero_int(int* __restrict__ x, int n) {
  const int i = threadIdx.x;
  if (i < n) x[i] = 0;
}

int check_ctx(const kdqmc_ctx* c) {
  if (!c) return set_error(KDQMC_EINVAL, "context is NULL");
  return KDQMC_OK;
}

}  // namespace

int prof_mark(kdqmc_ctx* c) {
  if (!c->prof_on) return -1;
  std::vector<hipEvent_t>& pool = c->capturing ? c->graph_events : c->prof_events;
  int& next = c->capturing ? c->graph_next : c->prof_next;
  if (next == (int)pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    pool.push_back(e);
  }
  const int i = next++;
  if (hipEventRecord(pool[i], c->stream) != hipSuccess) return -1;
  return i;
}

void prof_pair(kdqmc_ctx* c, int phase, int e0, int e1) {
  if (!c->prof_on || e0 < 0 || e1 < 0) return;
  std::vector<int>& t = c->capturing ? c->graph_triples : c->prof_triples;
  t.push_back(phase);
  t.push_back(e0);
  t.push_back(e1);
}

// Adds the elapsed times of recorded (phase, e0, e1) triples to the accumulators.
static int prof_accumulate(kdqmc_ctx* c, const std::vector<hipEvent_t>& pool, const std::vector<int>& t) {
  for (size_t q = 0; q + 2 < t.size(); q += 3) {
    float ms = 0.0f;
    KDQMC_HIP(hipEventElapsedTime(&ms, pool[t[q + 1]], pool[t[q + 2]]));
    c->prof_acc_ms[t[q]] += ms;
    c->prof_acc_n[t[q]] += 1;
  }
  return KDQMC_OK;
}

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}
void clear_error() { g_last_error.clear(); }

}  // namespace kdqmc

using namespace kdqmc;

extern "C" {

size_t kdqmc_workspace_bytes(const kdqmc_params* p) { return kdqmc_workspace_bytes_batch(p, 1); }

size_t kdqmc_workspace_bytes_batch(const kdqmc_params* p, int n_chains) {
  if (n_chains < 1 || n_chains > 65535) {
    set_error(KDQMC_EINVAL, "n_chains must be in 1..65535");
    return 0;
  }
  Derived d;
  if (derive(p, &d) != KDQMC_OK) return 0;
  return batch_bytes(p, d, n_chains);
}

double kdqmc_dirac_mu(int L, double t) { return kdqmc::dirac_mu(L, t); }

int kdqmc_trial_orbitals(int L, double t, int n_occ, double eps, double* P_host) {
  if (!lattice_supported(L)) return set_error(KDQMC_EUNSUPPORTED, "L must be one of 3, 6, 9, 12, 15, 18, 24");
  if (!P_host) return set_error(KDQMC_EINVAL, "P is NULL");
  if (!(std::isfinite(t) && std::isfinite(eps))) return set_error(KDQMC_EINVAL, "t, eps must be finite");
  return trial_orbitals(L, t, n_occ, eps, P_host);
}

int kdqmc_set_trial(kdqmc_ctx* c, const double* P_dev) {
  KDQMC_TRY(check_ctx(c));
  if (!c->proj) return set_error(KDQMC_EINVAL, "not a projector context (params.n_occ == 0)");
  if (!P_dev) return set_error(KDQMC_EINVAL, "P is NULL");
  // chain z's record at P_dev + z N n_occ, into its workspace copy (row stride N)
  const size_t w = (size_t)c->nocc * sizeof(double);
  for (int z = 0; z < c->nch; ++z)
    KDQMC_HIP(hipMemcpy2DAsync(reinterpret_cast<char*>(c->Ptrial) + (size_t)z * c->zs, (size_t)c->N * sizeof(double),
                               P_dev + (size_t)z * c->N * c->nocc, w, w, c->N, hipMemcpyDeviceToDevice, c->stream));
  c->trial_set = true;
  c->stacks_valid = false;
  c->l_cur = -1;
  return KDQMC_OK;
}

int kdqmc_init_lattice(kdqmc_ctx** out, const kdqmc_params* p, void* workspace_dev,
                       size_t workspace_bytes, void* hip_stream) {
  return kdqmc_init_batch(out, p, 1, nullptr, workspace_dev, workspace_bytes, hip_stream);
}

int kdqmc_init_batch(kdqmc_ctx** out, const kdqmc_params* p, int n_chains, const double* U_host,
                     void* workspace_dev, size_t workspace_bytes, void* hip_stream) {
  if (!out) return set_error(KDQMC_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_chains < 1 || n_chains > 65535) return set_error(KDQMC_EINVAL, "n_chains must be in 1..65535");
  Derived d;
  KDQMC_TRY(derive(p, &d, n_chains));
  std::vector<double> Uc(n_chains, p->U);
  if (U_host) {
    for (int z = 0; z < n_chains; ++z) {
      kdqmc_params q = *p;
      q.U = U_host[z];
      Derived dq;
      KDQMC_TRY(derive(&q, &dq));
      Uc[z] = U_host[z];
    }
  }
  if (!workspace_dev) return set_error(KDQMC_EINVAL, "workspace is NULL");
  const size_t need = batch_bytes(p, d, n_chains);
  if (workspace_bytes < need)
    return set_error(KDQMC_ENOSPACE, "workspace smaller than kdqmc_workspace_bytes_batch()");
  KDQMC_TRY(prepare_kinetic(p->L, d.S));
  KDQMC_TRY(prepare_updates());
  kdqmc_ctx* c = new kdqmc_ctx();
  c->p = *p;
  c->N = d.N;
  c->L = p->L;
  c->lattice = p->lattice;
  c->nsub = d.S;
  c->Ltau = d.Ltau;
  c->nc = d.nc;
  c->w = d.w;
  c->wm = d.wm;
  c->nw = d.nw;
  c->F = d.F;
  // the fused window launch for one chain; batched chains (whose shape groups
  // run on concurrent streams, hiding launch gaps) take the three-kernel
  // schedule, which forms each window's factors once instead of per tile
  c->fused = d.fp64 && d.F == 1 && d.w <= 32 && (64 % d.w == 0 || d.nw == 1) && n_chains == 1;
  // the persistent slice launch needs every workgroup resident, at most one
  // per compute unit: the decider and the tile workgroups
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) {
      // one 64 x 64 tile per workgroup where they fit, else two or three
      const int T = ((d.N + 63) / 64) * ((d.N + 63) / 64);
      int tpw = 1;
      while (tpw < 3 && 1 + (T + tpw - 1) / tpw > cus) ++tpw;
      c->persist_tpw = tpw;
      c->persist_ok = c->fused && 1 + (T + tpw - 1) / tpw <= cus;
    }
    c->persist = c->persist_ok;
  }
  c->kmax = d.kmax;
  c->P = d.P;
  c->P64 = d.P64;
  c->nb = 16;
  c->fp64 = d.fp64;
  c->proj = d.proj;
  c->nocc = p->n_occ;
  c->alpha = std::acosh(std::exp(p->dtau * std::fabs(Uc[0]) / 2.0));
  c->wrap_tol = d.fp64 ? 1e-5 : 1e-4;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->nch = n_chains;
  char* base = static_cast<char*>(workspace_dev);
  base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(base) + 255) & ~uintptr_t(255));
  c->zs = carve(p, d, c, base);
  // Bloch tables: exp(-dtau H(k)) and exp(+dtau H(k)) for the wrap (mu cancels),
  // exp(-dtau (H(k) - mu)) for the B-chains; 1/L^2 folded in.
  const size_t L2 = (size_t)p->L * p->L;
  std::vector<double> tm(L2 * 18), tp(L2 * 18), tmu(L2 * 18), otab((size_t)d.N * 8);
  if (p->lattice == KDQMC_KAGOME) measure_table(p->L, otab.data());  // (kagome estimators only)
  bloch_table(p->lattice, p->L, p->t, -p->dtau, 0.0, tm.data());
  bloch_table(p->lattice, p->L, p->t, +p->dtau, 0.0, tp.data());
  bloch_table(p->lattice, p->L, p->t, -p->dtau, p->mu, tmu.data());
  int rc = KDQMC_OK;
  auto upload = [&](void* dst, const std::vector<double>& src, bool as_float) -> int {
    if (as_float) {
      std::vector<float> f(src.begin(), src.end());
      KDQMC_HIP(hipMemcpyAsync(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice, c->stream));
      KDQMC_HIP(hipStreamSynchronize(c->stream));
    } else {
      KDQMC_HIP(hipMemcpyAsync(dst, src.data(), src.size() * 8, hipMemcpyHostToDevice, c->stream));
      KDQMC_HIP(hipStreamSynchronize(c->stream));
    }
    return KDQMC_OK;
  };
  // every chain holds its own copy of the tables and its decoupling scalars
  for (int z = 0; z < n_chains && rc == KDQMC_OK; ++z) {
    const size_t o = (size_t)z * c->zs;
    const double a = std::acosh(std::exp(p->dtau * std::fabs(Uc[z]) / 2.0));
    std::vector<double> scv(SC_COUNT);
    scv[SC_EA] = std::exp(a);
    scv[SC_EAINV] = std::exp(-a);
    scv[SC_EM2A] = std::exp(-2.0 * a);
    scv[SC_EP2A] = std::exp(2.0 * a);
    if ((rc = upload(static_cast<char*>(c->tab_m) + o, tm, !c->fp64)) != KDQMC_OK ||
        (rc = upload(static_cast<char*>(c->tab_p) + o, tp, !c->fp64)) != KDQMC_OK ||
        (rc = upload(reinterpret_cast<char*>(c->tab_mu64) + o, tmu, false)) != KDQMC_OK ||
        (rc = upload(reinterpret_cast<char*>(c->sc) + o, scv, false)) != KDQMC_OK ||
        (rc = upload(reinterpret_cast<char*>(c->obs_tab) + o, otab, false)) != KDQMC_OK)
      break;
  }
  if (rc == KDQMC_OK) rc = clear_health(c);
  if (rc == KDQMC_OK) {
    // the window snapshots are read whole (padding included) and multiplied
    // by exact zeros there, so they must never hold non-finite bit patterns
    const size_t sb = 2 * (size_t)d.N * d.wm * 8;
    if (hipMemset2DAsync(c->snapc, c->zs, 0, sb, n_chains, c->stream) != hipSuccess ||
        hipMemset2DAsync(c->snapr, c->zs, 0, sb, n_chains, c->stream) != hipSuccess ||
        hipMemset2DAsync(c->ctl, c->zs, 0, (size_t)(d.nw + 4) * 4, n_chains, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      rc = set_error(KDQMC_EHIP, "clearing the window snapshots and counters failed");
  }
  if (rc != KDQMC_OK) {
    delete c;
    return rc;
  }
  c->l_cur = -1;
  c->stacks_valid = false;
  *out = c;
  clear_error();
  return KDQMC_OK;
}

int kdqmc_set_fields(kdqmc_ctx* c, const int8_t* s_dev) {
  KDQMC_TRY(check_ctx(c));
  if (!s_dev) return set_error(KDQMC_EINVAL, "fields pointer is NULL");
  if (c->proj && !c->trial_set) return set_error(KDQMC_ESTATE, "projector context: call kdqmc_set_trial first");
  const size_t n = (size_t)c->Ltau * c->N;
  const size_t all = n * c->nch;  // chain z's fields at s_dev + z * n
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, c->stream, c->flag, 16);
  hipLaunchKernelGGL(k_check_fields, dim3((unsigned)((all + 255) / 256)), dim3(256), 0, c->stream, s_dev, all,
                     c->flag);
  int bad = 0;
  KDQMC_HIP(hipMemcpyAsync(&bad, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  KDQMC_HIP(hipStreamSynchronize(c->stream));
  if (bad) return set_error(KDQMC_EINVAL, "fields must be +1 or -1");
  KDQMC_HIP(hipMemcpy2DAsync(c->fields, c->zs, s_dev, n, n, c->nch, hipMemcpyDeviceToDevice, c->stream));
  KDQMC_TRY(clear_health(c));
  KDQMC_TRY(stab_build_left(c));
  KDQMC_TRY(stab_identity(c, false, 0));
  KDQMC_TRY(stab_green(c, 0, c->G64));
  KDQMC_TRY(copy_64_to_G(c, c->G64));
  c->l_cur = 0;
  c->dir = 0;
  c->stab_next = 1;
  c->left_valid = true;
  c->right_valid = false;
  c->stacks_valid = true;
  return KDQMC_OK;
}

int kdqmc_get_fields(kdqmc_ctx* c, int8_t* s_dev) {
  KDQMC_TRY(check_ctx(c));
  if (!s_dev) return set_error(KDQMC_EINVAL, "fields pointer is NULL");
  const size_t n = (size_t)c->Ltau * c->N;
  KDQMC_HIP(hipMemcpy2DAsync(s_dev, n, c->fields, c->zs, n, c->nch, hipMemcpyDeviceToDevice, c->stream));
  return KDQMC_OK;
}

int kdqmc_set_G(kdqmc_ctx* c, const double* G_dev, int l) {
  KDQMC_TRY(check_ctx(c));
  if (!G_dev) return set_error(KDQMC_EINVAL, "G pointer is NULL");
  if (l < 0 || l > c->Ltau) return set_error(KDQMC_EINVAL, "slice index out of range");
  KDQMC_TRY(copy_64_to_G(c, G_dev, (size_t)c->N * c->N));
  KDQMC_TRY(clear_health(c));
  // positions an upward pass at slice l: right stack entries up to slice l
  // stay usable when this pass (or a complete earlier one) built them
  if (l == 0) {
    c->dir = 0;
    c->stab_next = 1;
  } else {
    if (c->dir == 1) c->stab_next = std::min(c->stab_next, l / c->p.n_stab + 1);
    else c->stab_next = c->right_valid ? l / c->p.n_stab + 1 : 1;
    c->dir = 1;
  }
  c->l_cur = l;
  return KDQMC_OK;
}

// A slice step may not pass over a stabilization that is due: the stack entry
// it would build is needed by every later stabilization of the pass.
static int check_stab_due(kdqmc_ctx* c, int l) {
  const int lp = l - 1;
  if (lp > 0 && lp % c->p.n_stab == 0 && lp / c->p.n_stab >= c->stab_next)
    return set_error(KDQMC_ESTATE, "kdqmc_stabilize is due at the current slice");
  return KDQMC_OK;
}

static int check_stab_due_down(kdqmc_ctx* c, int l) {
  if (l < c->Ltau && l % c->p.n_stab == 0 && l / c->p.n_stab <= c->stab_next)
    return set_error(KDQMC_ESTATE, "kdqmc_stabilize is due at the current slice");
  return KDQMC_OK;
}

static int stabilize_impl(kdqmc_ctx* c, double* wrap_err_dev, size_t zn);
static void drop_graphs(kdqmc_ctx* c);

// Upward wrap G(l) = exp(-dtau K) [D G_store D^{-1}] exp(dtau K) (D = ev).
static int wrap_pass(kdqmc_ctx* c) {
  if (c->fp64) {
    KDQMC_TRY(launch_kinetic_f64(c, (double*)c->G, c->N, true, (const double*)c->tab_m, c->ev, c->evinv, nullptr));
    KDQMC_TRY(launch_kinetic_f64(c, (double*)c->G, c->N, false, (const double*)c->tab_p, nullptr, nullptr, nullptr));
  } else {
    KDQMC_TRY(launch_kinetic_f32(c, (float*)c->G, c->N, true, (const float*)c->tab_m, c->ev, c->evinv, nullptr));
    KDQMC_TRY(launch_kinetic_f32(c, (float*)c->G, c->N, false, (const float*)c->tab_p, nullptr, nullptr, nullptr));
  }
  return KDQMC_OK;
}

// Downward wrap into the store frame: G_store = D^{-1} exp(dtau K) G(l)
// exp(-dtau K) D (D = ev): the column pass applies exp(dtau K), the row pass
// exp(-dtau K) with the row scale D^{-1} and the column scale D.
static int wrap_pass_down(kdqmc_ctx* c) {
  if (c->fp64) {
    KDQMC_TRY(launch_kinetic_f64(c, (double*)c->G, c->N, true, (const double*)c->tab_p, nullptr, nullptr, nullptr));
    KDQMC_TRY(launch_kinetic_f64(c, (double*)c->G, c->N, false, (const double*)c->tab_m, nullptr, c->evinv, c->ev));
  } else {
    KDQMC_TRY(launch_kinetic_f32(c, (float*)c->G, c->N, true, (const float*)c->tab_p, nullptr, nullptr, nullptr));
    KDQMC_TRY(launch_kinetic_f32(c, (float*)c->G, c->N, false, (const float*)c->tab_m, nullptr, c->evinv, c->ev));
  }
  return KDQMC_OK;
}

// Starts an upward pass at slice 1 from slice 0, or continues one.
static int enter_up(kdqmc_ctx* c, int l, const char* what) {
  if (c->l_cur < 0) return set_error(KDQMC_ESTATE, "no G loaded (set_fields or set_G first)");
  if (c->dir < 0) return set_error(KDQMC_ESTATE, "a downward pass is in progress");
  if (l != c->l_cur + 1 || l > c->Ltau) return set_error(KDQMC_ESTATE, std::string(what) + " needs l == current slice + 1");
  if (c->dir == 0) {
    c->dir = 1;
    c->stab_next = 1;
  }
  return check_stab_due(c, l);
}

int kdqmc_wrap_slice(kdqmc_ctx* c, int l) {
  KDQMC_TRY(check_ctx(c));
  KDQMC_TRY(enter_up(c, l, "wrap_slice"));
  KDQMC_TRY(launch_frame_scale(c, l));
  KDQMC_TRY(wrap_pass(c));
  c->l_cur = l;
  return KDQMC_OK;
}

// zn: elements between consecutive chains' records of u, forced, accepted, ratio
static int sweep_slice_impl(kdqmc_ctx* c, int l, const double* u_dev, const uint8_t* forced_dev,
                            uint8_t* accepted_dev, double* ratio_dev, size_t zn) {
  if (!u_dev && !forced_dev) return set_error(KDQMC_EINVAL, "need uniforms or forced decisions");
  KDQMC_TRY(enter_up(c, l, "sweep_slice"));
  KDQMC_TRY(launch_frame_scale(c, l));
  KDQMC_TRY(run_slice_updates(c, l, u_dev, forced_dev, accepted_dev, ratio_dev, zn));
  KDQMC_TRY(wrap_pass(c));
  c->l_cur = l;
  return KDQMC_OK;
}

int kdqmc_sweep_slice(kdqmc_ctx* c, int l, const double* u_dev, const uint8_t* forced_dev,
                      uint8_t* accepted_dev, double* ratio_dev) {
  KDQMC_TRY(check_ctx(c));
  return sweep_slice_impl(c, l, u_dev, forced_dev, accepted_dev, ratio_dev, (size_t)c->N);
}

static int sweep_slice_down_impl(kdqmc_ctx* c, int l, const double* u_dev, const uint8_t* forced_dev,
                                 uint8_t* accepted_dev, double* ratio_dev, size_t zn) {
  if (!u_dev && !forced_dev) return set_error(KDQMC_EINVAL, "need uniforms or forced decisions");
  if (c->l_cur < 0) return set_error(KDQMC_ESTATE, "no G loaded (set_fields or set_G first)");
  if (!c->stacks_valid) return set_error(KDQMC_ESTATE, "stacks not built (call set_fields)");
  if (c->dir > 0) return set_error(KDQMC_ESTATE, "an upward pass is in progress");
  if (c->dir == 0) {
    // finite temperature: G(L_tau) = G(0); the projector form needs an upward
    // pass to have ended at slice L_tau
    if (c->l_cur != (c->proj ? c->Ltau : 0) || l != c->Ltau)
      return set_error(KDQMC_ESTATE, c->proj ? "a projector downward pass starts where an upward pass ended (slice L_tau)"
                                             : "a downward pass starts at slice L_tau from slice 0");
    c->dir = -1;
    c->l_cur = c->Ltau;  // G(L_tau) = G(0)
    c->stab_next = c->nc - 1;
  }
  if (l != c->l_cur) return set_error(KDQMC_ESTATE, "sweep_slice_down needs l == current slice");
  KDQMC_TRY(check_stab_due_down(c, l));
  KDQMC_TRY(launch_frame_scale(c, l));
  KDQMC_TRY(wrap_pass_down(c));
  KDQMC_TRY(run_slice_updates(c, l, u_dev, forced_dev, accepted_dev, ratio_dev, zn));
  KDQMC_TRY(launch_down_reframe(c, l));
  c->l_cur = l - 1;
  return KDQMC_OK;
}

int kdqmc_sweep_slice_down(kdqmc_ctx* c, int l, const double* u_dev, const uint8_t* forced_dev,
                           uint8_t* accepted_dev, double* ratio_dev) {
  KDQMC_TRY(check_ctx(c));
  return sweep_slice_down_impl(c, l, u_dev, forced_dev, accepted_dev, ratio_dev, (size_t)c->N);
}

// zn: elements between consecutive chains' wrap-error records
static int stabilize_timed(kdqmc_ctx* c, double* wrap_err_dev, size_t zn) {
  const int e0 = prof_mark(c);
  const int rc = stabilize_impl(c, wrap_err_dev, zn);
  prof_pair(c, PH_STABILIZE, e0, prof_mark(c));
  return rc;
}

// Reads every chain's health record (synchronizes).  latest: check the
// latest stabilization only; otherwise everything since the last clear.
static int read_health(kdqmc_ctx* c, bool latest, double* worst_out) {
  std::vector<double> h((size_t)c->nch * HL_COUNT);
  KDQMC_HIP(hipMemcpy2DAsync(h.data(), HL_COUNT * sizeof(double), c->health, c->zs, HL_COUNT * sizeof(double),
                             c->nch, hipMemcpyDeviceToHost, c->stream));
  KDQMC_HIP(hipStreamSynchronize(c->stream));
  double worst = 0.0;
  int bad = -1;
  for (int z = 0; z < c->nch; ++z) {
    const double* r = &h[(size_t)z * HL_COUNT];
    const double e = latest ? r[HL_LAST] : r[HL_WORST];
    if (e != e || e > worst) worst = (worst != worst) ? worst : e;
    const bool b = r[HL_NONFINITE] != 0.0 || (latest ? !(e <= c->wrap_tol) : r[HL_NVIOL] != 0.0);
    if (b && bad < 0) bad = z;
  }
  if (worst_out) *worst_out = worst;
  if (bad >= 0) {
    const double* r = &h[(size_t)bad * HL_COUNT];
    char msg[256];
    std::snprintf(msg, sizeof msg,
                  "chain %d: wrap error %.3e (tolerance %.3e)%s; G is not trusted (non-finite values or a "
                  "drift beyond the tolerance)",
                  bad, latest ? r[HL_LAST] : r[HL_WORST], c->wrap_tol,
                  r[HL_NONFINITE] != 0.0 ? ", non-finite column norm in a stabilization product" : "");
    return set_error(KDQMC_ENUMERIC, msg);
  }
  return KDQMC_OK;
}

int kdqmc_stabilize(kdqmc_ctx* c, double* wrap_err_dev) {
  KDQMC_TRY(check_ctx(c));
  KDQMC_TRY(stabilize_timed(c, wrap_err_dev, 1));
  return read_health(c, true, nullptr);
}

int kdqmc_set_wrap_tolerance(kdqmc_ctx* c, double tol) {
  KDQMC_TRY(check_ctx(c));
  if (!(tol > 0.0)) return set_error(KDQMC_EINVAL, "tolerance must be > 0 (inf disables the check)");
  if (tol != c->wrap_tol) {
    drop_graphs(c);  // captured graphs carry the old value
    c->wrap_tol = tol;
  }
  return KDQMC_OK;
}

int kdqmc_set_slice_launch(kdqmc_ctx* c, int persistent) {
  KDQMC_TRY(check_ctx(c));
  const bool want = persistent != 0 && c->persist_ok;
  if (want != c->persist) {
    drop_graphs(c);  // captured graphs carry the old schedule
    c->persist = want;
  }
  clear_error();
  return c->persist ? 1 : 0;
}

int kdqmc_health(kdqmc_ctx* c, double* worst_host) {
  KDQMC_TRY(check_ctx(c));
  const int rc = read_health(c, false, worst_host);
  KDQMC_TRY(clear_health(c));
  return rc;
}

// The state at the end of a whole pass: slice 0 (the projector form: an
// upward pass ends at slice L_tau, whose G differs from G(0)); an upward pass
// leaves the right stack matching the new fields, a downward pass the left
// stack.
static void end_of_pass(kdqmc_ctx* c, int dir) {
  c->l_cur = (c->proj && dir > 0) ? c->Ltau : 0;
  c->dir = 0;
  c->stab_next = 1;
  c->left_valid = dir < 0;
  c->right_valid = dir > 0;
}

static int stabilize_impl(kdqmc_ctx* c, double* wrap_err_dev, size_t zn) {
  if (!c->stacks_valid) return set_error(KDQMC_ESTATE, "stacks not built (call set_fields)");
  const int l = c->l_cur;
  if (c->dir == 0) return set_error(KDQMC_ESTATE, "no pass in progress");
  if (l % c->p.n_stab != 0 || (c->dir > 0 && l == 0) || (c->dir < 0 && l == c->Ltau))
    return set_error(KDQMC_ESTATE, "stabilize needs the current slice to be a multiple of n_stab inside a pass");
  const int j = l / c->p.n_stab;
  if (j != c->stab_next)
    return set_error(KDQMC_ESTATE, "an earlier stabilization was skipped (each multiple of n_stab needs one, in order)");
  if (c->dir > 0) {
    // the left entries used from here on depend only on slices not yet
    // visited in this pass, so a stale left stack is rebuilt from the fields
    if (!c->left_valid) {
      KDQMC_TRY(stab_build_left(c));
      c->left_valid = true;
    }
    KDQMC_TRY(stab_right_step(c, j));
  } else {
    if (!c->right_valid) {
      KDQMC_TRY(stab_build_right(c));
      c->right_valid = true;
    }
    KDQMC_TRY(stab_left_step(c, j));
  }
  KDQMC_TRY(stab_green(c, j, c->G64));
  KDQMC_TRY(max_abs_diff(c, c->G64, c->N, wrap_err_dev, zn));
  KDQMC_TRY(copy_64_to_G(c, c->G64));
  if (c->dir > 0) {
    c->stab_next = j + 1;
    if (j == c->nc) end_of_pass(c, 1);
  } else {
    c->stab_next = j - 1;
    if (j == 0) end_of_pass(c, -1);
  }
  return KDQMC_OK;
}

// Slices a..b of a pass (upward: a <= b, downward: a >= b), each followed by
// the stabilization that is due after it; caller records are L_tau * N apart
// per chain, wrap errors L_tau / n_stab apart.
static int pass_range(kdqmc_ctx* c, int dir, int a, int b, const double* u_dev, const uint8_t* forced_dev,
                      uint8_t* accepted_dev, double* ratio_dev, double* wrap_err_dev) {
  const size_t N = c->N;
  const size_t zn = (size_t)c->Ltau * N;
  const int ns = c->p.n_stab;
  for (int l = a; dir > 0 ? l <= b : l >= b; l += dir) {
    const size_t o = (size_t)(l - 1) * N;
    const double* u = u_dev ? u_dev + o : nullptr;
    const uint8_t* f = forced_dev ? forced_dev + o : nullptr;
    uint8_t* acc = accepted_dev ? accepted_dev + o : nullptr;
    double* rat = ratio_dev ? ratio_dev + o : nullptr;
    if (dir > 0) {
      KDQMC_TRY(sweep_slice_impl(c, l, u, f, acc, rat, zn));
      if (l % ns == 0)
        KDQMC_TRY(stabilize_timed(c, wrap_err_dev ? wrap_err_dev + (l / ns - 1) : nullptr, (size_t)c->nc));
    } else {
      KDQMC_TRY(sweep_slice_down_impl(c, l, u, f, acc, rat, zn));
      if ((l - 1) % ns == 0)
        KDQMC_TRY(stabilize_timed(c, wrap_err_dev ? wrap_err_dev + (l - 1) / ns : nullptr, (size_t)c->nc));
    }
  }
  return KDQMC_OK;
}

// Graph execs may still be queued on the stream (the host runs ahead of the
// device): they are destroyed only after the stream has drained.
static void drop_graphs(kdqmc_ctx* c) {
  if (!c->sweep_exec[0].empty() || !c->sweep_exec[1].empty()) (void)hipStreamSynchronize(c->stream);
  for (int g = 0; g < 2; ++g) {
    for (hipGraphExec_t e : c->sweep_exec[g]) (void)hipGraphExecDestroy(e);
    c->sweep_exec[g].clear();
  }
}

// Slices per captured graph: never across a stabilization, and at most
// about 4096 decision windows, so that no graph grows beyond some 15k nodes.
static int graph_segment_slices(const kdqmc_ctx* c) {
  return std::max(1, std::min(c->p.n_stab, 4096 / std::max(1, c->nw)));
}

// A whole pass (dir = +1 upward, -1 downward), from and back to slice 0.
static int run_pass(kdqmc_ctx* c, int dir, const double* u_dev, const uint8_t* forced_dev,
                    uint8_t* accepted_dev, double* ratio_dev, double* wrap_err_dev) {
  KDQMC_TRY(check_ctx(c));
  const int start = (dir < 0 && c->proj) ? c->Ltau : 0;
  if (c->l_cur != start || c->dir != 0)
    return set_error(KDQMC_ESTATE, c->proj ? "projector passes alternate: upward from slice 0, downward from L_tau"
                                           : "a pass needs the current slice to be 0");
  if (!c->stacks_valid) return set_error(KDQMC_ESTATE, "stacks not built (call set_fields)");
  if (!u_dev && !forced_dev) return set_error(KDQMC_EINVAL, "need uniforms or forced decisions");
  const int first = dir > 0 ? 1 : c->Ltau, last = dir > 0 ? c->Ltau : 1;
  // events recorded inside a captured graph cannot be timed: profiling runs eager
  if (!c->use_graphs || c->prof_on)
    return pass_range(c, dir, first, last, u_dev, forced_dev, accepted_dev, ratio_dev, wrap_err_dev);
  const int gi = dir > 0 ? 0 : 1;
  // what the captured launches depend on: the caller's buffers and whether
  // the stack the pass reads must be rebuilt first
  const bool stale = dir > 0 ? !c->left_valid : !c->right_valid;
  const bool left0 = c->left_valid, right0 = c->right_valid;
  const void* key[7] = {u_dev, forced_dev, accepted_dev, ratio_dev, wrap_err_dev,
                        reinterpret_cast<const void*>(uintptr_t(stale ? 2 : 1)), nullptr};
  bool same = !c->sweep_exec[gi].empty();
  for (int i = 0; i < 7 && same; ++i) same = (key[i] == c->sweep_key[gi][i]);
  if (!same) {
    // the execs being replaced may still be queued: wait for them first
    if (!c->sweep_exec[gi].empty()) KDQMC_HIP(hipStreamSynchronize(c->stream));
    for (hipGraphExec_t e : c->sweep_exec[gi]) (void)hipGraphExecDestroy(e);
    c->sweep_exec[gi].clear();
    if (!c->cap_stream) KDQMC_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    c->graph_next = 0;
    c->graph_triples.clear();
    const int seg = graph_segment_slices(c);
    const int ns = c->p.n_stab;
    hipStream_t user = c->stream;
    for (int a = first; dir > 0 ? a <= last : a >= last;) {
      // a segment ends at the next stabilization point at the latest
      int b;
      if (dir > 0) b = std::min(((a - 1) / ns + 1) * ns, a + seg - 1);
      else b = std::max(((a - 1) / ns) * ns + 1, a - seg + 1);
      KDQMC_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      c->stream = c->cap_stream;
      c->capturing = true;
      const int rc = pass_range(c, dir, a, b, u_dev, forced_dev, accepted_dev, ratio_dev, wrap_err_dev);
      c->capturing = false;
      c->stream = user;
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
      hipGraphExec_t ex = nullptr;
      hipError_t ei = hipSuccess;
      if (rc == KDQMC_OK && ec == hipSuccess) ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (rc != KDQMC_OK || ec != hipSuccess || ei != hipSuccess) {
        for (hipGraphExec_t e : c->sweep_exec[gi]) (void)hipGraphExecDestroy(e);
        c->sweep_exec[gi].clear();
        // nothing of the pass has run: the stacks and G are as before it
        c->l_cur = 0;
        c->dir = 0;
        c->stab_next = 1;
        c->left_valid = left0;
        c->right_valid = right0;
        if (rc != KDQMC_OK) return rc;
        if (ec != hipSuccess)
          return set_error(KDQMC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        return set_error(KDQMC_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
      }
      c->sweep_exec[gi].push_back(ex);
      a = b + dir;
    }
    for (int i = 0; i < 7; ++i) c->sweep_key[gi][i] = key[i];
  }
  for (hipGraphExec_t ex : c->sweep_exec[gi]) KDQMC_HIP(hipGraphLaunch(ex, c->stream));
  end_of_pass(c, dir);
  return KDQMC_OK;
}

int kdqmc_sweep(kdqmc_ctx* c, const double* u_dev, const uint8_t* forced_dev, uint8_t* accepted_dev,
                double* ratio_dev, double* wrap_err_dev) {
  return run_pass(c, 1, u_dev, forced_dev, accepted_dev, ratio_dev, wrap_err_dev);
}

int kdqmc_sweep_down(kdqmc_ctx* c, const double* u_dev, const uint8_t* forced_dev, uint8_t* accepted_dev,
                     double* ratio_dev, double* wrap_err_dev) {
  return run_pass(c, -1, u_dev, forced_dev, accepted_dev, ratio_dev, wrap_err_dev);
}

int kdqmc_use_graphs(kdqmc_ctx* c, int on) {
  KDQMC_TRY(check_ctx(c));
  c->use_graphs = (on != 0);
  if (!c->use_graphs) drop_graphs(c);
  return KDQMC_OK;
}

int kdqmc_num_chains(const kdqmc_ctx* c) {
  if (!c) return set_error(KDQMC_EINVAL, "context is NULL");
  return c->nch;
}

int kdqmc_measure_G(kdqmc_ctx* c, double* G_dev) {
  KDQMC_TRY(check_ctx(c));
  if (!G_dev) return set_error(KDQMC_EINVAL, "G pointer is NULL");
  if (c->l_cur < 0) return set_error(KDQMC_ESTATE, "no G loaded");
  return copy_G_to64(c, G_dev, (size_t)c->N * c->N);
}

int kdqmc_measure(kdqmc_ctx* c, double* obs_dev) {
  KDQMC_TRY(check_ctx(c));
  if (!obs_dev) return set_error(KDQMC_EINVAL, "obs pointer is NULL");
  if (c->l_cur < 0) return set_error(KDQMC_ESTATE, "no G loaded");
  if (c->lattice != KDQMC_KAGOME) return set_error(KDQMC_EUNSUPPORTED, "the estimators are defined for the kagome lattice");
  return launch_measure(c, obs_dev, KDQMC_NOBS);
}

int kdqmc_current_slice(const kdqmc_ctx* c) {
  if (!c) return set_error(KDQMC_EINVAL, "context is NULL");
  return c->l_cur;
}

int kdqmc_sync(kdqmc_ctx* c) {
  KDQMC_TRY(check_ctx(c));
  KDQMC_HIP(hipStreamSynchronize(c->stream));
  return KDQMC_OK;
}

void kdqmc_destroy(kdqmc_ctx* c) {
  if (!c) return;
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (hipEvent_t e : c->prof_events) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->graph_events) (void)hipEventDestroy(e);
  delete c;
}

int kdqmc_profile_enable(kdqmc_ctx* c, int on) {
  KDQMC_TRY(check_ctx(c));
  c->prof_on = (on != 0);
  c->prof_next = 0;
  c->prof_triples.clear();
  for (int i = 0; i < 16; ++i) {
    c->prof_acc_ms[i] = 0.0;
    c->prof_acc_n[i] = 0;
  }
  return KDQMC_OK;
}

int kdqmc_profile_read(kdqmc_ctx* c, double* ms, int* launches) {
  KDQMC_TRY(check_ctx(c));
  if (!ms || !launches) return set_error(KDQMC_EINVAL, "NULL output");
  for (int i = 0; i < KDQMC_NPHASE; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  KDQMC_HIP(hipStreamSynchronize(c->stream));
  KDQMC_TRY(prof_accumulate(c, c->prof_events, c->prof_triples));
  for (int i = 0; i < KDQMC_NPHASE; ++i) {
    ms[i] = c->prof_acc_ms[i];
    launches[i] = c->prof_acc_n[i];
    c->prof_acc_ms[i] = 0.0;
    c->prof_acc_n[i] = 0;
  }
  c->prof_next = 0;
  c->prof_triples.clear();
  return KDQMC_OK;
}

const char* kdqmc_phase_name(int phase) {
  static const char* names[KDQMC_NPHASE] = {"wrap_cols", "wrap_rows", "decide",  "extend",
                                            "prep",      "flush",     "bmul",    "qr_panel",
                                            "gemm",      "stabilize", "flush_decide", "measure"};
  return (phase >= 0 && phase < KDQMC_NPHASE) ? names[phase] : "";
}

const char* kdqmc_last_error(void) { return g_last_error.c_str(); }

int kdqmc_gemm_f64(kdqmc_ctx* c, int trans_a, int trans_b, int M, int N, int K, double alpha,
                   const double* A_dev, int lda, const double* B_dev, int ldb, double beta,
                   double* C_dev, int ldc) {
  KDQMC_TRY(check_ctx(c));
  if (!A_dev || !B_dev || !C_dev) return set_error(KDQMC_EINVAL, "NULL matrix");
  if (c->nch != 1) return set_error(KDQMC_EINVAL, "building blocks need a single-chain context");
  if (M < 0 || N < 0 || K < 0) return set_error(KDQMC_EINVAL, "negative size");
  const int acols = trans_a ? M : K, bcols = trans_b ? K : N;
  if (lda < std::max(1, acols) || ldb < std::max(1, bcols) || ldc < std::max(1, N))
    return set_error(KDQMC_EINVAL, "leading dimension too small");
  return gemm_f64(c, trans_a != 0, trans_b != 0, M, N, K, alpha, A_dev, lda, B_dev, ldb, beta, C_dev, ldc);
}

int kdqmc_expK_f64(kdqmc_ctx* c, double* A_dev, int lda, int ncols, int sign) {
  KDQMC_TRY(check_ctx(c));
  if (!A_dev) return set_error(KDQMC_EINVAL, "NULL matrix");
  if (c->nch != 1 || !c->fp64) return set_error(KDQMC_EINVAL, "needs a single-chain FP64 context");
  if (sign != 1 && sign != -1) return set_error(KDQMC_EINVAL, "sign must be +1 or -1");
  if (ncols < 1 || ncols > c->N || lda < c->N) return set_error(KDQMC_EINVAL, "bad ncols or lda");
  return launch_kinetic_f64(c, A_dev, lda, true, (const double*)(sign < 0 ? c->tab_m : c->tab_p), nullptr,
                            nullptr, nullptr, ncols);
}

int kdqmc_qr_f64(kdqmc_ctx* c, int n, double* A_dev, double* Q_dev) {
  KDQMC_TRY(check_ctx(c));
  if (!A_dev || !Q_dev) return set_error(KDQMC_EINVAL, "NULL matrix");
  if (c->nch != 1) return set_error(KDQMC_EINVAL, "building blocks need a single-chain context");
  if (n < 1 || n > c->N) return set_error(KDQMC_EINVAL, "QR order must be in 1..N");
  // the routine works with row stride N; callers pass N x N buffers
  return qr_f64(c, n, n, A_dev, Q_dev);
}

}  // extern "C"
