// The Householder QR building block for callers that cannot allocate device
// memory (code under HIP graph capture, tight loops, harnesses that forbid
// hipMalloc): the same kernels as kdqmc_qr_f64, with their scratch (the
// reflectors V, the block-reflector factors T, the partial V^T C products and
// tau) in one file-scope device array instead of a context's workspace.
#include <mutex>

#include "common.h"

namespace kdqmc {
namespace {

constexpr int kNoallocMaxLd = 512;  // largest row stride (and order) accepted
constexpr size_t kAlign = 32;       // doubles (256 bytes)

constexpr size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Layout for row stride ld (the QR routine's scratch, as carved from a
// context's workspace): V ld x ld; per-panel T factors then those of the
// merged panel pairs; the split apply's partials; tau.
struct NoallocLayout {
  size_t v, tq, wq, tau, total;
};

constexpr NoallocLayout noalloc_layout(int ld) {
  NoallocLayout l{};
  l.v = 0;
  l.tq = round_up(l.v + (size_t)ld * ld);
  l.wq = round_up(l.tq + (size_t)(ld / 16 + 2 + ld / 32 + 2) * 32 * 32);
  l.tau = round_up(l.wq + (size_t)16 * 32 * ld);
  l.total = round_up(l.tau + (size_t)ld);
  return l;
}

constexpr size_t kScratchDoubles = noalloc_layout(kNoallocMaxLd).total;  // 4.6 MB

}  // namespace

// One copy per GPU, alive until the process ends.  Host code never passes
// this name to a kernel (on the host it is not a device address): it takes
// the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[256] = {nullptr};

// The current device's address of `scratch`, looked up once per device.
int scratch_address(double** out) {
  int dev = 0;
  KDQMC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 256) return set_error(KDQMC_EUNSUPPORTED, "device index above 255");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(KDQMC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[dev]);
  return KDQMC_OK;
}

}  // namespace
}  // namespace kdqmc

using namespace kdqmc;

extern "C" int kdqmc_qr_f64_noalloc(int n, int ld, double* A_dev, double* Q_dev, void* hip_stream) {
  if (!A_dev || !Q_dev) return set_error(KDQMC_EINVAL, "NULL matrix");
  if (n < 1 || ld < n) return set_error(KDQMC_EINVAL, "need 1 <= n <= ld");
  if (ld > kNoallocMaxLd)
    return set_error(KDQMC_EINVAL, "kdqmc_qr_f64_noalloc: ld above 512 (the static scratch holds 512 x 512)");
  double* s = nullptr;
  KDQMC_TRY(scratch_address(&s));
  // a host-side description of the routine's buffers: nothing is allocated
  kdqmc_ctx c;
  c.N = ld;
  c.nch = 1;
  c.zs = 0;
  c.stream = static_cast<hipStream_t>(hip_stream);
  const NoallocLayout l = noalloc_layout(ld);
  c.Vq = s + l.v;
  c.Tq = s + l.tq;
  c.Tm = c.Tq + (size_t)(ld / 16 + 2) * 32 * 32;
  c.Wq = s + l.wq;
  c.tau = s + l.tau;
  return qr_f64(&c, n, n, A_dev, Q_dev);
}
