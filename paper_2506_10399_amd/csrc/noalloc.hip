// Relinearised product (the x^2 activation's CMult of paper Sec. 4.1, key
// switching of Sec. 2.1) for callers that cannot allocate device memory: its
// intermediates live in one fixed device array instead of the context's
// grow-only scratch.
//
// The array is a file-scope __device__ symbol.  Its name in host code is only
// a host-side stand-in, so host code never passes it to a kernel or a copy:
// the device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and kept, and every launch takes that address.
#include <map>
#include <mutex>
#include <string>

#include "../../include/ficgcn.h"
#include "internal.h"

static constexpr size_t kScratchBytes = (size_t)64 << 20;
static constexpr size_t kScratchWords = kScratchBytes / 8;

// Every word a call reads is written earlier in the same call (tensor
// product, ModUp digits, inner products, ModDown conversion), so the array
// needs no clearing between calls.
static __device__ __align__(256) uint64_t scratch[kScratchWords];

namespace {

std::mutex g_mu;
std::map<int, uint64_t*> g_scratch;   // device ordinal -> device address of `scratch`

uint64_t* scratch_on(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_scratch.find(device);
  if (it != g_scratch.end()) return it->second;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    FICGCN_THROW(ficgcn::EDEVICE_, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch[device] = (uint64_t*)p;
  return (uint64_t*)p;
}

template <typename F>
ficgcn_status guard(F&& f) {
  try {
    f();
    return FICGCN_OK;
  } catch (const ficgcn::Error& e) {
    ficgcn::set_error(e.msg);
    return (ficgcn_status)e.code;
  } catch (const std::exception& e) {
    ficgcn::set_error(e.what());
    return FICGCN_EINVAL;
  }
}

#define NA_REQUIRE(cond, code, msg) \
  do {                              \
    if (!(cond)) FICGCN_THROW(code, msg); \
  } while (0)

}  // namespace

using namespace ficgcn;

extern "C" size_t ckks_mul_relin_noalloc_limit(void) { return kScratchBytes; }

extern "C" ficgcn_status ckks_mul_relin_noalloc(ckks_ctx* ctx, const ckks_keys* eval_keys, const uint64_t* x_dev,
                                                const uint64_t* y_dev, uint32_t level, uint64_t* out_dev) {
  return guard([&] {
    NA_REQUIRE(ctx, EINVAL_, "null context");
    NA_REQUIRE(ctx->on_device, EINVAL_,
               "context has no device tables yet (any earlier device call on it, e.g. ckks_keygen, sets them up)");
    NA_REQUIRE((int)level < ctx->L, ELEVEL_, "level " + std::to_string(level) + " >= number of Q primes");
    NA_REQUIRE(x_dev && y_dev && out_dev, EINVAL_, "null argument");
    NA_REQUIRE(out_dev != x_dev && out_dev != y_dev, EINVAL_, "output aliases an input");
    int dev = -1;
    HIPCHECK(hipGetDevice(&dev));
    NA_REQUIRE(dev == ctx->device, EINVAL_, "the context's device is not the current device");
    const size_t N = ctx->N;
    const int l1 = (int)level + 1, ext = l1 + ctx->alpha;
    const int nd = (l1 + ctx->alpha - 1) / ctx->alpha;
    // tensor product d [3][l1] | ModUp digits D [nd][ext] | inner products acc [2][ext];
    // ModUp's coefficient-form copy of d2 ([l1]) sits in acc before the inner
    // product writes it, ModDown's conversion ([2][l1]) in D after the inner
    // product has read it (nd * ext >= 2 * l1 always holds)
    const size_t need = ((size_t)3 * l1 + (size_t)nd * ext + (size_t)2 * ext) * N;
    NA_REQUIRE(need <= kScratchWords, ENOMEM_,
               "relinearisation at level " + std::to_string(level) + " needs " + std::to_string(need * 8) +
                   " bytes of scratch; the fixed array holds " + std::to_string(kScratchBytes));
    NA_REQUIRE(eval_keys, EINVAL_, "null key set");
    auto it = eval_keys->swk.find(0);
    NA_REQUIRE(it != eval_keys->swk.end(), ENOKEY_, "missing relinearisation key");
    const uint64_t* rk = it->second;
    // the base-conversion tables of every level are built when the context
    // first goes to the device, so the lookups below allocate nothing
    for (int d = 0; d < nd; ++d)
      NA_REQUIRE(ctx->modup.count({(int)level, d}), EINVAL_, "base-conversion table missing");
    NA_REQUIRE(ctx->moddown.count((int)level), EINVAL_, "base-conversion table missing");
    uint64_t* base = scratch_on(dev);
    uint64_t* d = base;
    uint64_t* D = d + (size_t)3 * l1 * N;
    uint64_t* acc = D + (size_t)nd * ext * N;
    tensor(ctx, x_dev, y_dev, d, (int)level);
    modup(ctx, d + (size_t)2 * l1 * N, (int)level, D, /*tmp=*/acc);
    keymac(ctx, acc, D, rk, (int)level, 1);
    moddown(ctx, acc, (int)level, out_dev, d, 1, d + (size_t)l1 * N, /*conv=*/D);
  });
}
