// Rotation without device allocation, for callers that cannot allocate (code recorded into a HIP graph,
// tight serving loops, harnesses that forbid hipMalloc): the key switch's temporaries live in a static
// device array instead of the context's pool.
//
// `scratch` is one fixed region per device (each GPU the library runs on holds it until the process
// ends).  Its device address is looked up once per device, at context creation, with that device
// current; host code then only passes that address (the array's own name is a host-side stand-in, not a
// device address).  Every call on a device shares the region: calls that overlap on one GPU (two
// contexts on two streams, two threads) race on it.  Nothing in it needs to start at zero: every
// temporary of the key switch is written in full before it is read.
#include <mutex>

#include "handles.hpp"

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;  // a key switch at N = 2^16 with 12 + 3 primes, dnum = 4: 63 MiB

static __device__ __align__(256) u64 scratch[SCRATCH_BYTES / 8];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
u64* g_region[MAX_DEVICES] = {};

}  // namespace

namespace hetal {

void scratch_setup() {
  int dev = 0;
  HCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) fail(HETAL_E_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_region[dev]) return;
  void* p = nullptr;
  HCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) fail(HETAL_E_DEVICE, "no device address for the scratch region");
  g_region[dev] = static_cast<u64*>(p);
}

u64* scratch_region(int device, size_t* words) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (device < 0 || device >= MAX_DEVICES || !g_region[device])
    fail(HETAL_E_DEVICE, "scratch region not set up on this device");
  *words = SCRATCH_BYTES / 8;
  return g_region[device];
}

}  // namespace hetal

using namespace hetal;

extern "C" int hetal_hrot_noalloc(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* ct, int r, hetal_ct* out) {
  return guarded([&] {
    need(ctx && keys, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_ct(c, ct, "ciphertext");
    check_out(c, out, ct->level);
    need(out->data != ct->data, HETAL_E_INVALID_ARG, "the output must not be the input (in place needs a copy)");
    need(!c.timing, HETAL_E_INVALID_ARG, "per-kernel timing is on");
    const int lv = ct->level;
    const size_t need_words = key_switch_scratch_words(c, lv, 1);
    size_t have_words = 0;
    u64* region = scratch_region(ctx->device, &have_words);
    if (need_words > have_words)
      fail(HETAL_E_INVALID_ARG, "the rotation needs " + std::to_string(need_words * 8) +
                                    " bytes of scratch, above the fixed maximum of " +
                                    std::to_string(have_words * 8));
    const u32 g = galois_rot(c, r);
    need(g == 1 || keys->set.get(g) != nullptr, HETAL_E_NO_KEY, "no Galois key for this rotation");
    const double s = ct->scale;
    struct Arena {
      Pool& p;
      Arena(Pool& pl, u64* base, size_t words) : p(pl) { p.arena_begin(base, words); }
      ~Arena() { p.arena_end(); }
    } arena(c.pool, region, have_words);
    op_galois(c, keys->set, view_of(ct), g, out->data);
    c.counters[0] += 1;
    out->level = lv;
    out->scale = s;
  });
}
