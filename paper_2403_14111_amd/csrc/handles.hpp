// The C ABI's handle types and the argument checks and error translation shared by the extern "C" entry
// points (capi.hip, noalloc.hip).
#pragma once
#include <array>
#include <map>
#include <memory>
#include <new>
#include <string>

#include "hetal.h"
#include "matrix.hpp"

struct hetal_ctx {
  hetal::Context c;
  hetal::MaskCache masks;
  // A second stream for independent groups of hetal_enc_matmul_batch, sharing c's tables (created on first use;
  // side_masks is declared after side so that it returns its buffers to side's pool before side goes).
  std::unique_ptr<hetal::Context> side;
  hetal::MaskCache side_masks;
  hipStream_t side_stream = nullptr;
  hipEvent_t join[2] = {nullptr, nullptr};
  int device = 0;  // the HIP device that was current at creation
  // Schedule choices per shape class (op, c, s0, input levels) of hetal_enc_matmul_batch, as hetal_autotune_batch
  // or hetal_tune_set left them (classes not listed take the defaults), and whether independent classes use the
  // second stream.
  std::map<std::array<int, 5>, hetal::Tune> tuned;
  bool two_streams = true;
};

struct hetal_sk {
  hetal_ctx* ctx;
  hetal::SecretKeyDev key;
};

struct hetal_keys {
  hetal_ctx* ctx;
  hetal::KeySet set;
};

namespace hetal {

// The message of the calling thread's last failed call (hetal_last_error).
inline thread_local std::string g_last_error;

// Runs f, translating the library's errors into status codes.
template <typename F>
int guarded(F&& f) {
  try {
    f();
    return HETAL_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return HETAL_E_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HETAL_E_DEVICE;
  }
}

inline void need(bool ok, int code, const char* msg) {
  if (!ok) fail(code, msg);
}

inline void check_ct(const Context& c, const hetal_ct* ct, const char* what) {
  need(ct && ct->data, HETAL_E_INVALID_ARG, what);
  need(ct->level >= 0 && ct->level < c.num_q, HETAL_E_LEVEL, "ciphertext level out of range");
  need(ct->capacity >= c.ct_words(ct->level), HETAL_E_INVALID_ARG, "ciphertext capacity smaller than its level needs");
}

inline void check_out(const Context& c, const hetal_ct* out, int level) {
  need(out && out->data, HETAL_E_INVALID_ARG, "output ciphertext");
  need(out->capacity >= c.ct_words(level), HETAL_E_INVALID_ARG, "output capacity too small for the result");
}

inline void check_pt(const Context& c, const hetal_pt* pt) {
  need(pt && pt->data, HETAL_E_INVALID_ARG, "plaintext");
  need(pt->level >= 0 && pt->level < c.num_q, HETAL_E_LEVEL, "plaintext level out of range");
  need(pt->capacity >= c.poly_words(pt->level), HETAL_E_INVALID_ARG, "plaintext capacity too small");
}

inline CtView view_of(const hetal_ct* ct) { return CtView{ct->data, ct->level, ct->scale}; }

}  // namespace hetal
