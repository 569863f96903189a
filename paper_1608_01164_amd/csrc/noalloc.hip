// Allocation-free application of a HODLR matrix: the product Y = P X of apply_projector with its
// device workspace taken from one static device array per GPU instead of the runtime, for callers
// that must not allocate (code under HIP graph capture, serving loops, harnesses that forbid it).
#include "../../include/hq.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "engine.h"
#include "handle.h"
#include "predictor.h"

namespace {

// Largest device workspace an allocation-free apply may use.  Every GPU the library runs on holds
// one such array until the process ends; all allocation-free calls on that GPU share it.
constexpr size_t kScratchBytes = size_t(64) << 20;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // device address of `scratch` on each device, once looked up

// The array's address on the current device (the host symbol is not a device address).
void* scratch_on_current_device() {
  int dev = 0;
  HQ_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw std::runtime_error("device index beyond the library's table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    HQ_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

hq_status nofail(hq_status s, const std::string& m) {
  hq::set_last_error(m);
  return s;
}

}  // namespace

extern "C" size_t apply_projector_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" hq_status apply_projector_noalloc(hq_hodlr_t P, const double* X, int64_t ldx, int32_t ncols, double* Y,
                                             int64_t ldy, void* stream) {
  if (!P) return nofail(HQ_ERR_ARG, "P is NULL");
  if (ncols < 0) return nofail(HQ_ERR_ARG, "ncols < 0");
  if (ncols == 0) return HQ_OK;
  if (!X || !Y) return nofail(HQ_ERR_ARG, "X or Y is NULL");
  if (ldx < P->t.n || ldy < P->t.n) return nofail(HQ_ERR_ARG, "ldx/ldy < n");
  try {
    hq::Engine& e = *P->e;
    const std::vector<hq::Engine::ThinTask> task{
        hq::Engine::ThinTask{e.view(P->H), 0, X, (int)ldx, Y, (int)ldy, P->d_w, ncols, 1.0, 0.0}};
    const size_t need = hq::Engine::thin_scratch_bytes(task);
    if (need > kScratchBytes)
      return nofail(HQ_ERR_ARG, "apply_projector_noalloc: " + std::to_string(ncols) + " columns need " +
                                    std::to_string(need) + " bytes of workspace, above the static maximum of " +
                                    std::to_string(kScratchBytes) + " bytes (apply fewer columns per call)");
    void* ws = scratch_on_current_device();
    HQ_CHECK(hipEventSynchronize(P->done));  // the previous call's descriptors have been read
    e.st = (hipStream_t)stream;
    e.stage.reset();
    hq::DevArena fixed;
    fixed.attach_fixed(ws, kScratchBytes);
    e.scratch.swap(fixed);  // the engine's own chunks wait in `fixed` until the call ends
    e.stage.no_grow = true;
    struct Restore {
      hq::Engine& e;
      hq::DevArena& own;
      ~Restore() {
        e.scratch.swap(own);
        e.stage.no_grow = false;
      }
    } restore{e, fixed};
    hq::launch_fill_int(P->d_w, ncols, 1, e.st);
    e.mm_thin(task);
    HQ_CHECK(hipEventRecord(P->done, e.st));
    if (e.scratch.high_water() > need)  // the plan above must bound what the product took
      return nofail(HQ_ERR_DEVICE, "apply_projector_noalloc: workspace plan of " + std::to_string(need) +
                                       " bytes below the " + std::to_string(e.scratch.high_water()) + " used");
    return HQ_OK;
  } catch (const hq::NoAlloc& x) {
    return nofail(HQ_ERR_ALLOC, std::string("apply_projector_noalloc: ") + x.what());
  } catch (const hq::HipError& x) {
    return nofail(HQ_ERR_DEVICE, x.what());
  } catch (const std::exception& x) {
    return nofail(HQ_ERR_DEVICE, x.what());
  }
}
