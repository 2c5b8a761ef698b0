// Allocation-free total potential Pi(u) for callers that cannot allocate
// device memory (code under graph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// pfem_energy keeps its block partial sums and the permuted state in
// buffers that the mesh allocates on first use.  pfem_energy_noalloc runs
// the same kernels on the same arguments, but carves those buffers out of
// one file-scope device array of kScratchBytes.  The array's host-side name
// is only a stand-in for the runtime: its device address, one per GPU, is
// looked up once per device when a context is created (noalloc_init) and
// that address is what every launch receives.
#include <mutex>

#include "mesh.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_dev[kMaxDevices] = {};

size_t round256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

namespace pfem {

// With `device` current: record this device's address of the scratch array
// (every GPU holds its own copy at its own address).  Called by
// pfem_ctx_create; later calls for the same device return at once.
void noalloc_init(int device) {
  require(device >= 0 && device < kMaxDevices, PFEM_E_INVALID_ARG,
          "device index beyond the allocation-free table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch_dev[device] != nullptr) return;
  void* p = nullptr;
  PFEM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  require(p != nullptr, PFEM_E_DEVICE, "scratch array has no device address");
  g_scratch_dev[device] = p;
}

static void* scratch_for(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_dev[device] : nullptr;
}

}  // namespace pfem

using namespace pfem;

extern "C" pfem_status pfem_energy_noalloc(pfem_mesh* m, int prec, int layout, const void* u,
                                           double* energy_dev) {
  try {
    require(m != nullptr, PFEM_E_INVALID_ARG, "mesh is NULL");
    require(u != nullptr && energy_dev != nullptr, PFEM_E_INVALID_ARG, "NULL argument");
    require(prec == PFEM_FP64 || prec == PFEM_FP32, PFEM_E_INVALID_ARG, "bad precision");
    require(layout == PFEM_LAYOUT_USER || layout == PFEM_LAYOUT_INTERNAL, PFEM_E_INVALID_ARG,
            "bad layout");
    require(m->finalized, PFEM_E_STATE, "mesh not finalized");
    require(m->uploaded && m->ctx != nullptr, PFEM_E_STATE, "mesh has no device context");
    Ctx* ctx = m->ctx;
    PFEM_HIP(hipSetDevice(ctx->device));
    // layout of the scratch array: reduced sums | block partials | permuted u
    const size_t s = prec == PFEM_FP64 ? 8 : 4;
    const size_t out_bytes = round256(kRedSlots * sizeof(double));
    const size_t part_bytes =
        round256((size_t)std::max(m->n_blocks, 1) * kRedSlots * sizeof(double));
    const size_t u_bytes = layout == PFEM_LAYOUT_USER ? round256((size_t)m->n_dof() * s) : 0;
    const size_t need = out_bytes + part_bytes + u_bytes;
    if (need > kScratchBytes)
      throw Error{PFEM_E_INVALID_ARG,
                  "mesh needs " + std::to_string(need) +
                      " bytes of allocation-free scratch; the limit is " +
                      std::to_string(kScratchBytes) + " (16 MiB)"};
    unsigned char* base = static_cast<unsigned char*>(scratch_for(ctx->device));
    require(base != nullptr, PFEM_E_STATE,
            "allocation-free scratch not set up on this device (no context created on it)");
    double* out = reinterpret_cast<double*>(base);
    double* part = reinterpret_cast<double*>(base + out_bytes);
    const void* ui = u;
    if (layout == PFEM_LAYOUT_USER) {
      void* perm_u = base + out_bytes + part_bytes;
      launch_permute(ctx, prec, m->dim, m->dev.perm, m->n_nodes, true, u, perm_u);
      ui = perm_u;
    }
    // every block writes its own partials and the reduction writes `out`,
    // so nothing in the array has to start at zero
    Task t{};
    t.m = m->md;
    t.u = ui;
    t.active = 1;
    t.fscale = 1.0;
    t.red.part = part;
    t.red.out = out;
    const Task* td = static_cast<const Task*>(ctx->ring.put(&t, sizeof(Task)));
    launch_energy(ctx, m->kind(), prec, false, td, m->dev.work, m->n_blocks);
    launch_reduce_store(ctx, td, 1);
    launch_energy_out(ctx, out, energy_dev, 1, kRedSlots);
    set_error("");
    return PFEM_OK;
  } catch (const pfem::Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return PFEM_E_INVALID_ARG;
  } catch (...) {
    set_error("unknown failure");
    return PFEM_E_DEVICE;
  }
}
