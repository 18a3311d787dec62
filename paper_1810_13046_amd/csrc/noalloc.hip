// transfer_velocity_noalloc: the velocity transfer of transfer_velocity
// without any device allocation, for callers that cannot allocate (code
// under stream capture, tight serving loops, harnesses that forbid it).
//
// The only scratch of the velocity transfer is that of the consistent-mass
// solve (the right-hand side B u_f, the Chebyshev vectors, the double
// residual and its partials); here it lives in a file-scope device array of
// kScratchBytes.  Each GPU the library runs on holds its own copy of the
// array until the process ends; its address is looked up once per device
// (hipGetSymbolAddress, with that device current) and only that address is
// handed to kernels.  Every call on one GPU shares the array: calls that
// overlap on one GPU (different streams, or threads) race.  Nothing in the
// array has to start at zero: the solve writes every vector before reading
// it.
#include <mutex>

#include "internal.hpp"

namespace ibvt {

constexpr size_t kScratchBytes = size_t(256) << 20;  // 256 MiB per GPU

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

struct ScratchTable {
  std::mutex mu;
  void* ptr[kMaxDevices] = {};
};

ScratchTable& table() {
  static ScratchTable t;
  return t;
}

// The device address of this GPU's array (looked up on its first use).
int scratch_address(void** out) {
  int dev = 0;
  int st = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (st) return st;
  if (dev < 0 || dev >= kMaxDevices) return set_error(IBVT_E_UNSUPPORTED, "device index");
  ScratchTable& t = table();
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.ptr[dev]) {
    void* p = nullptr;
    if ((st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress")))
      return st;
    if (!p) return set_error(IBVT_E_HIP, "hipGetSymbolAddress returned NULL");
    t.ptr[dev] = p;
  }
  *out = t.ptr[dev];
  return IBVT_OK;
}

}  // namespace
}  // namespace ibvt

using namespace ibvt;

extern "C" int transfer_velocity_noalloc(ibvt_coupling* c, const void* const u_f[3], void* u_s,
                                         int mass, double cg_rtol, int cg_maxit,
                                         hipStream_t stream, ibvt_solve_info* info) {
  if (!c || !u_f || !u_s) return set_error(IBVT_E_INVALID, "NULL argument");
  if (!c->ready)
    return set_error(IBVT_E_INVALID,
                     "the coupling's last assembly failed: reassemble it successfully first");
  for (int d = 0; d < c->ncomp; ++d)
    if (!u_f[d]) return set_error(IBVT_E_INVALID, "NULL fluid component");
  if (mass != IBVT_LUMPED && mass != IBVT_CONSISTENT)
    return set_error(IBVT_E_INVALID, "mass must be IBVT_LUMPED or IBVT_CONSISTENT");
  if (c->dual && mass != IBVT_LUMPED)
    return set_error(IBVT_E_INVALID, "the dual basis has a diagonal S: use IBVT_LUMPED");
  c->stream = stream;
  if (info) *info = ibvt_solve_info{};
  if (mass == IBVT_LUMPED) return apply_B(c, u_f, u_s, true, stream);  // no scratch
  if (!c->has_M) return set_error(IBVT_E_INVALID, "consistent mass was not built");
  if (!(cg_rtol > 0.0) || cg_maxit < 1)
    return set_error(IBVT_E_INVALID, "bad mass-solve rtol/maxit");
  // right-hand side B u_f first, then the solve's workspace
  const size_t tsize = c->precision == IBVT_FP32_MIXED ? sizeof(float) : sizeof(double);
  const size_t rhs_bytes = (size_t(3 * c->n_vert) * tsize + 255) & ~size_t(255);
  const size_t need = rhs_bytes + mass_solve_workspace_bytes(c);
  if (need > kScratchBytes)
    return set_error(IBVT_E_CAPACITY,
                     "transfer_velocity_noalloc: the consistent solve needs " +
                         std::to_string(need) + " bytes of scratch, more than the " +
                         std::to_string(kScratchBytes) +
                         " the library holds per GPU (use transfer_velocity)");
  void* base = nullptr;
  int st = scratch_address(&base);
  if (st) return st;
  char* rhs = static_cast<char*>(base);
  if ((st = apply_B(c, u_f, rhs, false, stream))) return st;
  if ((st = lumped_solve(c, rhs, u_s, stream))) return st;
  return mass_solve(c, rhs, u_s, cg_rtol, cg_maxit, stream, info, true, rhs + rhs_bytes);
}
