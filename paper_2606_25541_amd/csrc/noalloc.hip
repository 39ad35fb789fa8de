// Operator apply that allocates nothing: the workspace of psfd_apply (the
// transverse spectrum the z-pencil kernel transforms in place) lives in a
// file-scope device array instead of plan memory, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops).
//
// Each device that runs the library holds its own copy of `scratch` until the
// process ends. In host code the array's name is only a stand-in for the
// symbol: its device address is looked up once per device with
// hipGetSymbolAddress and kept; kernels get that address, never the name.
// Every call on a device shares that device's array, so calls that overlap on
// one device race. Each call overwrites the part it uses before reading it
// (the forward transverse stage writes every value the pencil and the inverse
// stage read), so nothing has to start at zero.
#include <mutex>
#include <vector>

#include "engine.hpp"
#include "noalloc.hpp"

namespace psfd {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;  // per device ordinal, null until looked up

Status noalloc_scratch(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0) {
    Status st;
    st.code = PSFD_ERR_INVALID_ARG;
    st.msg = "bad device ordinal";
    return st;
  }
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    if (cur != device) {
      Status st;
      st.code = PSFD_ERR_INVALID_ARG;
      st.msg = "the scratch array is looked up with its device current";
      return st;
    }
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
    if (!p) {
      Status st;
      st.code = PSFD_ERR_HIP;
      st.msg = "hipGetSymbolAddress(scratch) returned a null address";
      return st;
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return Status();
}

Status apply_noalloc(Group& g, int device, const void* deps, const void* x, void* y, int dtype, int flags,
                     hipStream_t s) {
  const size_t esz = dtype == PSFD_C64 ? 8 : 16;
  const size_t need = (size_t)g.sh.n3 * esz;
  if (need > NOALLOC_SCRATCH_BYTES) {
    Status st;
    st.code = PSFD_ERR_UNSUPPORTED_SIZE;
    st.msg = "the workspace of this grid and dtype (3 nx ny nz complex values) exceeds the " +
             std::to_string(NOALLOC_SCRATCH_BYTES >> 20) + " MiB static scratch of the allocation-free apply";
    return st;
  }
  void* ws = nullptr;
  Status st = noalloc_scratch(device, &ws);
  if (!st.ok()) return st;
  const int kmode = (flags & PSFD_APPLY_K_ONLY) ? 1 : 0;
  const int tr = (flags & PSFD_APPLY_TRANSPOSE) ? 1 : 0;
  const int rf = (flags & PSFD_APPLY_REFLECT) ? 1 : 0;
  if (dtype == PSFD_C64)
    apply_op<float2>(g, (const float2*)deps, vr(x), vr(y), (float2*)ws, kmode, tr, rf, nullptr, s);
  else
    apply_op<double2>(g, (const double2*)deps, vr(x), vr(y), (double2*)ws, kmode, tr, rf, nullptr, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e, "apply launch");
  return Status();
}

}  // namespace psfd
