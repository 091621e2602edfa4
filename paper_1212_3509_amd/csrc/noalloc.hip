// Allocation-free structured apply.  The structured apply's only scratch
// memory is the column-spectrum buffer (one FP64 complex half spectrum per
// input column, e.g. 5.9 MB for CP rank 10 at n = 4096); here it lives in a
// file-scope static device array instead of the context workspace, for
// callers that cannot allocate device memory.
//
// Every GPU the library runs on holds its own copy of the array (at its own
// address) until the process ends.  Its address is looked up once per device
// by demag_create (with that device current) and kept per device; host code
// passes that address to the kernels, never the array's name.  Calls on one
// device share the array: calls that overlap in time on one device race.
#include "internal.h"

#include <mutex>

namespace demag {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // per device
constexpr size_t kFlagBytes = 256;                   // the input check's flag, then the spectra
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};

}  // namespace

demag_status scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return DEMAG_OK;   // the no-alloc call reports it
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_done[device]) return DEMAG_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_done[device] = true;
  g_err[device] = e;
  g_ptr[device] = (e == hipSuccess) ? p : nullptr;
  return DEMAG_OK;
}

}  // namespace demag

using namespace demag;

extern "C" demag_status demag_apply_columns_noalloc(demag_ctx *ctx, const demag_factors *fc, const int32_t R[3],
                                                    const float *const in[3], float *const out[3]) {
  DEMAG_REQUIRE(ctx && fc && R && in && out, "demag_apply_columns_noalloc: NULL argument");
  DEMAG_REQUIRE(!fc->dense, "demag_apply_columns_noalloc: needs a uniform grid (Toeplitz factors)");
  for (int d = 0; d < 3; ++d) {
    DEMAG_REQUIRE(R[d] >= 0 && R[d] <= 65536, "demag_apply_columns_noalloc: R out of range");
    DEMAG_REQUIRE(R[d] == 0 || (in[d] && out[d]), "demag_apply_columns_noalloc: NULL column buffer");
    DEMAG_REQUIRE(fft_length(fc->n[d]) <= 8192, "demag_apply_columns_noalloc: n <= 4096 per axis");
  }
  DEMAG_REQUIRE(fc->spec_ready,
                "demag_apply_columns_noalloc: the factors' kernel spectra are not prepared; call "
                "demag_prepare_structured first (it allocates them)");
  const size_t need = columns_workspace_bytes(fc, R);
  DEMAG_REQUIRE(need <= kScratchBytes - kFlagBytes,
                "demag_apply_columns_noalloc: the column spectra need " + std::to_string(need) +
                    " bytes; the static scratch holds " + std::to_string(kScratchBytes - kFlagBytes) +
                    " (use demag_apply_columns)");
  DEMAG_REQUIRE(ctx->device >= 0 && ctx->device < kMaxDevices, "demag_apply_columns_noalloc: device index too large");
  DEMAG_TRY_HIP(hipSetDevice(ctx->device));
  char *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    DEMAG_REQUIRE(g_done[ctx->device], "demag_apply_columns_noalloc: scratch not set up for this device");
    if (g_err[ctx->device] != hipSuccess) {
      set_error(std::string("demag_apply_columns_noalloc: hipGetSymbolAddress failed: ") +
                hipGetErrorString(g_err[ctx->device]));
      return DEMAG_E_HIP;
    }
    base = static_cast<char *>(g_ptr[ctx->device]);
  }
  demag_status st = DEMAG_OK;
  for (int d = 0; d < 3 && st == DEMAG_OK; ++d)
    st = check_finite(ctx, in[d], size_t(3) * R[d] * fc->n[d], false, "demag_apply_columns_noalloc",
                      reinterpret_cast<int *>(base));
  if (st != DEMAG_OK) return st;
  // every spectrum point is written by the forward transforms before the
  // jobs read it, so the array needs no clearing between calls
  st = launch_columns(ctx, fc, DEMAG_FP64, R, in, out, base + kFlagBytes, kScratchBytes - kFlagBytes);
  if (st != DEMAG_OK) return st;
  if (fc->used) DEMAG_TRY_HIP(hipEventRecord(fc->used, ctx->stream));   // the event exists since assembly
  return DEMAG_OK;
}
