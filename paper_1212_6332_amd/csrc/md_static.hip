// md_forces_static: forces and energies of one set of positions, with every
// device buffer carved from a fixed array in the library's own device memory
// instead of from hipMalloc or a caller's workspace.
//
// For callers that cannot allocate device memory (tight serving loops,
// harnesses that forbid allocation).  The evaluation builds a one-shot
// context inside the array (the same set-up, list build, density, embedding
// and force kernels as md_create + md_set_state + md_forces), reads the
// device status word, and tears the host side down again.
#include <hip/hip_runtime.h>

#include <mutex>

#include "md_internal.h"

namespace {

// 64 MiB per device, held from the first use of the library on that device
// until the process ends.
constexpr size_t kStaticBytes = size_t(64) << 20;

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// Device address of `scratch` on each device (its host-side name is only a
// stand-in for the symbol): looked up once per device, with that device
// current.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

int scratch_address(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return MD_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MD_ERR_DEVICE;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return MD_OK;
}

}  // namespace

extern "C" {

size_t md_static_bytes(void) { return kStaticBytes; }

int md_forces_static(const md_system *sys, const md_potential *pot, const double *pos,
                     double *f_out, double *e_atom, double *e_box, void *stream)
{
    if (!sys || !pot || !pos) return MD_ERR_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // the workspace this system needs, counted on the host
    md_ctx *h = nullptr;
    int rc = mdk::create_context(sys, pot, &h, nullptr, 0, mdk::kMeasure, nullptr);
    if (rc != MD_OK) return rc;
    const size_t need = h->c.alloc_bytes;
    md_destroy(h);
    h = nullptr;
    if (need > kStaticBytes) return MD_ERR_SCRATCH;
    void *base = nullptr;
    if ((rc = scratch_address(&base)) != MD_OK) return rc;
    // earlier evaluations on this stream may still read the array
    if (hipStreamSynchronize(s) != hipSuccess) return MD_ERR_DEVICE;
    rc = mdk::create_context(sys, pot, &h, base, kStaticBytes, mdk::kOneShot, s);
    if (rc != MD_OK) return rc;
    rc = md_set_state(h, pos, nullptr, stream);
    if (rc == MD_OK) rc = md_forces(h, f_out, e_atom, e_box, stream);
    unsigned w = 0;
    if (rc == MD_OK &&
        (hipMemcpyAsync(&w, h->c.dev.flags, sizeof(w), hipMemcpyDeviceToHost, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
        rc = MD_ERR_DEVICE;
    md_destroy(h);
    if (rc != MD_OK) return rc;
    if (w & (MD_FLAG_NLIST_OVERFLOW | MD_FLAG_TILE_OVERFLOW)) return MD_ERR_NLIST_OVERFLOW;
    if (w & MD_FLAG_NONFINITE) return MD_ERR_NONFINITE;
    if (w & MD_FLAG_TABLE_RANGE) return MD_ERR_TABLE_RANGE;
    return MD_OK;
}

}  // extern "C"
