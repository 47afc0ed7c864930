// gv_noalloc.hip -- gv_energy_grad for callers that cannot allocate device
// memory: the state vector, the adjoint vector and every table and partial
// sum live in one library-owned device array instead of caller buffers.
//
// The array is a file-scope __device__ object, so every GPU the library runs
// on holds its own copy from module load until the process ends.  Its
// address differs per device and is not the host-side symbol: it is looked up
// once per device with hipGetSymbolAddress (with that device current) and
// only that address is handed to kernels.  Every call on one device shares
// the array, so calls that overlap on one GPU (different streams, or threads)
// race.  No kernel of the uncompute sweep reads scratch memory it has not
// written in the same call (every partial-sum column and vector entry is
// written before it is read), so nothing has to be cleared between calls.
#include <mutex>

#include "gv_internal.hpp"

namespace gv {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // GV_NOALLOC_SCRATCH_BYTES
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices];

// The device address of this device's copy of `scratch` (looked up once).
gv_status scratch_ptr(void **out)
{
    int dev = 0;
    if (gv_status r = check_hip(hipGetDevice(&dev), "hipGetDevice")) return r;
    if (dev < 0 || dev >= kMaxDevices) return set_error(GV_EUNSUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (gv_status r = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                                    "hipGetSymbolAddress(scratch)"))
            return r;
        if (!p) return set_error(GV_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return GV_OK;
}

}  // namespace

}  // namespace gv

using namespace gv;

extern "C" {

gv_status gv_energy_grad_noalloc(int32_t n, gv_precision prec, gv_pauli_sum h,
                                 const double *params_dev, const gv_ansatz *a,
                                 const uint8_t *grad_mask_dev, double *energy_dev,
                                 double *grad_dev, void *stream)
{
    if (!h || !params_dev || !a || !energy_dev || !grad_dev)
        return set_error(GV_EINVAL, "NULL argument");
    if (n < 1 || n > kMaxQubits) return set_error(GV_EINVAL, "n=%d outside 1..%d", n, kMaxQubits);
    if (prec != GV_C64 && prec != GV_C128) return set_error(GV_EINVAL, "precision %d", prec);
    if (a->n != n) return set_error(GV_ESTATE, "ansatz n=%d but n=%d", a->n, n);
    WorkLayout w;
    if (gv_status r = work_layout(*a, prec, GV_ENGINE_FUSED, GV_GRAD_UNCOMPUTE, &w)) return r;
    const size_t sb = align_up(((size_t)1 << n) * amp_bytes(prec));
    if (sb + w.total > kScratchBytes)
        return set_error(GV_ESIZE,
                         "n=%d needs %zu scratch bytes (state %zu + work %zu); the library's "
                         "static scratch holds %zu",
                         n, sb + w.total, sb, w.total, kScratchBytes);
    void *base = nullptr;
    if (gv_status r = scratch_ptr(&base)) return r;
    gv_state_s st;
    st.n = n;
    st.prec = prec;
    st.engine = GV_ENGINE_FUSED;
    st.amps = base;
    st.amps_bytes = sb;
    st.work = (char *)base + sb;
    st.work_bytes = w.total;
    st.stream = (hipStream_t)stream;
    return gv_energy_grad(&st, h, params_dev, a, grad_mask_dev, GV_GRAD_UNCOMPUTE, energy_dev,
                          grad_dev);
}

size_t gv_noalloc_scratch_bytes(void) { return kScratchBytes; }

}  // extern "C"
