// The solve for callers that cannot allocate memory (nair_solve_noalloc):
// nair_solve's stationary iteration on a set-up single-system hierarchy, with
// every buffer that iteration would otherwise allocate -- the norm chunk
// tables and their partial sums, the per-system state and counters, the
// residual history -- carved from one file-scope device array.  No hipMalloc,
// hipFree or other allocating call is made; host bookkeeping stays on the
// stack.
//
// The array is one per device (each GPU the library runs on holds its own
// copy until the process ends) and every call on a device shares it, keeping
// the last call's contents: everything the iteration reads is initialised by
// kernels at the start of each call, and calls that overlap on one device
// race.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address comes from hipGetSymbolAddress, once per device
// (at the setup of a single-system hierarchy on it, which also loads this
// file's kernels there), and only that address is ever passed to kernels.
#include <algorithm>
#include <mutex>
#include <string>

#include "hier.h"

namespace nair {
namespace {

constexpr int64_t kScratchWords = NAIR_NOALLOC_SCRATCH_BYTES / sizeof(double);
__device__ __align__(256) double scratch[kScratchWords];

constexpr int kMaxDevices = 64;

struct ScratchAddr {
    std::mutex mu;
    double *ptr[kMaxDevices] = {};
};

ScratchAddr &scratch_addr() {
    static ScratchAddr a;
    return a;
}

// The device address of this device's scratch array (the current device).
double *scratch_ptr() {
    int dev = 0;
    NAIR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(NAIR_EDEVICE, "device index out of range for the scratch table");
    ScratchAddr &a = scratch_addr();
    std::lock_guard<std::mutex> lk(a.mu);
    if (!a.ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(NAIR_EDEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
        a.ptr[dev] = static_cast<double *>(p);
    }
    return a.ptr[dev];
}

// x = 0; the norm chunks of one system of n dofs (chunk c: dofs [c K, min(n, (c+1) K)));
// the tolerance.
__global__ __launch_bounds__(256) void k_noalloc_prep(double *__restrict__ x, int64_t n, int64_t *__restrict__ clo,
                                                     int *__restrict__ clen, int *__restrict__ cptr, int nchunk,
                                                     double *__restrict__ rtol, double rtol_v) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n; g += stride) x[g] = 0.0;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < nchunk; g += stride) {
        const int64_t rem = n - g * kSolveChunk;
        clo[g] = g * kSolveChunk;
        clen[g] = rem < kSolveChunk ? static_cast<int>(rem) : kSolveChunk;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        cptr[0] = 0;
        cptr[1] = nchunk;
        *rtol = rtol_v;
    }
}

// Words of the scratch array a solve of n dofs with max_iter iterations takes.
int64_t words_needed(int64_t n, int max_iter, int64_t *nchunk) {
    const int64_t nch = std::max<int64_t>((n + kSolveChunk - 1) / kSolveChunk, 1);
    *nchunk = nch;
    // part, clo, clen (ints), cptr, bn/last/rtol, six int counters, history
    return nch + nch + (nch + 1) / 2 + 1 + 3 + 3 + std::max(max_iter, 1);
}

}  // namespace

void noalloc_prepare() { (void)scratch_ptr(); }

nair_status solve_noalloc(Hier &h, const double *b, double *x, double rtol, int max_iter, nair_result *res,
                          hipStream_t s) {
    if (h.nsys != 1) fail(NAIR_EINVAL, "nair_solve_noalloc takes single-system handles");
    if (h.prm.gmres > 0) fail(NAIR_EINVAL, "nair_solve_noalloc runs the stationary iteration (gmres = 0)");
    for (size_t l = 1; h.prm.cycle == 1 && l < h.lv.size(); ++l)   // allocated by the setup
        if (h.prm.precision == 1 ? !h.lv[l]->fsave32.get() : !h.lv[l]->fsave.get())
            fail(NAIR_EDEVICE, "nair_solve_noalloc: the F-cycle's saved vectors are missing");
    Level &L0 = *h.lv[0];
    const int64_t n = static_cast<int64_t>(L0.A.nb) * h.bs;
    int64_t nch = 0;
    const int64_t need = words_needed(n, max_iter, &nch);
    if (need > kScratchWords)
        fail(NAIR_EINVAL, "nair_solve_noalloc: " + std::to_string(n) + " dofs and max_iter " + std::to_string(max_iter) +
                              " need " + std::to_string(need * 8) + " bytes of scratch, more than its " +
                              std::to_string(kScratchWords * 8) + " (use nair_solve)");
    double *base = scratch_ptr();
    SolveBufs V;
    V.nchunk = static_cast<int>(nch);
    V.hist_cap = std::max(max_iter, 1);
    double *p = base;
    V.part = p;
    p += nch;
    V.clo = reinterpret_cast<int64_t *>(p);
    p += nch;
    V.clen = reinterpret_cast<int *>(p);
    p += (nch + 1) / 2;
    V.cptr = reinterpret_cast<int *>(p);
    p += 1;
    V.bn = p;
    V.last = p + 1;
    V.rtol = p + 2;
    p += 3;
    int *ip = reinterpret_cast<int *>(p);
    V.active = ip;
    V.status = ip + 1;
    V.iters = ip + 2;
    V.it = ip + 3;
    V.nact = ip + 4;
    V.nact_acc = ip + 5;
    p += 3;
    V.hist = p;
    const int64_t work = std::max(n, nch);
    k_noalloc_prep<<<grid_for(work, 256), 256, 0, s>>>(x, n, V.clo, V.clen, V.cptr, V.nchunk, V.rtol, rtol);
    NAIR_HIP(hipGetLastError());
    return run_solve_bufs(h, b, x, rtol, max_iter, res, s, V);
}

}  // namespace nair
