// Block inner product without allocation: hsym_kernel_gram_noalloc.
//
// The Gram products write one partial (K1 x K2) per row slice and then reduce
// the partials in a fixed order.  hsym_kernel_gram allocates that partial
// buffer per call; this entry point takes it from a file-scope device array
// instead, sized for the largest Gram the solver forms (K1 <= 48, K2 <= 96,
// at most 1024 row slices: 36 MiB per GPU, held until the process ends).
//
// The array's host-side name is only a stand-in for the symbol: its device
// address is looked up with hipGetSymbolAddress once per device (with that
// device current) on the first call there, and only that address is handed
// to the kernels.
#include <cstring>
#include <mutex>

#include "../../include/hsym_kernels.h"
#include "dense.h"

namespace hsym {
namespace {

constexpr size_t NOALLOC_PARTS = 1024, NOALLOC_K1 = 48, NOALLOC_K2 = 96;
constexpr size_t NOALLOC_DOUBLES = NOALLOC_PARTS * NOALLOC_K1 * NOALLOC_K2;

__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_ptr[MAX_DEVICES] = {};

// device address of this device's copy of the array (the current device)
double *device_scratch() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) fail(HSYM_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(HSYM_E_DEVICE, std::string("hipGetSymbolAddress of the Gram scratch: ") + hipGetErrorString(e));
        }
        scratch_ptr[dev] = (double *)p;
    }
    return scratch_ptr[dev];
}

}  // namespace
}  // namespace hsym

using namespace hsym;

extern "C" int hsym_kernel_gram_noalloc(int64_t n, int m, int na, const double *const *A, int nb,
                                        const double *const *B, double *G, void *stream) {
    try {
        if (n < 1 || m < 1 || m > HSYM_MAX_BLOCK) fail(HSYM_E_INVALID_ARG, "need n >= 1 and 1 <= m <= 16");
        if (na < 1 || na > 3 || nb < 1 || nb > 6 || !A || !B || !G) fail(HSYM_E_INVALID_ARG, "bad gram arguments");
        const size_t need = gram_scratch_bytes(n, na * m, nb * m);
        if (need > NOALLOC_DOUBLES * sizeof(double))
            fail(HSYM_E_INVALID_ARG, "Gram partials of " + std::to_string(need) + " bytes exceed the " +
                                         std::to_string(NOALLOC_DOUBLES * sizeof(double)) + "-byte static scratch");
        GramArgs g{};
        for (int i = 0; i < na; i++) g.a[i] = A[i];
        for (int i = 0; i < nb; i++) g.b[i] = B[i];
        g.na = na; g.nb = nb; g.m = m; g.n = n;
        gram(g, G, device_scratch(), (hipStream_t)stream);
        set_error("");
        return HSYM_OK;
    } catch (Error &e) {
        set_error(e.msg);
        return e.status;
    } catch (std::bad_alloc &) {
        set_error("host allocation failed");
        return HSYM_E_OUT_OF_MEMORY;
    }
}
