// Device memory that exists without an allocation call, one copy per GPU the
// library runs on (held until the process ends):
//   * the float32 twiddle table exp(-2 pi i t / N), t < N, of every transform
//     length the library supports (even N in 8..512 of the form 2^a 3^b 5^c),
//     each rounded once from a double evaluation; every plan points into it;
//   * the scratch array of fvr_reconstruct_noalloc, whose callers cannot
//     allocate device memory.
// Host code never passes the arrays' names to a kernel: at set-up, once per
// device and with that device current, their addresses are looked up with
// hipGetSymbolAddress and kept, and only those addresses are used.
#include <cmath>
#include <mutex>
#include <vector>

#include "fvr.h"
#include "fvr_common.h"

namespace fvr {

namespace {

constexpr bool supported_length(int n) {
    if (n < 8 || n > kMaxDim || (n & 1)) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    while (n % 5 == 0) n /= 5;
    return n == 1;
}

constexpr int twiddle_total() {
    int t = 0;
    for (int n = 8; n <= kMaxDim; n += 2)
        if (supported_length(n)) t += n;
    return t;
}

constexpr int kTwiddleTotal = twiddle_total();
constexpr int kMaxDevices = 64;

static __device__ __align__(256) float2 twiddle_table[kTwiddleTotal];
static __device__ __align__(256) unsigned char scratch[FVR_NOALLOC_SCRATCH_BYTES];

struct DeviceStatics {
    bool ready = false;
    float2 *twiddles = nullptr;
    unsigned char *scratch = nullptr;
};

std::mutex g_mutex;
DeviceStatics g_dev[kMaxDevices];

}  // namespace

int twiddle_offset(int n) {
    if (!supported_length(n)) return -1;
    int t = 0;
    for (int k = 8; k < n; k += 2)
        if (supported_length(k)) t += k;
    return t;
}

hipError_t statics_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mutex);
    DeviceStatics &d = g_dev[device];
    if (d.ready) return hipSuccess;
    // the caller made `device` current
    void *tw = nullptr, *sc = nullptr;
    hipError_t e = hipGetSymbolAddress(&tw, HIP_SYMBOL(twiddle_table));
    if (e != hipSuccess) return e;
    e = hipGetSymbolAddress(&sc, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    std::vector<float2> tab((size_t)kTwiddleTotal);
    for (int n = 8; n <= kMaxDim; n += 2) {
        if (!supported_length(n)) continue;
        const int off = twiddle_offset(n);
        for (int t = 0; t < n; ++t) {
            const double ang = 2.0 * M_PI * (double)t / (double)n;
            tab[(size_t)off + t] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
        }
    }
    e = hipMemcpy(tw, tab.data(), tab.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    d.twiddles = static_cast<float2 *>(tw);
    d.scratch = static_cast<unsigned char *>(sc);
    d.ready = true;
    return hipSuccess;
}

const float2 *statics_twiddles(int device, int n) {
    if (device < 0 || device >= kMaxDevices || !g_dev[device].ready) return nullptr;
    const int off = twiddle_offset(n);
    return off < 0 ? nullptr : g_dev[device].twiddles + off;
}

unsigned char *statics_scratch(int device) {
    if (device < 0 || device >= kMaxDevices || !g_dev[device].ready) return nullptr;
    return g_dev[device].scratch;
}

}  // namespace fvr
