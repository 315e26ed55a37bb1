// hmc_noalloc.hip -- hmc_texture_histogram_noalloc: the volume-weighted texture histogram of
// hmc_texture_histogram (the Sec. 7 orientation measure) for a caller's spin field and
// orientations, without a context and without any device allocation, for callers that
// cannot allocate or provide a workspace.
//
// Its scratch memory (the per-grain bin table, the 64 histogram bins and an error flag) is
// the file-scope device array `scratch` below, which every GPU the library runs on holds until
// the process ends.  Host code never passes the array's name to a kernel or a copy: on each
// device its address is taken once with hipGetSymbolAddress (that device current) and kept
// per device.  Every call on a device shares that device's array, so calls that overlap on one
// GPU (different streams or threads) race; calls on one stream are ordered.
#include <cmath>
#include <mutex>
#include <string>

#include "hmc_internal.h"

namespace hmc {

namespace {

constexpr int kNaMaxQ = 32767;                 // grains (the library's limit)
constexpr size_t kNaFlag = 0;                  // uint32: a spin outside [0, Q)
constexpr size_t kNaHist = 256;                // 64 uint64 bins
constexpr size_t kNaBins = 1024;               // Q int32 per-grain bins
constexpr size_t kNaBytes = (kNaBins + sizeof(int32_t) * kNaMaxQ + 255) / 256 * 256;   // 132 352 bytes

static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kNaMaxDevices = 64;
std::mutex g_addr_mu;
unsigned char* g_addr[kNaMaxDevices] = {};     // per device: scratch's address there

// Host bin table of the call in progress: a fixed array, so that a call allocates nothing on
// the host either; the lock is held until the call's stream is synchronised, which is after
// the copy that reads it.
std::mutex g_bins_mu;
int32_t g_bins[kNaMaxQ];

// The scratch array's device address on the current device (taken once per device).
hipError_t scratch_address(unsigned char** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kNaMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_addr_mu);
    if (!g_addr[(size_t)dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_addr[(size_t)dev] = (unsigned char*)p;
    }
    *out = g_addr[(size_t)dev];
    return hipSuccess;
}

// Zeroes the error flag and the histogram: the previous call's contents stay in the array.
__global__ void k_na_clear(unsigned char* s)
{
    if (threadIdx.x == 0) *(uint32_t*)(s + kNaFlag) = 0u;
    if (threadIdx.x < 64) ((unsigned long long*)(s + kNaHist))[threadIdx.x] = 0ull;
}

// One count per site in the bin of its grain; a spin outside [0, Q) raises the flag and is
// not counted (it would index outside the bin table).
__global__ __launch_bounds__(256) void k_na_hist(const int32_t* __restrict__ spins, int64_t n3, int32_t Q, int nbins,
                                                 unsigned char* s)
{
    __shared__ unsigned int h[64];
    const int32_t* bins = (const int32_t*)(s + kNaBins);
    if (threadIdx.x < 64) h[threadIdx.x] = 0;
    __syncthreads();
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t q = spins[i];
        if (q < 0 || q >= Q)
            bad = true;
        else
            atomicAdd(&h[bins[q]], 1u);
    }
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr((uint32_t*)(s + kNaFlag), 1u);
    __syncthreads();
    if (threadIdx.x < nbins && h[threadIdx.x])
        atomicAdd(&((unsigned long long*)(s + kNaHist))[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

hmc_status na_fail(hmc_status st, const char* what, hipError_t e = hipSuccess)
{
    std::string m = what;
    if (e != hipSuccess) {
        m += ": ";
        m += hipGetErrorString(e);
    }
    set_thread_error(m.c_str());
    return st;
}

}  // namespace

}  // namespace hmc

using namespace hmc;

extern "C" hmc_status hmc_texture_histogram_noalloc(const int32_t* spins_dev, int32_t K, int32_t Q,
                                                    const double* euler_host, const double axis[3], double bin_deg,
                                                    int32_t nbins, int64_t* counts_host, hipStream_t stream)
{
    set_thread_error("");
    if (!spins_dev || !euler_host || !axis || !counts_host) return na_fail(HMC_EINVAL, "null argument");
    if (K < 1 || K > 1024) return na_fail(HMC_ESHAPE, "need 1 <= K <= 1024");
    if (Q < 1 || Q > kNaMaxQ) return na_fail(HMC_ESHAPE, "need 1 <= Q <= 32767 (the scratch array's bin table)");
    if (nbins < 1 || nbins > 64 || !(bin_deg > 0) || !std::isfinite(bin_deg))
        return na_fail(HMC_EINVAL, "need 1 <= nbins <= 64 and bin_deg > 0");
    const double nrm = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    if (!(nrm > 0) || !std::isfinite(nrm)) return na_fail(HMC_EINVAL, "axis must be finite and non-zero");
    for (int64_t i = 0; i < 3 * (int64_t)Q; ++i)
        if (!std::isfinite(euler_host[i])) return na_fail(HMC_ENUMERIC, "non-finite Euler angle");
    std::lock_guard<std::mutex> bins_lock(g_bins_mu);
    texture_bins(euler_host, Q, axis, bin_deg, nbins, g_bins);

    unsigned char* s = nullptr;
    hipError_t e = scratch_address(&s);
    if (e != hipSuccess) return na_fail(HMC_EDEVICE, "address of the scratch array", e);
    const int64_t n3 = (int64_t)K * K * K;
    int64_t g = (n3 + 255) / 256;
    if (g > 2048) g = 2048;
    unsigned long long h[64];
    uint32_t flag = 0;
    e = hipMemcpyAsync(s + kNaBins, g_bins, (size_t)Q * sizeof(int32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_na_clear, dim3(1), dim3(64), 0, stream, s);
        hipLaunchKernelGGL(k_na_hist, dim3((unsigned)g), dim3(256), 0, stream, spins_dev, n3, Q, (int)nbins, s);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(h, s + kNaHist, sizeof h, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, s + kNaFlag, sizeof flag, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return na_fail(HMC_EDEVICE, "texture histogram", e);
    if (flag) return na_fail(HMC_EINVAL, "spin value outside [0, Q)");
    for (int b = 0; b < nbins; ++b) counts_host[b] = (int64_t)h[b];
    return HMC_OK;
}
