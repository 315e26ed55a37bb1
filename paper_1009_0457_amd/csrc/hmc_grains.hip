// hmc_grains.hip -- grains of a spin field: the face-connected clusters of equal spins on the
// periodic lattice, the measure behind the mean grain volume V(t) of the grain-growth law of
// Sec. 6 (V^(2/3) linear in t).
//
// Labels start as the site index and only ever decrease to the index of a same-spin face
// neighbour's label, so every label is always the index of a site of the same grain; their
// fixed point gives each grain the smallest site index it contains, whatever the order in which
// threads see each other's updates.  Each round is a propagation pass (a site takes the smallest
// label among itself and its same-spin face neighbours, written in place: only its own thread
// writes it) and a pointer jump (label <- label of the label, which lies in the same grain).
// The host repeats rounds until a round changes nothing, then counts the sites that are their
// own label.  Every round either changes a label to a strictly smaller value or ends the loop.
#include "hmc_internal.h"

namespace hmc {

namespace {

__global__ __launch_bounds__(256) void k_label_init(int32_t* lab, int64_t n3)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n3; v += (int64_t)gridDim.x * blockDim.x)
        lab[v] = (int32_t)v;
}

__global__ __launch_bounds__(256) void k_label_propagate(const int16_t* __restrict__ spins, int32_t* lab, int K,
                                                         uint32_t* changed)
{
    const int64_t n3 = (int64_t)K * K * K, KK = (int64_t)K * K;
    bool any = false;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n3; v += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(v % K), y = (int)((v / K) % K), z = (int)(v / KK);
        const int16_t s = spins[v];
        const int64_t nb[6] = {(x + 1 < K ? v + 1 : v + 1 - K), (x > 0 ? v - 1 : v - 1 + K),
                               (y + 1 < K ? v + K : v + K - KK), (y > 0 ? v - K : v - K + KK),
                               (z + 1 < K ? v + KK : v + KK - n3), (z > 0 ? v - KK : v - KK + n3)};
        const int32_t old = lab[v];
        int32_t m = old;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if (spins[nb[k]] == s) {
                const int32_t l = lab[nb[k]];
                m = l < m ? l : m;
            }
        if (m < old) {
            lab[v] = m;
            any = true;
        }
    }
    if (__any(any) && (threadIdx.x & 63) == 0) *changed = 1u;
}

__global__ __launch_bounds__(256) void k_label_jump(int32_t* lab, int64_t n3)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n3; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t l = lab[v];
        const int32_t ll = lab[l];
        if (ll < l) lab[v] = ll;
    }
}

__global__ __launch_bounds__(256) void k_label_roots(const int32_t* lab, int64_t n3, unsigned long long* count)
{
    uint32_t n = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n3; v += (int64_t)gridDim.x * blockDim.x)
        n += lab[v] == (int32_t)v ? 1u : 0u;
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    __shared__ uint32_t s[4];
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(count, (unsigned long long)(s[0] + s[1] + s[2] + s[3]));
}

unsigned grid_of(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

hipError_t launch_grain_labels(hmc_ctx_s* c, int rep, int32_t* lab, int64_t* n_grains, int* rounds)
{
    const RepDev& R = c->reps[rep];
    const int64_t n3 = R.n3;
    const unsigned g = grid_of(n3);
    const int16_t* spins = c->d.spins + R.site_off;
    uint32_t* changed = c->d.counters + kLabelChanged;
    hipLaunchKernelGGL(k_label_init, dim3(g), dim3(256), 0, c->stream, lab, n3);
    hipError_t e = hipGetLastError();
    int r = 0;
    // each round lowers at least one label or ends the loop, so n3 rounds always suffice
    for (; e == hipSuccess && r < n3 + 1; ++r) {
        uint32_t h = 0;
        e = launch_fill_u32(changed, 0u, 1, c->stream);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_label_propagate, dim3(g), dim3(256), 0, c->stream, spins, lab, R.K, changed);
        hipLaunchKernelGGL(k_label_jump, dim3(g), dim3(256), 0, c->stream, lab, n3);
        e = hipMemcpyAsync(&h, changed, sizeof h, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess || h == 0u) break;
    }
    if (rounds) *rounds = r + 1;
    if (e != hipSuccess) return e;
    unsigned long long cnt = 0;
    e = hipMemsetAsync(c->d.bonds, 0, sizeof(unsigned long long), c->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_label_roots, dim3(g), dim3(256), 0, c->stream, (const int32_t*)lab, n3, c->d.bonds);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&cnt, c->d.bonds, sizeof cnt, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    *n_grains = (int64_t)cnt;
    return e;
}

}  // namespace hmc
