// hmc_elastic.hip -- global quasi-static elastic state (Sec. 5) and lattice reductions.
//
// The periodic K^3 lattice carries one material point per site at the centre of a voxel
// whose 8 corners are background-grid nodes (K^3 nodes, periodic).  Unknowns: nodal
// displacement fluctuation u (3 planes of K^3) and macroscopic strain E (6); the strain of
// site v is E + B_v u, its stress C_{q_v} times that, and the load is the average stress
// Sigma.  One explicit step (damped dynamics written as a heavy ball, alpha = dt^2/m,
// beta = 1 - c dt):
//     r_n = -sum_{v at n} B_v(n)^T sigma_v,   w <- beta w + alpha r,   u <- u + w
//     r_E = Sigma - mean_v sigma_v,          wE <- beta wE + alphaE r_E,  E <- E + wE
// k_global_step does the node part for every node (reading u, writing the other u
// buffer, so no node sees a half-updated neighbour) and writes per-block sums of the
// stresses it formed; k_global_E folds those sums in a fixed order (deterministic) and
// advances E.  k_global_final writes the stress field the zone solves read.
#include "hmc_internal.h"

namespace hmc {

__device__ __forceinline__ int wrapk(int a, int K) { return a < 0 ? a + K : (a >= K ? a - K : a); }

__device__ __forceinline__ void symv21(const float* __restrict__ c, const float e[6], float s[6])
{
    s[0] = c[0] * e[0] + c[1] * e[1] + c[2] * e[2] + c[3] * e[3] + c[4] * e[4] + c[5] * e[5];
    s[1] = c[1] * e[0] + c[6] * e[1] + c[7] * e[2] + c[8] * e[3] + c[9] * e[4] + c[10] * e[5];
    s[2] = c[2] * e[0] + c[7] * e[1] + c[11] * e[2] + c[12] * e[3] + c[13] * e[4] + c[14] * e[5];
    s[3] = c[3] * e[0] + c[8] * e[1] + c[12] * e[2] + c[15] * e[3] + c[16] * e[4] + c[17] * e[5];
    s[4] = c[4] * e[0] + c[9] * e[1] + c[13] * e[2] + c[16] * e[3] + c[18] * e[4] + c[19] * e[5];
    s[5] = c[5] * e[0] + c[10] * e[1] + c[14] * e[2] + c[17] * e[3] + c[19] * e[4] + c[20] * e[5];
}

// Strain E + B_v u of voxel (vx,vy,vz) of the periodic grid.
__device__ __forceinline__ void voxel_strain(const float* __restrict__ u, int64_t n3, int K, int vx, int vy,
                                             int vz, const float E[6], float e[6])
{
    const int x1 = wrapk(vx + 1, K), y1 = wrapk(vy + 1, K), z1 = wrapk(vz + 1, K);
    const int64_t n[8] = {
        vx + (int64_t)K * (vy + (int64_t)K * vz), x1 + (int64_t)K * (vy + (int64_t)K * vz),
        vx + (int64_t)K * (y1 + (int64_t)K * vz), x1 + (int64_t)K * (y1 + (int64_t)K * vz),
        vx + (int64_t)K * (vy + (int64_t)K * z1), x1 + (int64_t)K * (vy + (int64_t)K * z1),
        vx + (int64_t)K * (y1 + (int64_t)K * z1), x1 + (int64_t)K * (y1 + (int64_t)K * z1)};
    float g[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float* uj = u + (int64_t)j * n3;
        const float c0 = uj[n[0]], c1 = uj[n[1]], c2 = uj[n[2]], c3 = uj[n[3]];
        const float c4 = uj[n[4]], c5 = uj[n[5]], c6 = uj[n[6]], c7 = uj[n[7]];
        g[j][0] = 0.25f * ((c1 - c0) + (c3 - c2) + (c5 - c4) + (c7 - c6));
        g[j][1] = 0.25f * ((c2 + c3) - (c0 + c1) + (c6 + c7) - (c4 + c5));
        g[j][2] = 0.25f * ((c4 + c5 + c6 + c7) - (c0 + c1 + c2 + c3));
    }
    e[0] = E[0] + g[0][0];
    e[1] = E[1] + g[1][1];
    e[2] = E[2] + g[2][2];
    e[3] = E[3] + g[1][2] + g[2][1];
    e[4] = E[4] + g[0][2] + g[2][0];
    e[5] = E[5] + g[0][1] + g[1][0];
}

// Deterministic block sum of NV doubles per thread into partials[blockIdx.x * 8 + k].
template <int NVALS>
__device__ __forceinline__ void block_sum_to(double* __restrict__ partials, const double v[NVALS])
{
    __shared__ double red[NVALS][256];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NVALS; ++k) red[k][t] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int k = 0; k < NVALS; ++k) red[k][t] += red[k][t + s];
        }
        __syncthreads();
    }
    if (t < NVALS) partials[(int64_t)blockIdx.x * 8 + t] = red[t][0];
}

struct GlobArgs {
    const int16_t* spins;
    const float* Ctab;
    const float* uin;
    float* uout;
    float* w;
    double* partials;
    const double* state;
    int K;
    int64_t n3;
    float alpha, beta;
};

__global__ __launch_bounds__(256) void k_global_step(GlobArgs a)
{
    const int K = a.K;
    float E[6];
#pragma unroll
    for (int I = 0; I < 6; ++I) E[I] = (float)a.state[kE + I];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < a.n3; n += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(n % K), y = (int)((n / K) % K), z = (int)(n / ((int64_t)K * K));
        float f[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int ca = c & 1, cb = (c >> 1) & 1, cc = c >> 2;
            const int vx = wrapk(x - ca, K), vy = wrapk(y - cb, K), vz = wrapk(z - cc, K);
            float e[6], s[6];
            voxel_strain(a.uin, a.n3, K, vx, vy, vz, E, e);
            const int g = a.spins[vx + (int64_t)K * (vy + (int64_t)K * vz)];
            symv21(a.Ctab + (int64_t)g * kTab, e, s);
            const float sx = ca ? 0.25f : -0.25f, sy = cb ? 0.25f : -0.25f, sz = cc ? 0.25f : -0.25f;
            f[0] += sx * s[0] + sy * s[5] + sz * s[4];
            f[1] += sx * s[5] + sy * s[1] + sz * s[3];
            f[2] += sx * s[4] + sy * s[3] + sz * s[2];
            if (c == 0) {
#pragma unroll
                for (int I = 0; I < 6; ++I) acc[I] += (double)s[I];
            }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int64_t idx = (int64_t)j * a.n3 + n;
            const float wn = a.beta * a.w[idx] - a.alpha * f[j];
            a.w[idx] = wn;
            a.uout[idx] = a.uin[idx] + wn;
        }
    }
    block_sum_to<6>(a.partials, acc);
}

struct EArgs {
    double* state;
    const double* partials;
    int nblocks;
    double inv_n3, betaE, alphaE;
    double Sigma[6];
};

// Folds the per-block stress sums (fixed order) and advances the macroscopic strain.
__global__ __launch_bounds__(256) void k_global_E(EArgs a)
{
    __shared__ double red[6][256];
    const int t = threadIdx.x;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int b = t; b < a.nblocks; b += 256)
#pragma unroll
        for (int I = 0; I < 6; ++I) s[I] += a.partials[(int64_t)b * 8 + I];
#pragma unroll
    for (int I = 0; I < 6; ++I) red[I][t] = s[I];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int I = 0; I < 6; ++I) red[I][t] += red[I][t + h];
        __syncthreads();
    }
    if (t < 6) {
        const double rE = a.Sigma[t] - red[t][0] * a.inv_n3;
        const double wE = a.betaE * a.state[kWE + t] + a.alphaE * rE;
        a.state[kWE + t] = wE;
        a.state[kE + t] += wE;
    }
}

struct FinalArgs {
    const int16_t* spins;
    const float* Ctab;
    const float* u;
    float* sigma;       // may be null
    double* partials;
    const double* state;
    int K;
    int64_t n3;
};

__global__ __launch_bounds__(256) void k_global_final(FinalArgs a)
{
    const int K = a.K;
    float E[6];
#pragma unroll
    for (int I = 0; I < 6; ++I) E[I] = (float)a.state[kE + I];
    double U[1] = {0.0};
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n3; v += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(v % K), y = (int)((v / K) % K), z = (int)(v / ((int64_t)K * K));
        float e[6], s[6];
        voxel_strain(a.u, a.n3, K, x, y, z, E, e);
        symv21(a.Ctab + (int64_t)a.spins[v] * kTab, e, s);
        double d = 0.0;
#pragma unroll
        for (int I = 0; I < 6; ++I) d += (double)s[I] * (double)e[I];
        U[0] += 0.5 * d;
        if (a.sigma)
#pragma unroll
            for (int I = 0; I < 6; ++I) a.sigma[(int64_t)I * a.n3 + v] = s[I];
    }
    block_sum_to<1>(a.partials, U);
}

__global__ __launch_bounds__(256) void k_sum_scalar(double* out, const double* partials, int nblocks)
{
    __shared__ double red[256];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int b = t; b < nblocks; b += 256) s += partials[(int64_t)b * 8];
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) *out = red[0];
}

struct ReussArgs {
    const int16_t* spins;
    const float* Stab;
    double* partials;
    int64_t n3;
    float Sig[6];
};

// Per-block sums of S_{q_v} Sigma (the uniform-stress strain of each site).
__global__ __launch_bounds__(256) void k_reuss(ReussArgs a)
{
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n3; v += (int64_t)gridDim.x * blockDim.x) {
        float e[6];
        symv21(a.Stab + (int64_t)a.spins[v] * kTab, a.Sig, e);
#pragma unroll
        for (int I = 0; I < 6; ++I) acc[I] += (double)e[I];
    }
    block_sum_to<6>(a.partials, acc);
}

// E = mean(S_q) Sigma, wE = 0.
__global__ __launch_bounds__(256) void k_reuss_E(double* state, const double* partials, int nblocks, double inv_n3)
{
    __shared__ double red[6][256];
    const int t = threadIdx.x;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int b = t; b < nblocks; b += 256)
#pragma unroll
        for (int I = 0; I < 6; ++I) s[I] += partials[(int64_t)b * 8 + I];
#pragma unroll
    for (int I = 0; I < 6; ++I) red[I][t] = s[I];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
#pragma unroll
            for (int I = 0; I < 6; ++I) red[I][t] += red[I][t + h];
        __syncthreads();
    }
    if (t < 6) {
        state[kE + t] = red[t][0] * inv_n3;
        state[kWE + t] = 0.0;
    }
}

__global__ void k_zero_wE(double* state)
{
    if (threadIdx.x < 6) state[kWE + threadIdx.x] = 0.0;
}

// ---- lattice reductions ----

template <int M>
__global__ __launch_bounds__(256) void k_unlike(const int16_t* spins, int K, int64_t n3, unsigned long long* out)
{
    unsigned long long cnt = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % K), y = (int)((i / K) % K), z = (int)(i / ((int64_t)K * K));
        const int q = spins[i];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            int dx, dy, dz;
            if (M == 6) {
                dx = (k == 0) ? -1 : (k == 1 ? 1 : 0);
                dy = (k == 2) ? -1 : (k == 3 ? 1 : 0);
                dz = (k == 4) ? -1 : (k == 5 ? 1 : 0);
            } else {
                const int n = k + (k >= 13);
                dx = n % 3 - 1;
                dy = (n / 3) % 3 - 1;
                dz = n / 9 - 1;
            }
            cnt += (spins[wrapk(x + dx, K) + (int64_t)K * (wrapk(y + dy, K) + (int64_t)K * wrapk(z + dz, K))] != q);
        }
    }
    // wave sum then one atomic per wave (integers: order-free)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if (__lane_id() == 0 && cnt) atomicAdd(out, cnt);
}

__global__ __launch_bounds__(256) void k_texture(const int16_t* spins, const int32_t* bin, int64_t n3, int nbins,
                                                 unsigned long long* hist)
{
    __shared__ unsigned int h[64];
    if (threadIdx.x < 64) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[bin[spins[i]]], 1u);
    __syncthreads();
    if (threadIdx.x < nbins && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// ---- launchers ----

static int reduce_blocks(int64_t n3)
{
    int64_t b = (n3 + 255) / 256;
    if (b > kMaxPartials) b = kMaxPartials;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_reuss(hmc_ctx_s* c)
{
    ReussArgs a;
    a.spins = c->d.spins;
    a.Stab = c->d.Stab;
    a.partials = c->d.partials;
    a.n3 = c->n3;
    for (int I = 0; I < 6; ++I) a.Sig[I] = (float)c->sigma_GPa[I];
    const int nb = reduce_blocks(c->n3);
    hipLaunchKernelGGL(k_reuss, dim3(nb), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL(k_reuss_E, dim3(1), dim3(256), 0, c->stream, c->d.state, c->d.partials, nb, 1.0 / (double)c->n3);
    return hipGetLastError();
}

hipError_t launch_global_steps(hmc_ctx_s* c, int n_steps)
{
    const int nb = reduce_blocks(c->n3);
    GlobArgs a;
    a.spins = c->d.spins;
    a.Ctab = c->d.Ctab;
    a.w = c->d.w;
    a.partials = c->d.partials;
    a.state = c->d.state;
    a.K = c->p.K;
    a.n3 = c->n3;
    a.alpha = (float)c->p.glob_alpha;
    a.beta = (float)c->p.glob_beta;
    EArgs ea;
    ea.state = c->d.state;
    ea.partials = c->d.partials;
    ea.nblocks = nb;
    ea.inv_n3 = 1.0 / (double)c->n3;
    ea.betaE = c->p.glob_beta;
    ea.alphaE = c->p.glob_alphaE;
    for (int I = 0; I < 6; ++I) ea.Sigma[I] = c->sigma_GPa[I];
    for (int s = 0; s < n_steps; ++s) {
        a.uin = c->d.u[c->cur_u];
        a.uout = c->d.u[1 - c->cur_u];
        int tok = prof_begin(c, kProfRefreshStep);
        hipLaunchKernelGGL(k_global_step, dim3(nb), dim3(256), 0, c->stream, a);
        prof_end(c, tok);
        tok = prof_begin(c, kProfRefreshOther);
        hipLaunchKernelGGL(k_global_E, dim3(1), dim3(256), 0, c->stream, ea);
        prof_end(c, tok);
        c->cur_u = 1 - c->cur_u;
    }
    return hipGetLastError();
}

hipError_t launch_global_final(hmc_ctx_s* c, bool write_sigma)
{
    const int nb = reduce_blocks(c->n3);
    FinalArgs a;
    a.spins = c->d.spins;
    a.Ctab = c->d.Ctab;
    a.u = c->d.u[c->cur_u];
    a.sigma = write_sigma ? c->d.sigma : nullptr;
    a.partials = c->d.partials;
    a.state = c->d.state;
    a.K = c->p.K;
    a.n3 = c->n3;
    const int tok = prof_begin(c, kProfRefreshOther);
    hipLaunchKernelGGL(k_global_final, dim3(nb), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL(k_sum_scalar, dim3(1), dim3(256), 0, c->stream, c->d.state + kU, c->d.partials, nb);
    prof_end(c, tok);
    return hipGetLastError();
}

hipError_t launch_zero_wE(hmc_ctx_s* c)
{
    hipLaunchKernelGGL(k_zero_wE, dim3(1), dim3(64), 0, c->stream, c->d.state);
    return hipGetLastError();
}

hipError_t launch_unlike_bonds(hmc_ctx_s* c)
{
    int64_t g = (c->n3 + 255) / 256;
    if (g > 4096) g = 4096;
    if (c->p.neighbors == 26)
        hipLaunchKernelGGL(k_unlike<26>, dim3((unsigned)g), dim3(256), 0, c->stream, c->d.spins, c->p.K, c->n3, c->d.bonds);
    else
        hipLaunchKernelGGL(k_unlike<6>, dim3((unsigned)g), dim3(256), 0, c->stream, c->d.spins, c->p.K, c->n3, c->d.bonds);
    return hipGetLastError();
}

hipError_t launch_texture(hmc_ctx_s* c, int nbins)
{
    int64_t g = (c->n3 + 255) / 256;
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_texture, dim3((unsigned)g), dim3(256), 0, c->stream, c->d.spins, c->d.tex_bin, c->n3, nbins,
                       c->d.hist);
    return hipGetLastError();
}

}  // namespace hmc
