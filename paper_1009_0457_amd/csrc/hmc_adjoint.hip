// hmc_adjoint.hip -- reverse-mode derivative of the global explicit elastic solve (Sec. 5)
// with respect to the per-grain Euler angles and the applied stress.
//
// Forward (as hmc_stress_refresh with a cold start): E_0 = mean(S_q) Sigma, u_0 = w_0 = 0,
// then n explicit steps; U = 1/2 sum_v eps_v . C_v eps_v at the final state.  With the state
// of step t written (u_t, w_t, E_t, wE_t), the adjoint runs the recurrence backwards:
//
//   w~ = w^_{t+1} + u^_{t+1},  a = alpha w~          (nodal)
//   wE~ = wE^_{t+1} + E^_{t+1}, b = alphaE wE~       (6)
//   eta_v = B_v a + b / K^3,  tau_v = C_v eta_v      (per voxel: the adjoint stress)
//   u^_t = u^_{t+1} - sum_v B_v^T tau_v,   w^_t = beta w~
//   E^_t = E^_{t+1} - sum_v tau_v,         wE^_t = beta wE~
//   dU/dtheta_g += -sum_{v in g} eta_v . (dC_g/dtheta) eps_{t,v},   dU/dSigma += b
//
// from u^_n = sum_v B_v^T sigma_v, E^_n = sum_v sigma_v, w^_n = wE^_n = 0 and the direct
// term dU/dtheta_g += sum_{v in g} 1/2 eps_v . (dC_g/dtheta) eps_v; after step 0 the start
// E_0 = mean(S_q) Sigma adds E^_0 . (n_g/K^3) (dS_g/dtheta) Sigma and mean(S) E^_0.
//
// The stiffness-derivative terms are contracted with the voxel's dC/dtheta (three angles)
// as they arise and summed per voxel in FP64: G_v = 1/2 eps_n.dC eps_n - sum_t eta_t.dC eps_t;
// per-grain sums of G use 64-bit fixed-point atomics (order-independent, so the result is
// deterministic).  Forward states are recovered from checkpoints every `ckpt_every` steps
// by recomputing one segment at a time.  The adjoint step is tiled like the forward step.
#include <cmath>
#include <cstring>
#include <vector>

#include "hmc_device.h"

namespace hmc {

constexpr double kFixScale = 1099511627776.0;   // 2^40

struct AdjLayout {
    size_t ckpt, seg_u, seg_E, ub0, ub1, wb0, wb1, G, dC, dS, adj, grad, total;
    int n_ck;          // checkpoints of segment starts
    size_t ck_bytes;   // bytes per checkpoint: u, w planes then 12 doubles
};

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

static AdjLayout adj_layout(const hmc_ctx_s* c, int n_steps, int k)
{
    AdjLayout L{};
    const size_t n3 = (size_t)c->reps[0].n3;
    const size_t Q = (size_t)c->reps[0].Q;
    L.n_ck = (n_steps + k - 1) / k + 1;          // + the final state
    L.ck_bytes = al256(6 * n3 * sizeof(float)) + 256;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t at = o;
        o = al256(o + b);
        return at;
    };
    L.ckpt = take((size_t)L.n_ck * L.ck_bytes);
    L.seg_u = take((size_t)(k + 1) * 3 * n3 * sizeof(float));
    L.seg_E = take((size_t)(k + 1) * 8 * sizeof(double));
    L.ub0 = take(3 * n3 * sizeof(float));
    L.ub1 = take(3 * n3 * sizeof(float));
    L.wb0 = take(3 * n3 * sizeof(float));
    L.wb1 = take(3 * n3 * sizeof(float));
    L.G = take(3 * n3 * sizeof(double));
    L.dC = take(Q * 3 * kTab * sizeof(float));
    L.dS = take(Q * 3 * kTab * sizeof(float));
    L.adj = take(64 * sizeof(double));
    L.grad = take(Q * 3 * sizeof(unsigned long long));
    L.total = o;
    return L;
}

// Slots of the adjoint's small state block.
enum AdjSlot { kEb = 0, kWEb = 6, kB = 12, kSigb = 18, kWEt = 24, kE0 = 30, kAdjDoubles = 64 };

// eta . (dC_q eps) for the three angles q of grain g
__device__ __forceinline__ void angle_contractions(const float* __restrict__ dC, int g, const float eta[6],
                                                  const float eps[6], double out[3])
{
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        float d6[6];
        symv21(dC + ((int64_t)g * 3 + q) * kTab, eps, d6);
        double v = 0.0;
#pragma unroll
        for (int I = 0; I < 6; ++I) v += (double)eta[I] * (double)d6[I];
        out[q] = v;
    }
}

struct AdjInitArgs {
    const int16_t* spins;
    const float* Ctab;
    const float* dC;
    const float* u;
    float* ub;
    float* wb;
    double* G;
    double* partials;
    const double* state;
    int K;
    int64_t n3;
};

// Final-state adjoint: u^_n = sum_v B_v^T sigma_v, G_v = 1/2 eps.dC eps, partial sums of sigma.
__global__ __launch_bounds__(256) void k_adj_init(AdjInitArgs a)
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
            voxel_strain(a.u, a.n3, K, vx, vy, vz, E, e);
            const int g = a.spins[vx + (int64_t)K * (vy + (int64_t)K * vz)];
            symv21(a.Ctab + (int64_t)g * kTab, e, s);
            const float sx = ca ? 0.25f : -0.25f, sy = cb ? 0.25f : -0.25f, sz = cc ? 0.25f : -0.25f;
            f[0] += sx * s[0] + sy * s[5] + sz * s[4];
            f[1] += sx * s[5] + sy * s[1] + sz * s[3];
            f[2] += sx * s[4] + sy * s[3] + sz * s[2];
            if (c == 0) {
#pragma unroll
                for (int I = 0; I < 6; ++I) acc[I] += (double)s[I];
                double gq[3];
                angle_contractions(a.dC, g, e, e, gq);
#pragma unroll
                for (int q = 0; q < 3; ++q) a.G[(int64_t)q * a.n3 + n] = 0.5 * gq[q];
            }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            a.ub[(int64_t)j * a.n3 + n] = f[j];
            a.wb[(int64_t)j * a.n3 + n] = 0.f;
        }
    }
    block_sum_to<6>(a.partials, acc);
}

struct AdjStepArgs {
    const int16_t* spins;
    const float* Ctab;
    const float* dC;         // Q x 3 x kTab
    const float* ub_in;
    float* ub_out;
    const float* wb_in;      // read at neighbour nodes: ping-pong like ub
    float* wb_out;
    const float* u_t;        // forward displacement of step t
    const double* E_t;       // forward macroscopic strain of step t (6)
    const double* adj;       // b
    double* G;               // 3 planes
    double* partials;
    const RepDev* reps;
    float alpha, beta;
};

// One adjoint step, tiled as the forward step: a block owns a 32 x 8 x tile_z node tile;
// the nodal field a = alpha (w~) and the forward displacement u_t pass through two-slot LDS
// rings of node layers (one-node halo), the adjoint stresses tau through a ring of voxel
// layers.  Each voxel's tau is formed once per tile; the voxels the block owns also add
// their angle contractions to G and their tau to the block's partial sums.
__global__ __launch_bounds__(256) void k_adj_step(AdjStepArgs a)
{
    constexpr int NX = kTileX + 2, NY = kTileY + 2, VX = kTileX + 1, VY = kTileY + 1;
    __shared__ float sa[2][3][NY][NX];
    __shared__ float sf[2][3][NY][NX];
    __shared__ float ss[2][6][VY][VX];

    const RepDev R = a.reps[0];
    const int K = R.K;
    const int64_t n3 = R.n3;
    const int ntx = (K + kTileX - 1) / kTileX, nty = (K + kTileY - 1) / kTileY, tz = R.tile_z;
    const int lb = xcd_block((int)blockIdx.x, (int)gridDim.x);
    int b = lb;
    const int bx = b % ntx;
    b /= ntx;
    const int by = b % nty, bz = b / nty;
    const int x0 = bx * kTileX, y0 = by * kTileY, z0 = bz * tz;
    const int z1 = (z0 + tz < K) ? z0 + tz : K;
    float b3[6], E[6];
    const double inv_n3 = 1.0 / (double)n3;
#pragma unroll
    for (int I = 0; I < 6; ++I) {
        b3[I] = (float)(a.adj[kB + I] * inv_n3);
        E[I] = (float)a.E_t[I];
    }
    const float alpha = a.alpha, beta = a.beta;
    const int t = threadIdx.x, lx = t % kTileX, ly = t / kTileX;
    const int nx = x0 + lx, ny = y0 + ly;
    const bool own = nx < K && ny < K;
    double acc[6] = {0, 0, 0, 0, 0, 0};

    auto load_nodes = [&](int slot, int z) {
        const int64_t zoff = (int64_t)K * K * wrap_tile(z, K);
        for (int i = t; i < NX * NY; i += 256) {
            const int ix = i % NX, iy = i / NX;
            const int64_t n = wrap_tile(x0 - 1 + ix, K) + (int64_t)K * wrap_tile(y0 - 1 + iy, K) + zoff;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                sa[slot][j][iy][ix] = alpha * (a.wb_in[j * n3 + n] + a.ub_in[j * n3 + n]);
                sf[slot][j][iy][ix] = a.u_t[j * n3 + n];
            }
        }
    };
    // centre-point gradient of a node field held in two ring slots
    auto gradient = [&](float (*f)[3][NY][NX], int lo, int hi, int ix, int iy, float g[3][3]) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float c0 = f[lo][j][iy][ix], c1 = f[lo][j][iy][ix + 1];
            const float c2 = f[lo][j][iy + 1][ix], c3 = f[lo][j][iy + 1][ix + 1];
            const float c4 = f[hi][j][iy][ix], c5 = f[hi][j][iy][ix + 1];
            const float c6 = f[hi][j][iy + 1][ix], c7 = f[hi][j][iy + 1][ix + 1];
            g[j][0] = 0.25f * ((c1 - c0) + (c3 - c2) + (c5 - c4) + (c7 - c6));
            g[j][1] = 0.25f * ((c2 + c3) - (c0 + c1) + (c6 + c7) - (c4 + c5));
            g[j][2] = 0.25f * ((c4 + c5 + c6 + c7) - (c0 + c1 + c2 + c3));
        }
    };
    auto voxel_layer = [&](int vs, int lo, int hi, int z, bool owned_layer) {
        const int64_t zoff = (int64_t)K * K * wrap_tile(z, K);
        for (int i = t; i < VX * VY; i += 256) {
            const int ix = i % VX, iy = i / VX;
            float g[3][3];
            gradient(sa, lo, hi, ix, iy, g);
            float eta[6], tau[6];
            eta[0] = b3[0] + g[0][0];
            eta[1] = b3[1] + g[1][1];
            eta[2] = b3[2] + g[2][2];
            eta[3] = b3[3] + g[1][2] + g[2][1];
            eta[4] = b3[4] + g[0][2] + g[2][0];
            eta[5] = b3[5] + g[0][1] + g[1][0];
            const int gx = x0 - 1 + ix, gy = y0 - 1 + iy;
            const int64_t v = wrap_tile(gx, K) + (int64_t)K * wrap_tile(gy, K) + zoff;
            const int q = a.spins[v];
            symv21(a.Ctab + (int64_t)q * kTab, eta, tau);
#pragma unroll
            for (int I = 0; I < 6; ++I) ss[vs][I][iy][ix] = tau[I];
            if (owned_layer && ix >= 1 && iy >= 1 && gx < K && gy < K) {
#pragma unroll
                for (int I = 0; I < 6; ++I) acc[I] += (double)tau[I];
                gradient(sf, lo, hi, ix, iy, g);
                float eps[6];
                eps[0] = E[0] + g[0][0];
                eps[1] = E[1] + g[1][1];
                eps[2] = E[2] + g[2][2];
                eps[3] = E[3] + g[1][2] + g[2][1];
                eps[4] = E[4] + g[0][2] + g[2][0];
                eps[5] = E[5] + g[0][1] + g[1][0];
                double gq[3];
                angle_contractions(a.dC, q, eta, eps, gq);
#pragma unroll
                for (int qa = 0; qa < 3; ++qa) a.G[(int64_t)qa * n3 + v] -= gq[qa];
            }
        }
    };

    load_nodes(0, z0 - 1);
    load_nodes(1, z0);
    __syncthreads();
    voxel_layer(0, 0, 1, z0 - 1, false);
    int nlo = 1, vprev = 0;
    for (int z = z0; z < z1; ++z) {
        const int nhi = 1 - nlo, vcur = 1 - vprev;
        __syncthreads();
        load_nodes(nhi, z + 1);
        __syncthreads();
        voxel_layer(vcur, nlo, nhi, z, true);
        __syncthreads();
        if (own) {
            float f[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int ca = c & 1, cb = (c >> 1) & 1, cc = c >> 2;
                const int vx = lx + 1 - ca, vy = ly + 1 - cb, vsl = cc ? vprev : vcur;
                const float s0 = ss[vsl][0][vy][vx], s1 = ss[vsl][1][vy][vx], s2 = ss[vsl][2][vy][vx];
                const float s3 = ss[vsl][3][vy][vx], s4 = ss[vsl][4][vy][vx], s5 = ss[vsl][5][vy][vx];
                const float sx = ca ? 0.25f : -0.25f, sy = cb ? 0.25f : -0.25f, sz = cc ? 0.25f : -0.25f;
                f[0] += sx * s0 + sy * s5 + sz * s4;
                f[1] += sx * s5 + sy * s1 + sz * s3;
                f[2] += sx * s4 + sy * s3 + sz * s2;
            }
            const int64_t n = nx + (int64_t)K * (ny + (int64_t)K * z);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int64_t idx = (int64_t)j * n3 + n;
                const float u_in = a.ub_in[idx];
                a.ub_out[idx] = u_in - f[j];
                a.wb_out[idx] = beta * (a.wb_in[idx] + u_in);
            }
        }
        nlo = nhi;
        vprev = vcur;
    }
    block_sum_to<6>(a.partials, acc, lb);
}

// Folds the per-block sums (fixed order).  mode 0 (start): E^ = sum sigma, wE^ = 0,
// Sigma^ = 0.  mode 1 (after a step): E^ -= sum tau, wE^ = beta wE~, Sigma^ += b.  Both then
// prepare the next step: wE~ = wE^ + E^, b = alphaE wE~.
__global__ __launch_bounds__(256) void k_adj_E(double* adj, const double* partials, int nblocks, int mode,
                                               double betaE, double alphaE)
{
    const int t = threadIdx.x;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int bk = t; bk < nblocks; bk += 256)
#pragma unroll
        for (int I = 0; I < 6; ++I) s[I] += partials[(int64_t)bk * 8 + I];
    const double tot = block_total<6>(s);
    if (t < 6) {
        if (mode == 0) {
            adj[kEb + t] = tot;
            adj[kWEb + t] = 0.0;
            adj[kSigb + t] = 0.0;
        } else {
            adj[kEb + t] -= tot;
            adj[kWEb + t] = betaE * adj[kWEt + t];
            adj[kSigb + t] += adj[kB + t];
        }
        const double wt = adj[kWEb + t] + adj[kEb + t];
        adj[kWEt + t] = wt;
        adj[kB + t] = alphaE * wt;
    }
}

struct AdjGradArgs {
    const int16_t* spins;
    const float* Stab;
    const float* dS;    // Q x 3 x kTab
    const double* G;
    const double* adj;  // E^_0 at kEb
    double Sigma[6];
    unsigned long long* grad;   // Q x 3 fixed point
    double* partials;
    int64_t n3;
};

// Per voxel: the three stiffness-angle sums G_v plus the start-strain term
// (1/K^3) E^_0 . dS Sigma into its grain (fixed-point atomics); partial sums of S E^_0.
__global__ __launch_bounds__(256) void k_adj_grad(AdjGradArgs a)
{
    double Eb[6];
    float Ebf[6];
    const double inv_n3 = 1.0 / (double)a.n3;
#pragma unroll
    for (int I = 0; I < 6; ++I) {
        Eb[I] = a.adj[kEb + I];
        Ebf[I] = (float)Eb[I];
    }
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < a.n3; v += (int64_t)gridDim.x * blockDim.x) {
        const int g = a.spins[v];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float* ds = a.dS + ((int64_t)g * 3 + q) * kTab;
            double val = a.G[(int64_t)q * a.n3 + v];
            int k = 0;
#pragma unroll
            for (int I = 0; I < 6; ++I)
#pragma unroll
                for (int J = I; J < 6; ++J) {
                    // start term: E^_0 . (dS Sigma) with the symmetric dS
                    const double sym = (I == J) ? Eb[I] * a.Sigma[I] : Eb[I] * a.Sigma[J] + Eb[J] * a.Sigma[I];
                    val += inv_n3 * (double)ds[k] * sym;
                    ++k;
                }
            const long long fx = llrint(val * kFixScale);
            atomicAdd(&a.grad[(int64_t)g * 3 + q], (unsigned long long)fx);
        }
        float se[6];
        symv21(a.Stab + (int64_t)g * kTab, Ebf, se);
#pragma unroll
        for (int I = 0; I < 6; ++I) acc[I] += (double)se[I];
    }
    block_sum_to<6>(a.partials, acc);
}

}  // namespace hmc

using namespace hmc;

namespace {

hmc_status afail(hmc_ctx c, hmc_status s, const char* m)
{
    c->err = m;
    return s;
}

hmc_status adev(hmc_ctx c, hipError_t e, const char* where)
{
    c->err = std::string(where) + ": " + hipGetErrorString(e);
    return HMC_EDEVICE;
}

#define ATRY(expr, where)                              \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return adev(c, e_, where); \
    } while (0)

int adj_blocks(int64_t n3)
{
    int64_t b = (n3 + 255) / 256;
    if (b > kMaxChunkBlocks) b = kMaxChunkBlocks;
    return (int)(b < 1 ? 1 : b);
}

// checkpoint j: u (3 planes), w (3 planes), then E, wE (12 doubles)
hmc_status save_ckpt(hmc_ctx c, char* base, const AdjLayout& L, int j)
{
    const size_t n3 = (size_t)c->reps[0].n3;
    char* ck = base + L.ckpt + (size_t)j * L.ck_bytes;
    ATRY(hipMemcpyAsync(ck, c->d.u[c->cur_u], 3 * n3 * sizeof(float), hipMemcpyDeviceToDevice, c->stream), "ckpt");
    ATRY(hipMemcpyAsync(ck + 3 * n3 * sizeof(float), c->d.w, 3 * n3 * sizeof(float), hipMemcpyDeviceToDevice,
                        c->stream),
         "ckpt");
    ATRY(hipMemcpyAsync(ck + al256(6 * n3 * sizeof(float)), c->d.state + kE, 12 * sizeof(double),
                        hipMemcpyDeviceToDevice, c->stream),
         "ckpt");
    return HMC_OK;
}

// restores checkpoint j with u into `u_dst`
hmc_status load_ckpt(hmc_ctx c, char* base, const AdjLayout& L, int j, float* u_dst)
{
    const size_t n3 = (size_t)c->reps[0].n3;
    char* ck = base + L.ckpt + (size_t)j * L.ck_bytes;
    ATRY(hipMemcpyAsync(u_dst, ck, 3 * n3 * sizeof(float), hipMemcpyDeviceToDevice, c->stream), "restore");
    ATRY(hipMemcpyAsync(c->d.w, ck + 3 * n3 * sizeof(float), 3 * n3 * sizeof(float), hipMemcpyDeviceToDevice,
                        c->stream),
         "restore");
    ATRY(hipMemcpyAsync(c->d.state + kE, ck + al256(6 * n3 * sizeof(float)), 12 * sizeof(double),
                        hipMemcpyDeviceToDevice, c->stream),
         "restore");
    return HMC_OK;
}

hmc_status check_adj(hmc_ctx c, int n_steps, int k, void* ws, size_t bytes, AdjLayout* L)
{
    if (c->is_batch || c->n_rep != 1) return afail(c, HMC_ESTATE, "the adjoint acts on a single lattice");
    if (!c->elastic_buffers) return afail(c, HMC_ESTATE, "elastic term disabled (lambda_el == 0)");
    if (n_steps < 1 || k < 1) return afail(c, HMC_EINVAL, "need n_steps >= 1 and ckpt_every >= 1");
    if (!ws || ((uintptr_t)ws % 256) != 0) return afail(c, HMC_EINVAL, "adjoint workspace must be 256-byte aligned");
    *L = adj_layout(c, n_steps, k);
    if (bytes < L->total) return afail(c, HMC_ESHAPE, "adjoint workspace too small");
    return HMC_OK;
}

}  // namespace

namespace hmc {
hipError_t launch_global_step_ptrs(hmc_ctx_s* c, const float* uin, float* uout, double* E_record);
}

extern "C" {

size_t hmc_adjoint_workspace_bytes(hmc_ctx c, int32_t n_steps, int32_t ckpt_every)
{
    if (!c || c->n_rep != 1 || n_steps < 1 || ckpt_every < 1) return 0;
    return adj_layout(c, n_steps, ckpt_every).total;
}

hmc_status hmc_elastic_forward(hmc_ctx c, int32_t n_steps, int32_t ckpt_every, void* ws, size_t bytes, double* U)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    AdjLayout L;
    hmc_status st = check_adj(c, n_steps, ckpt_every, ws, bytes, &L);
    if (st != HMC_OK) return st;
    if (!U) return afail(c, HMC_EINVAL, "null output");
    if (!c->have_orient || !c->have_spins || !c->have_load)
        return afail(c, HMC_ESTATE, "forward needs orientations, spins and a load");
    char* base = (char*)ws;
    // cold start exactly as hmc_stress_refresh
    ATRY(launch_fill_f32(c->d.u[0], 0.f, 3 * c->total_sites, c->stream), "forward");
    ATRY(launch_fill_f32(c->d.w, 0.f, 3 * c->total_sites, c->stream), "forward");
    c->cur_u = 0;
    ATRY(launch_reuss(c), "forward");
    for (int t = 0; t < n_steps; ++t) {
        if (t % ckpt_every == 0) {
            st = save_ckpt(c, base, L, t / ckpt_every);
            if (st != HMC_OK) return st;
        }
        ATRY(launch_global_steps(c, 1), "forward");
    }
    st = save_ckpt(c, base, L, L.n_ck - 1);   // final state
    if (st != HMC_OK) return st;
    ATRY(launch_global_final(c, true), "forward");
    double u = 0;
    ATRY(hipMemcpyAsync(&u, c->d.state + kU, sizeof u, hipMemcpyDeviceToHost, c->stream), "forward");
    ATRY(hipStreamSynchronize(c->stream), "forward");
    c->host_refresh_steps += n_steps;
    c->have_state = c->have_stress = true;
    c->adj_steps = n_steps;
    c->adj_every = ckpt_every;
    *U = u;
    return HMC_OK;
}

hmc_status hmc_elastic_backward(hmc_ctx c, void* ws, size_t bytes, double dU, double* grad_euler,
                                double grad_sigma_MPa[6])
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (c->adj_steps < 1) return afail(c, HMC_ESTATE, "no forward pass recorded");
    AdjLayout L;
    const int n = c->adj_steps, k = c->adj_every;
    hmc_status st = check_adj(c, n, k, ws, bytes, &L);
    if (st != HMC_OK) return st;
    if (!grad_euler || !grad_sigma_MPa) return afail(c, HMC_EINVAL, "null output");
    const RepDev& R = c->reps[0];
    const int64_t n3 = R.n3;
    const int Q = R.Q;
    char* base = (char*)ws;
    float* seg_u = (float*)(base + L.seg_u);
    double* seg_E = (double*)(base + L.seg_E);
    float* ub[2] = {(float*)(base + L.ub0), (float*)(base + L.ub1)};
    float* wb[2] = {(float*)(base + L.wb0), (float*)(base + L.wb1)};
    double* G = (double*)(base + L.G);
    float* dC = (float*)(base + L.dC);
    float* dS = (float*)(base + L.dS);
    double* adj = (double*)(base + L.adj);
    unsigned long long* grad = (unsigned long long*)(base + L.grad);
    const int nb = adj_blocks(n3);

    // per-grain derivative tables
    {
        std::vector<float> hC((size_t)Q * 3 * kTab, 0.f), hS((size_t)Q * 3 * kTab, 0.f);
        std::vector<double> dCd((size_t)Q * 108), dSd((size_t)Q * 108);
        if (hmc_grain_table_derivatives(c->euler.data(), Q, c->p.C11, c->p.C12, c->p.C44, dCd.data(), dSd.data()) !=
            HMC_OK)
            return afail(c, HMC_ENUMERIC, "orientation derivatives");
        for (int g = 0; g < Q; ++g)
            for (int q = 0; q < 3; ++q)
                for (int i = 0; i < 6; ++i)
                    for (int j = i; j < 6; ++j) {
                        hC[((size_t)g * 3 + q) * kTab + sym_index(i, j)] = (float)dCd[(size_t)g * 108 + q * 36 + 6 * i + j];
                        hS[((size_t)g * 3 + q) * kTab + sym_index(i, j)] = (float)dSd[(size_t)g * 108 + q * 36 + 6 * i + j];
                    }
        ATRY(hipMemcpyAsync(dC, hC.data(), hC.size() * sizeof(float), hipMemcpyHostToDevice, c->stream), "backward");
        ATRY(hipMemcpyAsync(dS, hS.data(), hS.size() * sizeof(float), hipMemcpyHostToDevice, c->stream), "backward");
        ATRY(hipMemsetAsync(grad, 0, (size_t)Q * 3 * sizeof(unsigned long long), c->stream), "backward");
        ATRY(hipStreamSynchronize(c->stream), "backward");
    }

    // final state -> initial adjoint
    st = load_ckpt(c, base, L, L.n_ck - 1, c->d.u[0]);
    if (st != HMC_OK) return st;
    c->cur_u = 0;
    {
        AdjInitArgs a{c->d.spins, c->d.Ctab, dC, c->d.u[0], ub[0], wb[0], G, c->d.partials, c->d.state, R.K, n3};
        hipLaunchKernelGGL(k_adj_init, dim3(nb), dim3(256), 0, c->stream, a);
        hipLaunchKernelGGL(k_adj_E, dim3(1), dim3(256), 0, c->stream, adj, c->d.partials, nb, 0, (double)R.glob_beta,
                           R.glob_alphaE);
        ATRY(hipGetLastError(), "backward: start");
    }
    int cur_b = 0;
    const int n_seg = (n + k - 1) / k;
    for (int j = n_seg - 1; j >= 0; --j) {
        const int t0 = j * k, t1 = (t0 + k < n) ? t0 + k : n;
        // recompute the segment's forward states u_t, E_t for t in [t0, t1)
        st = load_ckpt(c, base, L, j, seg_u);
        if (st != HMC_OK) return st;
        for (int t = t0; t < t1; ++t) {
            float* ut = seg_u + (size_t)(t - t0) * 3 * n3;
            double* Et = seg_E + (size_t)(t - t0) * 8;
            if (t + 1 < t1)
                ATRY(launch_global_step_ptrs(c, ut, ut + 3 * n3, Et), "backward: recompute");   // records E_t
            else
                ATRY(hipMemcpyAsync(Et, c->d.state + kE, 6 * sizeof(double), hipMemcpyDeviceToDevice, c->stream),
                     "backward: recompute");
        }
        // adjoint steps t1-1 .. t0
        for (int t = t1 - 1; t >= t0; --t) {
            AdjStepArgs a;
            a.spins = c->d.spins;
            a.Ctab = c->d.Ctab;
            a.dC = dC;
            a.ub_in = ub[cur_b];
            a.ub_out = ub[1 - cur_b];
            a.wb_in = wb[cur_b];
            a.wb_out = wb[1 - cur_b];
            a.u_t = seg_u + (size_t)(t - t0) * 3 * n3;
            a.E_t = seg_E + (size_t)(t - t0) * 8;
            a.adj = adj;
            a.G = G;
            a.partials = c->d.partials;
            a.reps = c->d.reps;
            a.alpha = R.glob_alpha;
            a.beta = R.glob_beta;
            const int tok = prof_begin(c, kProfRefreshStep);
            hipLaunchKernelGGL(k_adj_step, dim3(c->tile_blocks), dim3(256), 0, c->stream, a);
            prof_end(c, tok);
            hipLaunchKernelGGL(k_adj_E, dim3(1), dim3(256), 0, c->stream, adj, c->d.partials, c->tile_blocks, 1,
                               (double)R.glob_beta, R.glob_alphaE);
            ATRY(hipGetLastError(), "backward: step");
            cur_b = 1 - cur_b;
        }
    }
    // contractions and the start-strain terms
    {
        AdjGradArgs a;
        a.spins = c->d.spins;
        a.Stab = c->d.Stab;
        a.dS = dS;
        a.G = G;
        a.adj = adj;
        for (int I = 0; I < 6; ++I) a.Sigma[I] = R.Sigma[I];
        a.grad = grad;
        a.partials = c->d.partials;
        a.n3 = n3;
        hipLaunchKernelGGL(k_adj_grad, dim3(nb), dim3(256), 0, c->stream, a);
        ATRY(hipGetLastError(), "backward: gradient");
    }
    std::vector<unsigned long long> g((size_t)Q * 3);
    std::vector<double> parts((size_t)nb * 8);
    double ad[kAdjDoubles];
    ATRY(hipMemcpyAsync(g.data(), grad, g.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream),
         "backward");
    ATRY(hipMemcpyAsync(parts.data(), c->d.partials, parts.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream),
         "backward");
    ATRY(hipMemcpyAsync(ad, adj, sizeof ad, hipMemcpyDeviceToHost, c->stream), "backward");
    ATRY(hipStreamSynchronize(c->stream), "backward");
    for (size_t i = 0; i < g.size(); ++i) grad_euler[i] = dU * (double)(long long)g[i] / kFixScale;
    for (int I = 0; I < 6; ++I) {
        double s = 0.0;   // mean(S) E^_0, folded in block order
        for (int b = 0; b < nb; ++b) s += parts[(size_t)b * 8 + I];
        // dU/dSigma in GPa^-1 * GPa*voxel; per MPa: x 1e-3
        grad_sigma_MPa[I] = dU * (ad[kSigb + I] + s / (double)n3) * 1e-3;
    }
    // leave the context at the final forward state
    st = load_ckpt(c, base, L, L.n_ck - 1, c->d.u[0]);
    if (st != HMC_OK) return st;
    c->cur_u = 0;
    ATRY(launch_global_final(c, true), "backward: restore");
    ATRY(hipStreamSynchronize(c->stream), "backward: restore");
    return HMC_OK;
}

}  // extern "C"
