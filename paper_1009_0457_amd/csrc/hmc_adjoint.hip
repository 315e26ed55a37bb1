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
// Doubles per copy of the part of the adjoint state the adjoint steps advance (the slots
// kEb .. kWEt below), kept per step like the forward sequence's (E, wE); the tau sums between
// steps use the forward's fixed-point accumulators.
constexpr int kAdjSeq = 32;

struct AdjLayout {
    size_t ckpt, seg_u[2], seg_E[2], ub0, ub1, wb0, wb1, G, dC, dS, adj, asums, aseq, grad, total;
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
    // two segment buffers: one segment's adjoint steps read one while the next segment is
    // recomputed into the other
    for (int b = 0; b < 2; ++b) {
        L.seg_u[b] = take((size_t)(k + 1) * 3 * n3 * sizeof(float));
        L.seg_E[b] = take((size_t)(k + 1) * 8 * sizeof(double));
    }
    L.ub0 = take(3 * n3 * sizeof(float));
    L.ub1 = take(3 * n3 * sizeof(float));
    L.wb0 = take(3 * n3 * sizeof(float));
    L.wb1 = take(3 * n3 * sizeof(float));
    L.G = take(3 * n3 * sizeof(double));
    L.dC = take(Q * 3 * kTab * sizeof(float));
    L.dS = take(Q * 3 * kTab * sizeof(float));
    L.adj = take(64 * sizeof(double));
    L.asums = take(3 * kSumSlots * sizeof(unsigned long long));
    L.aseq = take(2 * kAdjSeq * sizeof(double));
    L.grad = take(Q * 3 * sizeof(unsigned long long));
    L.total = o;
    return L;
}

// Slots of the adjoint's small state block.
enum AdjSlot { kEb = 0, kWEb = 6, kB = 12, kSigb = 18, kWEt = 24, kE0 = 30, kAdjDoubles = 64 };

// Component I of the adjoint state after one more adjoint step whose tau sums are in `sums`
// (null: unchanged): E^ -= sum tau, wE^ = beta wE~, Sigma^ += b, wE~ = wE^ + E^, b = alphaE wE~.
__device__ __forceinline__ void adj_advance(const double* in, const unsigned long long* sums, int I, double betaE,
                                            double alphaE, double out[5])
{
    double Eb = in[kEb + I], wEb = in[kWEb + I], b = in[kB + I], Sb = in[kSigb + I], wt = in[kWEt + I];
    if (sums) {
        long long tot = 0;
#pragma unroll
        for (int c = 0; c < kSumCopies; ++c) tot += (long long)sums[c * 8 + I];
        Eb -= (double)tot / kSumScale;
        wEb = betaE * wt;
        Sb += b;
        wt = wEb + Eb;
        b = alphaE * wt;
    }
    out[0] = Eb;
    out[1] = wEb;
    out[2] = b;
    out[3] = Sb;
    out[4] = wt;
}

__device__ __forceinline__ void adj_store(double* dst, int I, const double v[5])
{
    dst[kEb + I] = v[0];
    dst[kWEb + I] = v[1];
    dst[kB + I] = v[2];
    dst[kSigb + I] = v[3];
    dst[kWEt + I] = v[4];
}

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
    const double* st_in;     // adjoint state the previous step started from (or the initial one)
    double* st_out;          // this step's (written by block 0)
    const unsigned long long* sums_in;   // the previous step's tau sums (null: first step)
    unsigned long long* sums_out;        // this step's
    unsigned long long* sums_clear;      // the next step's, cleared by block 0
    double* G;               // 3 planes
    const RepDev* reps;
    float alpha, beta;
    double betaE, alphaE;
    int order;               // logical block order (hmc_set_block_order)
};

// tau = C_q eta and, where `owned`, gq_k = eta . (dC_{q,k} eps) for the three angles k,
// with the tables of a wavefront's first two grains from scalar loads (as symv21_grains);
// wavefronts with more grains gather per lane.
__device__ __forceinline__ void adjoint_voxel(const float* Ctab, const float* dC, int q, bool owned,
                                              const float eta[6], const float eps[6], float tau[6], double gq[3])
{
    auto with_rows = [&](int g) {   // g is the same in every active lane
        float c[21];
        uniform_row(Ctab, g, c);
        symv21(c, eta, tau);
        if (owned) angle_contractions(dC, g, eta, eps, gq);
    };
    const int q0 = __builtin_amdgcn_readfirstlane(q);
    const uint64_t other = __builtin_amdgcn_ballot_w64(q != q0);
    if (other == 0) {
        with_rows(q0);
    } else {
        const int q1 = __builtin_amdgcn_readlane(q, (int)__builtin_ctzll(other));
        if (__builtin_amdgcn_ballot_w64(q != q0 && q != q1) == 0) {
            with_rows(q0);
            if (q == q1) with_rows(q1);
        } else {
            symv21(Ctab + (int64_t)q * kTab, eta, tau);
            if (owned) angle_contractions(dC, q, eta, eps, gq);
        }
    }
}

// One adjoint step, tiled as the forward step (32 x 8 x tile_z nodes per block, layer-pair
// sums of the nodal fields and of the voxel stresses in LDS, previous layer in registers):
// the nodal field a = alpha (w^ + u^) and the forward displacement u_t give each voxel its
// adjoint strain eta and forward strain eps; tau = C eta is formed once per tile, and the
// voxels the block owns also add their angle contractions to G and tau to the block's sums.
__global__ __launch_bounds__(256, 3) void k_adj_step(AdjStepArgs a)
{
    constexpr int NX = kTileX + 2, NY = kTileY + 2, VX = kTileX + 1, VY = kTileY + 1;
    constexpr int NP = (NX * NY + 255) / 256, VP = (kStepVox + 255) / 256;
    __shared__ float4 sAa[NY][NX], sUa[NY][NX];
    __shared__ float2 sAb[NY][NX], sUb[NY][NX];
    __shared__ float4 sPa[VY][VX], sPb[VY][VX];

    const RepDev R = a.reps[0];
    const int K = R.K;
    const int64_t n3 = R.n3;
    const int ntx = (K + kTileX - 1) / kTileX, nty = (K + kTileY - 1) / kTileY, tz = R.tile_z;
    const int lb = logical_block((int)blockIdx.x, (int)gridDim.x, a.order);
    int b = lb;
    const int bx = b % ntx;
    b /= ntx;
    const int by = b % nty, bz = b / nty;
    const int x0 = bx * kTileX, y0 = by * kTileY, z0 = bz * tz;
    const int z1 = (z0 + tz < K) ? z0 + tz : K;
    // this step's adjoint state from the previous one and its tau sums (read after the
    // prologue's first barrier); block 0 records it and clears the sums of the step after
    __shared__ double sb[6];
    if (threadIdx.x < 6) {
        double v[5];
        adj_advance(a.st_in, a.sums_in, threadIdx.x, a.betaE, a.alphaE, v);
        sb[threadIdx.x] = v[2];
        if (lb == 0) adj_store(a.st_out, threadIdx.x, v);
    }
    if (lb == 0 && threadIdx.x < kSumSlots) a.sums_clear[threadIdx.x] = 0ull;
    float b3[6], E[6];
    const double inv_n3 = 1.0 / (double)n3;
#pragma unroll
    for (int I = 0; I < 6; ++I) E[I] = (float)a.E_t[I];
    const float alpha = a.alpha, beta = a.beta;
    const int t = threadIdx.x, lx = t % kTileX, ly = t / kTileX;
    const int nx = x0 + lx, ny = y0 + ly;
    const bool own = nx < K && ny < K;
    double acc[6] = {0, 0, 0, 0, 0, 0};

    int node_xy[NP], vox_xy[VP];
    bool vox_own[VP];   // only interior positions (k = 0) can be owned
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int i = t + 256 * k, ix = i % NX, iy = i / NX;
        node_xy[k] = wrap_tile(x0 - 1 + ix, K) + K * wrap_tile(y0 - 1 + iy, K);
    }
#pragma unroll
    for (int k = 0; k < VP; ++k) {
        int ix, iy;
        step_voxel_pos(t + 256 * k, ix, iy);
        vox_xy[k] = wrap_tile(x0 - 1 + ix, K) + K * wrap_tile(y0 - 1 + iy, K);
        vox_own[k] = t + 256 * k < kStepVox && ix >= 1 && iy >= 1 && x0 - 1 + ix < K && y0 - 1 + iy < K;
    }
    // the fetched node layer (w^, u^ for a, and u_t) at the thread's positions; the previous
    // layer's a and u_t stay in registers for the pair sums
    float fw[NP][3], fb[NP][3], fu[NP][3], prevA[NP][3], prevU[NP][3];
    int sp[VP];
    auto fetch_nodes = [&](int z) {
        const int64_t zoff = (int64_t)K * K * wrap_tile(z, K);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (t + 256 * k < NX * NY) {
                const int64_t n = node_xy[k] + zoff;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    fw[k][j] = a.wb_in[j * n3 + n];
                    fb[k][j] = a.ub_in[j * n3 + n];
                    fu[k][j] = a.u_t[j * n3 + n];
                }
            }
        }
    };
    auto fetch_spins = [&](int z) {
        const int64_t zoff = (int64_t)K * K * wrap_tile(z, K);
#pragma unroll
        for (int k = 0; k < VP; ++k) {
            sp[k] = 0;
            if (t + 256 * k < kStepVox) sp[k] = a.spins[vox_xy[k] + zoff];
        }
    };
    // the fetched layer is z+1, prev* hold layer z: write the pair's entries
    auto store_pair = [&]() {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int i = t + 256 * k;
            if (i < NX * NY) {
                const int ix = i % NX, iy = i / NX;
                float an[3];
#pragma unroll
                for (int j = 0; j < 3; ++j) an[j] = alpha * (fw[k][j] + fb[k][j]);
                pair_node_entry(an, prevA[k], sAa[iy][ix], sAb[iy][ix]);
                pair_node_entry(fu[k], prevU[k], sUa[iy][ix], sUb[iy][ix]);
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    prevA[k][j] = an[j];
                    prevU[k][j] = fu[k][j];
                }
            }
        }
    };
    auto take_prev = [&]() {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                prevA[k][j] = alpha * (fw[k][j] + fb[k][j]);
                prevU[k][j] = fu[k][j];
            }
    };
    // adjoint stress of voxel position k (and, if owned, its angle contractions)
    auto voxel_adj = [&](int k, int q, bool owned, float tau[6], double gq[3]) {
        int ix, iy;
        step_voxel_pos(t + 256 * k, ix, iy);
        float eta[6], eps[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        pair_strain<NX>(sAa, sAb, ix, iy, b3, eta);
        if (owned) pair_strain<NX>(sUa, sUb, ix, iy, E, eps);
        adjoint_voxel(a.Ctab, a.dC, q, owned, eta, eps, tau, gq);
    };

    // prologue: node layers z0-1, z0 -> voxel layer z0-1 (kept in registers)
    fetch_nodes(z0 - 1);
    take_prev();
    fetch_nodes(z0);
    fetch_spins(z0 - 1);
    store_pair();
    __syncthreads();
#pragma unroll
    for (int I = 0; I < 6; ++I) b3[I] = (float)(sb[I] * inv_n3);
    float tprev[VP][6];
#pragma unroll
    for (int k = 0; k < VP; ++k)
        if (t + 256 * k < kStepVox) {
            double unused[3];
            voxel_adj(k, sp[k], false, tprev[k], unused);
        }
    fetch_spins(z0);
    __syncthreads();

    for (int z = z0; z < z1; ++z) {
        fetch_nodes(z + 1);
        store_pair();                            // pair (z, z+1)
        int sp_cur[VP];
#pragma unroll
        for (int k = 0; k < VP; ++k) {
            sp_cur[k] = sp[k];
            asm volatile("" ::"v"(sp_cur[k]));   // take them before the loads below are issued
        }
        // requested in the order needed: this layer's G of the owned voxels, the own nodes'
        // w^ and u^, then the next layer's grains
        const int64_t zoff = (int64_t)K * K * z;
        double Gv[3] = {0.0, 0.0, 0.0};
        if (vox_own[0]) {
#pragma unroll
            for (int qa = 0; qa < 3; ++qa) Gv[qa] = a.G[(int64_t)qa * n3 + vox_xy[0] + zoff];
        }
        float wn_in[3] = {0.f, 0.f, 0.f}, un_in[3] = {0.f, 0.f, 0.f};
        const int64_t n = nx + (int64_t)K * ny + zoff;
        if (own) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                wn_in[j] = a.wb_in[(int64_t)j * n3 + n];
                un_in[j] = a.ub_in[(int64_t)j * n3 + n];
            }
        }
        if (z + 1 < z1) fetch_spins(z + 1);
        __syncthreads();                         // the node pairs are complete
#pragma unroll
        for (int k = 0; k < VP; ++k) {
            const int i = t + 256 * k;
            if (i >= kStepVox) continue;
            int ix, iy;
            step_voxel_pos(i, ix, iy);
            const bool owned = k == 0 && vox_own[0];   // the halo (k >= 1) is never owned
            float tau[6];
            double gq[3] = {0.0, 0.0, 0.0};
            voxel_adj(k, sp_cur[k], owned, tau, gq);
            pair_voxel_entry(tau, tprev[k], sPa[iy][ix], sPb[iy][ix]);
#pragma unroll
            for (int I = 0; I < 6; ++I) tprev[k][I] = tau[I];
            if (owned) {
#pragma unroll
                for (int I = 0; I < 6; ++I) acc[I] += (double)tau[I];
#pragma unroll
                for (int qa = 0; qa < 3; ++qa) a.G[(int64_t)qa * n3 + vox_xy[k] + zoff] = Gv[qa] - gq[qa];
            }
        }
        __syncthreads();                         // the voxel pair is complete
        if (own) {
            float F[3];
            pair_force<VX>(sPa, sPb, lx, ly, F);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int64_t idx = (int64_t)j * n3 + n;
                a.ub_out[idx] = un_in[j] - 0.25f * F[j];
                a.wb_out[idx] = beta * (wn_in[j] + un_in[j]);
            }
        }
    }
    const double tot = block_total<6>(acc);
    if (threadIdx.x < 6)
        atomicAdd(a.sums_out + (lb & (kSumCopies - 1)) * 8 + threadIdx.x, (unsigned long long)llrint(tot * kSumScale));
}

// After the last adjoint step: the adjoint state block.
__global__ void k_adj_seq_fold(double* adj, const double* st_last, const unsigned long long* sums_last, double betaE,
                               double alphaE)
{
    const int I = threadIdx.x;
    if (I >= 6) return;
    double v[5];
    adj_advance(st_last, sums_last, I, betaE, alphaE, v);
    adj_store(adj, I, v);
}

// Starts the adjoint state from the per-block sums of the final stresses (fixed order):
// E^ = sum sigma, wE^ = 0, Sigma^ = 0, then wE~ = wE^ + E^ and b = alphaE wE~ for the first
// adjoint step (later steps advance the state themselves, adj_advance).
__global__ __launch_bounds__(256) void k_adj_E(double* adj, const double* partials, int nblocks, double alphaE)
{
    const int t = threadIdx.x;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int bk = t; bk < nblocks; bk += 256)
#pragma unroll
        for (int I = 0; I < 6; ++I) s[I] += partials[(int64_t)bk * 8 + I];
    const double tot = block_total<6>(s);
    if (t < 6) {
        adj[kEb + t] = tot;
        adj[kWEb + t] = 0.0;
        adj[kSigb + t] = 0.0;
        adj[kWEt + t] = tot;
        adj[kB + t] = alphaE * tot;
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

// restores checkpoint j with u into `u_dst`, on stream s
hmc_status load_ckpt(hmc_ctx c, char* base, const AdjLayout& L, int j, float* u_dst, hipStream_t s)
{
    const size_t n3 = (size_t)c->reps[0].n3;
    char* ck = base + L.ckpt + (size_t)j * L.ck_bytes;
    ATRY(hipMemcpyAsync(u_dst, ck, 3 * n3 * sizeof(float), hipMemcpyDeviceToDevice, s), "restore");
    ATRY(hipMemcpyAsync(c->d.w, ck + 3 * n3 * sizeof(float), 3 * n3 * sizeof(float), hipMemcpyDeviceToDevice, s),
         "restore");
    ATRY(hipMemcpyAsync(c->d.state + kE, ck + al256(6 * n3 * sizeof(float)), 12 * sizeof(double),
                        hipMemcpyDeviceToDevice, s),
         "restore");
    return HMC_OK;
}

hmc_status check_adj(hmc_ctx c, int n_steps, int k, void* ws, size_t bytes, AdjLayout* L)
{
    if (c->is_batch || c->n_rep != 1) return afail(c, HMC_ESTATE, "the adjoint acts on a single lattice");
    if (c->p.material_points == 8) return afail(c, HMC_ESTATE, "the adjoint covers one material point per voxel");
    if (!c->elastic_buffers) return afail(c, HMC_ESTATE, "elastic term disabled (lambda_el == 0)");
    if (n_steps < 1 || k < 1) return afail(c, HMC_EINVAL, "need n_steps >= 1 and ckpt_every >= 1");
    if (!ws || ((uintptr_t)ws % 256) != 0) return afail(c, HMC_EINVAL, "adjoint workspace must be 256-byte aligned");
    *L = adj_layout(c, n_steps, k);
    if (bytes < L->total) return afail(c, HMC_ESHAPE, "adjoint workspace too small");
    return HMC_OK;
}

}  // namespace

namespace hmc {
}

extern "C" {

size_t hmc_adjoint_workspace_bytes(hmc_ctx c, int32_t n_steps, int32_t ckpt_every)
{
    if (!c || c->n_rep != 1 || n_steps < 1 || ckpt_every < 1) return 0;
    return adj_layout(c, n_steps, ckpt_every).total;
}

hmc_status hmc_elastic_forward(hmc_ctx c, int32_t n_steps, int32_t ckpt_every, void* ws, size_t bytes, double* U)
{
    TraceRange range("hmc adjoint forward");
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
    for (int t = 0; t < n_steps; t += ckpt_every) {
        st = save_ckpt(c, base, L, t / ckpt_every);
        if (st != HMC_OK) return st;
        ATRY(launch_global_steps(c, (t + ckpt_every < n_steps) ? ckpt_every : n_steps - t), "forward");
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
    return report_nonfinite(c);
}

hmc_status hmc_elastic_backward(hmc_ctx c, void* ws, size_t bytes, double dU, double* grad_euler,
                                double grad_sigma_MPa[6])
{
    if (!c) return HMC_EINVAL;
    TraceRange range("hmc adjoint backward");
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
    float* seg_u[2] = {(float*)(base + L.seg_u[0]), (float*)(base + L.seg_u[1])};
    double* seg_E[2] = {(double*)(base + L.seg_E[0]), (double*)(base + L.seg_E[1])};
    float* ub[2] = {(float*)(base + L.ub0), (float*)(base + L.ub1)};
    float* wb[2] = {(float*)(base + L.wb0), (float*)(base + L.wb1)};
    double* G = (double*)(base + L.G);
    float* dC = (float*)(base + L.dC);
    float* dS = (float*)(base + L.dS);
    double* adj = (double*)(base + L.adj);
    unsigned long long* asums = (unsigned long long*)(base + L.asums);
    double* aseq = (double*)(base + L.aseq);
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
    st = load_ckpt(c, base, L, L.n_ck - 1, c->d.u[0], c->stream);
    if (st != HMC_OK) return st;
    c->cur_u = 0;
    {
        AdjInitArgs a{c->d.spins, c->d.Ctab, dC, c->d.u[0], ub[0], wb[0], G, c->d.partials, c->d.state, R.K, n3};
        hipLaunchKernelGGL(k_adj_init, dim3(nb), dim3(256), 0, c->stream, a);
        hipLaunchKernelGGL(k_adj_E, dim3(1), dim3(256), 0, c->stream, adj, c->d.partials, nb, R.glob_alphaE);
        ATRY(hipGetLastError(), "backward: start");
    }
    int cur_b = 0, i_adj = 0;   // i_adj: adjoint steps taken
    // the first adjoint step adds into tau-sum buffer 0 (2 uint32 per 64-bit word)
    ATRY(launch_fill_u32((uint32_t*)asums, 0u, 2 * kSumSlots, c->stream), "backward: start");
    const int n_seg = (n + k - 1) / k;
    // Segment j's forward states are recomputed from its checkpoint into buffer j & 1.  With
    // the auxiliary stream the recomputation of segment j-1 runs while the context's stream
    // takes segment j's adjoint steps (both are latency-bound at this size); events order
    // them: ev[0..1] "buffer b free", ev[2..3] "buffer b recomputed", ev[4] start.  With
    // profiling on, everything stays on the context's stream.
    const bool overlap = !c->profiling;
    hipStream_t rs = c->stream;
    if (overlap) {
        if (!c->aux_stream) {
            ATRY(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking), "backward: stream");
            for (auto& e : c->aux_ev) ATRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "backward: events");
        }
        rs = c->aux_stream;
        // the recomputation overwrites the context's w and (E, wE), which the start above read
        ATRY(hipEventRecord(c->aux_ev[4], c->stream), "backward: events");
        ATRY(hipStreamWaitEvent(rs, c->aux_ev[4], 0), "backward: events");
        ATRY(hipEventRecord(c->aux_ev[0], c->stream), "backward: events");
        ATRY(hipEventRecord(c->aux_ev[1], c->stream), "backward: events");
    }
    auto recompute = [&](int j) -> hmc_status {
        const int b = j & 1;
        const int t0 = j * k, t1 = (t0 + k < n) ? t0 + k : n;
        if (overlap) ATRY(hipStreamWaitEvent(rs, c->aux_ev[b], 0), "backward: events");
        hmc_status s2 = load_ckpt(c, base, L, j, seg_u[b], rs);
        if (s2 != HMC_OK) return s2;
        if (t1 - 1 > t0) {
            ATRY(seq_begin(c, rs), "backward: recompute");
            for (int t = t0; t + 1 < t1; ++t) {
                float* ut = seg_u[b] + (size_t)(t - t0) * 3 * n3;
                ATRY(seq_step(c, rs, t - t0, ut, ut + 3 * n3, seg_E[b] + (size_t)(t - t0) * 8),
                     "backward: recompute");   // records E_t
            }
            ATRY(seq_end(c, rs, t1 - 1 - t0), "backward: recompute");
        }
        ATRY(hipMemcpyAsync(seg_E[b] + (size_t)(t1 - 1 - t0) * 8, c->d.state + kE, 6 * sizeof(double),
                            hipMemcpyDeviceToDevice, rs),
             "backward: recompute");
        if (overlap) ATRY(hipEventRecord(c->aux_ev[2 + b], rs), "backward: events");
        return HMC_OK;
    };
    st = recompute(n_seg - 1);
    if (st != HMC_OK) return st;
    for (int j = n_seg - 1; j >= 0; --j) {
        const int b = j & 1;
        const int t0 = j * k, t1 = (t0 + k < n) ? t0 + k : n;
        if (j > 0) {
            st = recompute(j - 1);
            if (st != HMC_OK) return st;
        }
        if (overlap) ATRY(hipStreamWaitEvent(c->stream, c->aux_ev[2 + b], 0), "backward: events");
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
            a.u_t = seg_u[b] + (size_t)(t - t0) * 3 * n3;
            a.E_t = seg_E[b] + (size_t)(t - t0) * 8;
            a.st_in = i_adj > 0 ? aseq + ((i_adj - 1) & 1) * kAdjSeq : adj;
            a.st_out = aseq + (i_adj & 1) * kAdjSeq;
            a.sums_in = i_adj > 0 ? asums + ((i_adj - 1) % 3) * kSumSlots : nullptr;
            a.sums_out = asums + (i_adj % 3) * kSumSlots;
            a.sums_clear = asums + ((i_adj + 1) % 3) * kSumSlots;
            a.G = G;
            a.reps = c->d.reps;
            a.alpha = R.glob_alpha;
            a.beta = R.glob_beta;
            a.betaE = (double)R.glob_beta;
            a.alphaE = R.glob_alphaE;
            a.order = c->block_order;
            const int tok = prof_begin(c, kProfRefreshStep);
            // the adjoint step keeps 32 x 8 tiles whatever the forward step's rows
            hipLaunchKernelGGL(k_adj_step, dim3(tile_blocks_of(R.K, R.tile_z, kTileY)), dim3(256), 0, c->stream, a);
            prof_end(c, tok);
            ATRY(hipGetLastError(), "backward: step");
            cur_b = 1 - cur_b;
            ++i_adj;
        }
        if (overlap) ATRY(hipEventRecord(c->aux_ev[b], c->stream), "backward: events");
    }
    hipLaunchKernelGGL(k_adj_seq_fold, dim3(1), dim3(64), 0, c->stream, adj, aseq + ((i_adj - 1) & 1) * kAdjSeq,
                       asums + ((i_adj - 1) % 3) * kSumSlots, (double)R.glob_beta, R.glob_alphaE);
    ATRY(hipGetLastError(), "backward: step");
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
    st = load_ckpt(c, base, L, L.n_ck - 1, c->d.u[0], c->stream);
    if (st != HMC_OK) return st;
    c->cur_u = 0;
    ATRY(launch_global_final(c, true), "backward: restore");
    ATRY(hipStreamSynchronize(c->stream), "backward: restore");
    return HMC_OK;
}

}  // extern "C"
