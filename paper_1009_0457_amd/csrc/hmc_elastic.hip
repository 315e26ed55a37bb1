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
// k_global_step_tiled does the node part for every node (reading u, writing the other u
// buffer, so no node sees a half-updated neighbour) and adds its blocks' stress sums into
// fixed-point accumulators; the next step's blocks first advance E from them, and
// k_seq_fold does so after a sequence's last step.  k_global_final writes the stress field
// the zone solves read.
#include "hmc_device.h"

namespace hmc {

struct GlobArgs {
    const int16_t* spins;
    const float* Ctab;
    const float* uin;
    float* uout;
    float* w;
    const unsigned long long* sums_in;   // the previous step's stress sums (null: first step)
    unsigned long long* sums_out;        // this step's
    unsigned long long* sums_clear;      // the next step's, cleared here
    const double* st_in;     // (E, wE) the previous step started from, or the context's state
    int st_in_stride;        // doubles per replica in st_in
    double* st_out;          // (E, wE) of this step (kSeqState per replica)
    double* E_record;        // optional: receives the step's E (single lattice)
    const RepDev* reps;
    const int32_t* tile_rep;
    int64_t plane;
    int order;                           // logical block order (hmc_set_block_order)
};

// (E, wE) of the step after the one that started from st_in and whose stress sums are in
// sums (Sec. 5's average-stress control: r_E = Sigma - <sigma>, wE <- beta wE + alphaE r_E,
// E <- E + wE), component I; sums == null: st_in unchanged.
__device__ __forceinline__ void advance_E(const RepDev* reps, int r, const double* st_in, int stride,
                                          const unsigned long long* sums, int I, double& E_I, double& wE_I)
{
    const RepDev& R = reps[r];
    E_I = st_in[(int64_t)r * stride + I];
    wE_I = st_in[(int64_t)r * stride + 6 + I];
    if (sums) {
        const unsigned long long* sm = sums + (int64_t)r * kSumSlots + I;
        long long tot = 0;
#pragma unroll
        for (int c = 0; c < kSumCopies; ++c) tot += (long long)sm[c * 8];
        const double rE = R.Sigma[I] - (double)tot / (kSumScale * (double)R.n3);
        wE_I = (double)R.glob_beta * wE_I + R.glob_alphaE * rE;
        E_I += wE_I;
    }
}


// Tiled explicit step.  A block owns a 32 x 8 tile of nodes in x, y and marches through
// tile_z node layers in z, so each voxel stress is formed once per tile (1.3x with the halo
// voxels) instead of once per corner node (8x).  The trilinear element's sums are factored
// along z, where the march shares them between neighbouring layers:
//  * per node of the layer pair (z, z+1) and component: S = u(z+1) + u(z), D = u(z+1) - u(z);
//    a voxel's gradient is then 1/4 of (S10 - S00) + (S11 - S01) in x, (S01 - S00) + (S11 - S10)
//    in y and D00 + D10 + D01 + D11 in z over its four node columns;
//  * per voxel column of the layer pair (z-1, z): the stress sums P = s(z) + s(z-1) and
//    differences M = s(z) - s(z-1) that the three force components need (P of xx, yy, yz,
//    xz, xy; M of zz, yz, xz); a node's force is then 1/4 of a signed sum over its four
//    voxel columns.
// Each thread loads the same (x, y) positions of every layer, so the previous layer's
// displacements and stresses stay in its registers.  The own nodes' displacements pass
// through a three-layer LDS ring, which leaves two barriers per layer.  The interior voxels
// are formed in 8 x 8 patches, one per wavefront, so that a wavefront's voxels mostly share
// one grain and its stiffness comes through the scalar cache.
// (At most 128 VGPRs, so that four blocks share a CU: the LDS would allow five.)
// TY = 8 (256 threads, four blocks per CU), 16 (512 threads, two) or 32 (1024 threads, one):
// taller tiles load fewer halo nodes and voxels per owned node and re-read fewer y-halo rows
// of neighbouring tiles.  All give bit-identical results: wavefronts 4g .. 4g+3 of a tall tile
// hold exactly the voxels and sums of the g-th 8-row tile inside it, and each 8-row group's
// stress sums are totalled and rounded to fixed point on their own, as an 8-row block would.
// The own nodes' u and w are read and written once per step; with NT (lattices too large for
// the Infinity Cache) non-temporal accesses keep them from displacing the halo rows that
// neighbouring tiles read from L2 (512^3 on 16-row tiles: 1.73 -> 1.66 ms).
template <int TY, bool NT>
__global__ __launch_bounds__(32 * TY, TY == 8 ? 4 : TY == 16 ? 2 : 1) void k_global_step_tiled(GlobArgs a)
{
    constexpr int THREADS = kTileX * TY;
    constexpr int NX = kTileX + 2, NY = TY + 2, VX = kTileX + 1, VY = TY + 1;
    constexpr int NVOX = VX * VY;
    constexpr int NP = (NX * NY + THREADS - 1) / THREADS, VP = (NVOX + THREADS - 1) / THREADS;
    // LDS entries are vectors, so that each holds what one lane writes or reads at a time:
    // node pair (S0, D0, S1, D1) and (S2, D2); voxel pair (P_xx, P_yy, P_yz, P_xz) and
    // (P_xy, M_zz, M_yz, M_xz); own node (u0, u1, u2, -)
    __shared__ float4 sNa[NY][NX];
    __shared__ float2 sNb[NY][NX];
    __shared__ float4 sPa[VY][VX], sPb[VY][VX];
    __shared__ float4 sraw[3][TY][kTileX];

    const int lb = logical_block((int)blockIdx.x, (int)gridDim.x, a.order);   // neighbouring tiles share an L2
    const int r = a.tile_rep[lb];
    const RepDev R = a.reps[r];
    const int K = R.K;
    const int ntx = (K + kTileX - 1) / kTileX, nty = (K + TY - 1) / TY, tz = R.tile_z;
    int b = lb - R.tile_first;
    const int bx = b % ntx;
    b /= ntx;
    const int by = b % nty, bz = b / nty;
    const int x0 = bx * kTileX, y0 = by * TY, z0 = bz * tz;
    const int z1 = (z0 + tz < K) ? z0 + tz : K;
    const int16_t* spins = a.spins + R.site_off;
    const float* Ctab = a.Ctab + R.grain_off * kTab;
    const float* uin = a.uin + R.site_off;
    float* uout = a.uout + R.site_off;
    float* w = a.w + R.site_off;
    const int64_t P = a.plane;
    // this step's E (read after the prologue's first barrier); the replica's first block
    // records it and clears the accumulators of the step after
    __shared__ double sE[6];
    if (threadIdx.x < 6) {
        double E_I, wE_I;
        advance_E(a.reps, r, a.st_in, a.st_in_stride, a.sums_in, threadIdx.x, E_I, wE_I);
        sE[threadIdx.x] = E_I;
        if (lb == R.tile_first) {
            a.st_out[(int64_t)r * kSeqState + threadIdx.x] = E_I;
            a.st_out[(int64_t)r * kSeqState + 6 + threadIdx.x] = wE_I;
            if (a.E_record) a.E_record[threadIdx.x] = E_I;
        }
    }
    if (lb == R.tile_first && threadIdx.x < kSumSlots) a.sums_clear[(int64_t)r * kSumSlots + threadIdx.x] = 0ull;
    float E[6];
    const float alpha4 = 0.25f * R.glob_alpha, beta = R.glob_beta;
    const int t = threadIdx.x, lx = t % kTileX, ly = t / kTileX;
    const int nx = x0 + lx, ny = y0 + ly;
    const bool own = nx < K && ny < K;
    double acc[6] = {0, 0, 0, 0, 0, 0};

    // tile positions this thread loads (nodes) and forms (voxels), the same in every layer
    int node_xy[NP], vox_xy[VP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int i = t + THREADS * k, ix = i % NX, iy = i / NX;
        node_xy[k] = wrap_tile(x0 - 1 + ix, K) + K * wrap_tile(y0 - 1 + iy, K);
    }
#pragma unroll
    for (int k = 0; k < VP; ++k) {
        int ix, iy;
        step_voxel_pos<TY>(t + THREADS * k, ix, iy);
        vox_xy[k] = wrap_tile(x0 - 1 + ix, K) + K * wrap_tile(y0 - 1 + iy, K);
    }
    // Node layer z+2 and voxel layer z+1's grains are fetched into registers while layer z
    // is computed.
    float pf[NP][3], prev[NP][3];
    int sp[VP];
    auto fetch_nodes = [&](int z) {
        const int64_t zoff = (int64_t)K * K * wrap_tile(z, K);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int i = t + THREADS * k;
            if (i < NX * NY) {
                const int64_t n = node_xy[k] + zoff;
                pf[k][0] = uin[n];
                pf[k][1] = uin[P + n];
                pf[k][2] = uin[2 * P + n];
            }
        }
    };
    auto fetch_spins = [&](int z) {
        const int64_t zoff = (int64_t)K * K * wrap_tile(z, K);
#pragma unroll
        for (int k = 0; k < VP; ++k) {
            const int i = t + THREADS * k;
            sp[k] = 0;
            if (i < NVOX) sp[k] = spins[vox_xy[k] + zoff];
        }
    };
    // pf holds node layer z+1 and prev layer z: write the pair's S and D, and layer z+1's own
    // nodes into ring slot `raw`
    auto store_pair = [&](int raw) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int i = t + THREADS * k;
            if (i < NX * NY) {
                const int ix = i % NX, iy = i / NX;
                pair_node_entry(pf[k], prev[k], sNa[iy][ix], sNb[iy][ix]);
#pragma unroll
                for (int j = 0; j < 3; ++j) prev[k][j] = pf[k][j];
                if (ix >= 1 && ix <= kTileX && iy >= 1 && iy <= TY)
                    sraw[raw][iy - 1][ix - 1] = make_float4(pf[k][0], pf[k][1], pf[k][2], 0.f);
            }
        }
    };
    // stress of voxel position k of the layer whose node pair is in sNa / sNb (grains in q)
    auto voxel_stress = [&](int k, int q, float s6[6]) {
        int ix, iy;
        step_voxel_pos<TY>(t + THREADS * k, ix, iy);
        float e[6];
        pair_strain<NX>(sNa, sNb, ix, iy, E, e);
        symv21_grains(Ctab, q, e, s6);
    };

    // prologue: node layers z0-1, z0 -> voxel layer z0-1 (kept in registers)
    int ring = 0;                                // sraw slot of layer z
    fetch_nodes(z0 - 1);
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) prev[k][j] = pf[k][j];
    fetch_nodes(z0);
    fetch_spins(z0 - 1);
    store_pair(ring);
    __syncthreads();
#pragma unroll
    for (int I = 0; I < 6; ++I) E[I] = (float)sE[I];
    float sprev[VP][6];
#pragma unroll
    for (int k = 0; k < VP; ++k)
        if (t + THREADS * k < NVOX) voxel_stress(k, sp[k], sprev[k]);
    fetch_nodes(z0 + 1);
    fetch_spins(z0);
    __syncthreads();                             // the prologue's reads of sNa / sNb are done

    for (int z = z0; z < z1; ++z) {
        const int ring_next = ring == 2 ? 0 : ring + 1;
        store_pair(ring_next);                   // pair (z, z+1); own nodes of layer z+1
        // This layer's grains arrived during the last layer: take them now, so that no
        // later wait on them also waits for the loads issued below.  The own nodes' w is
        // needed first (at the end of this layer), so it is requested before the prefetch.
        int sp_cur[VP];
#pragma unroll
        for (int k = 0; k < VP; ++k) {
            sp_cur[k] = sp[k];
            asm volatile("" ::"v"(sp_cur[k]));
        }
        float wz[3] = {0.f, 0.f, 0.f};
        const int64_t n = nx + (int64_t)K * (ny + (int64_t)K * z);
        if (own) {
#pragma unroll
            for (int j = 0; j < 3; ++j) wz[j] = NT ? __builtin_nontemporal_load(&w[(int64_t)j * P + n]) : w[(int64_t)j * P + n];
        }
        if (z + 1 < z1) {
            fetch_nodes(z + 2);                  // in flight during this layer
            fetch_spins(z + 1);
        }
        __syncthreads();                         // the node pair is complete
#pragma unroll
        for (int k = 0; k < VP; ++k) {
            const int i = t + THREADS * k;
            if (i >= NVOX) continue;
            int ix, iy;
            step_voxel_pos<TY>(i, ix, iy);
            float s6[6];
            voxel_stress(k, sp_cur[k], s6);
            pair_voxel_entry(s6, sprev[k], sPa[iy][ix], sPb[iy][ix]);
#pragma unroll
            for (int I = 0; I < 6; ++I) sprev[k][I] = s6[I];
            const int gx = x0 - 1 + ix, gy = y0 - 1 + iy;
            if (ix >= 1 && iy >= 1 && gx < K && gy < K) {
#pragma unroll
                for (int I = 0; I < 6; ++I) acc[I] += (double)s6[I];
            }
        }
        __syncthreads();                         // the voxel pair is complete
        if (own) {
            float F[3];
            pair_force<VX>(sPa, sPb, lx, ly, F);
            const float4 u = sraw[ring][ly][lx];
            const float uz[3] = {u.x, u.y, u.z};
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int64_t idx = (int64_t)j * P + n;
                const float wn = beta * wz[j] - alpha4 * F[j];
                if (NT) {
                    __builtin_nontemporal_store(wn, &w[idx]);
                    __builtin_nontemporal_store(uz[j] + wn, &uout[idx]);
                } else {
                    w[idx] = wn;
                    uout[idx] = uz[j] + wn;
                }
            }
        }
        ring = ring_next;
    }
    const double tot = block_total_quads<6, TY / 8>(acc);
    const int k = threadIdx.x & 255;             // total k of the half threadIdx.x / 256
    if (k < 6) {
        const unsigned copy = (unsigned)(lb - R.tile_first + (threadIdx.x >> 8)) & (kSumCopies - 1);
        atomicAdd(a.sums_out + (int64_t)r * kSumSlots + copy * 8 + k, (unsigned long long)llrint(tot * kSumScale));
    }
}

// After a sequence's last step: the context's (E, wE), one block per replica.
__global__ void k_seq_fold(double* state, const double* st_last, const unsigned long long* sums_last,
                           const RepDev* reps)
{
    const int r = blockIdx.x, I = threadIdx.x;
    if (I >= 6) return;
    double E_I, wE_I;
    advance_E(reps, r, st_last, kSeqState, sums_last, I, E_I, wE_I);
    state[(int64_t)r * kStateDoubles + kE + I] = E_I;
    state[(int64_t)r * kStateDoubles + kWE + I] = wE_I;
}

struct FinalArgs {
    const int16_t* spins;
    const float* Ctab;
    const float* u;
    float* sigma;       // may be null
    double* partials;
    const double* state;
    const RepDev* reps;
    const int32_t* node_rep;
    int64_t plane;
};

__global__ __launch_bounds__(256) void k_global_final(FinalArgs a)
{
    const NodeRange nr = node_range(a.reps, a.node_rep);
    const RepDev& R = nr.R;
    const int K = R.K;
    const double* st = a.state + (int64_t)a.node_rep[blockIdx.x] * kStateDoubles;
    float E[6];
#pragma unroll
    for (int I = 0; I < 6; ++I) E[I] = (float)st[kE + I];
    const int16_t* spins = a.spins + R.site_off;
    const float* Ctab = a.Ctab + R.grain_off * kTab;
    const float* u = a.u + R.site_off;
    double U[1] = {0.0};
    for (int64_t v = nr.first; v < R.n3; v += nr.stride) {
        const int x = (int)(v % K), y = (int)((v / K) % K), z = (int)(v / ((int64_t)K * K));
        float e[6], s[6];
        voxel_strain(u, a.plane, K, x, y, z, E, e);
        symv21(Ctab + (int64_t)spins[v] * kTab, e, s);
        double d = 0.0;
#pragma unroll
        for (int I = 0; I < 6; ++I) d += (double)s[I] * (double)e[I];
        U[0] += 0.5 * d;
        if (a.sigma)
#pragma unroll
            for (int I = 0; I < 6; ++I) a.sigma[(int64_t)I * a.plane + R.site_off + v] = s[I];
    }
    block_sum_to<1>(a.partials, U);
}

// One block per replica: stored energy = fixed-order sum of the block partials.
// A non-finite stress or strain anywhere in the replica makes its energy non-finite, which
// raises kNfGlobal.
__global__ __launch_bounds__(256) void k_sum_U(double* state, const double* partials, const RepDev* reps,
                                               uint32_t* nonfinite)
{
    const RepDev R = reps[blockIdx.x];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int b = t; b < R.node_blocks; b += 256) s += partials[(int64_t)(R.node_first + b) * 8];
    const double v[1] = {s};
    const double tot = block_total<1>(v);
    if (t == 0) {
        state[(int64_t)blockIdx.x * kStateDoubles + kU] = tot;
        if (!isfinite(tot)) atomicOr(nonfinite, (uint32_t)kNfGlobal);
    }
}

struct ReussArgs {
    const int16_t* spins;
    const float* Stab;
    double* partials;
    const RepDev* reps;
    const int32_t* node_rep;
};

// Per-block sums of S_{q_v} Sigma (the uniform-stress strain of each site).
__global__ __launch_bounds__(256) void k_reuss(ReussArgs a)
{
    const NodeRange nr = node_range(a.reps, a.node_rep);
    const RepDev& R = nr.R;
    const int16_t* spins = a.spins + R.site_off;
    const float* Stab = a.Stab + R.grain_off * kTab;
    float Sig[6];
#pragma unroll
    for (int I = 0; I < 6; ++I) Sig[I] = (float)R.Sigma[I];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t v = nr.first; v < R.n3; v += nr.stride) {
        float e[6];
        symv21(Stab + (int64_t)spins[v] * kTab, Sig, e);
#pragma unroll
        for (int I = 0; I < 6; ++I) acc[I] += (double)e[I];
    }
    block_sum_to<6>(a.partials, acc);
}

// One block per replica: E = mean(S_q) Sigma, wE = 0.
__global__ __launch_bounds__(256) void k_reuss_E(double* state, const double* partials, const RepDev* reps)
{
    const RepDev R = reps[blockIdx.x];
    const int t = threadIdx.x;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int b = t; b < R.node_blocks; b += 256)
#pragma unroll
        for (int I = 0; I < 6; ++I) s[I] += partials[(int64_t)(R.node_first + b) * 8 + I];
    const double tot = block_total<6>(s);
    if (t < 6) {
        double* st = state + (int64_t)blockIdx.x * kStateDoubles;
        st[kE + t] = tot / (double)R.n3;
        st[kWE + t] = 0.0;
    }
}

__global__ void k_zero_wE(double* state, int n_rep)
{
    for (int r = blockIdx.x; r < n_rep; r += gridDim.x)
        if (threadIdx.x < 6) state[(int64_t)r * kStateDoubles + kWE + threadIdx.x] = 0.0;
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

hipError_t launch_reuss(hmc_ctx_s* c)
{
    ReussArgs a;
    a.spins = c->d.spins;
    a.Stab = c->d.Stab;
    a.partials = c->d.partials;
    a.reps = c->d.reps;
    a.node_rep = c->d.node_rep;
    hipLaunchKernelGGL(k_reuss, dim3(c->node_blocks), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL(k_reuss_E, dim3(c->n_rep), dim3(256), 0, c->stream, c->d.state, c->d.partials, c->d.reps);
    return hipGetLastError();
}

hipError_t seq_begin(hmc_ctx_s* c, hipStream_t s)
{
    // the first step adds into buffer 0, which starts cleared; each step clears the next
    const int tok = s == c->stream ? prof_begin(c, kProfRefreshOther) : -1;
    // (buffers 0 and 1: 2 x kSumSlots 64-bit words per replica, 2 uint32 each)
    const hipError_t e = launch_fill_u32((uint32_t*)c->d.sums, 0u, 4 * (int64_t)c->n_rep * kSumSlots, s);
    prof_end(c, tok);
    return e;
}

hipError_t seq_step(hmc_ctx_s* c, hipStream_t s, int i, const float* uin, float* uout, double* E_record)
{
    const int64_t per = (int64_t)c->n_rep * kSumSlots;
    GlobArgs a;
    a.spins = c->d.spins;
    a.Ctab = c->d.Ctab;
    a.uin = uin;
    a.uout = uout;
    a.w = c->d.w;
    a.sums_in = i > 0 ? c->d.sums + ((i - 1) % 3) * per : nullptr;
    a.sums_out = c->d.sums + (i % 3) * per;
    a.sums_clear = c->d.sums + ((i + 1) % 3) * per;
    a.st_in = i > 0 ? c->d.seq_state + (int64_t)((i - 1) & 1) * c->n_rep * kSeqState : c->d.state + kE;
    a.st_in_stride = i > 0 ? kSeqState : kStateDoubles;
    a.st_out = c->d.seq_state + (int64_t)(i & 1) * c->n_rep * kSeqState;
    a.E_record = E_record;
    a.reps = c->d.reps;
    a.tile_rep = c->d.tile_rep;
    a.order = c->block_order;
    a.plane = c->total_sites;
    const int tok = s == c->stream ? prof_begin(c, kProfRefreshStep) : -1;
    const dim3 g(c->tile_blocks);
    if (c->reps[0].tile_y == 32) {
        if (c->step_streams)
            hipLaunchKernelGGL((k_global_step_tiled<32, true>), g, dim3(kTileX * 32), 0, s, a);
        else
            hipLaunchKernelGGL((k_global_step_tiled<32, false>), g, dim3(kTileX * 32), 0, s, a);
    } else if (c->reps[0].tile_y == 16) {
        if (c->step_streams)
            hipLaunchKernelGGL((k_global_step_tiled<16, true>), g, dim3(kTileX * 16), 0, s, a);
        else
            hipLaunchKernelGGL((k_global_step_tiled<16, false>), g, dim3(kTileX * 16), 0, s, a);
    } else {
        if (c->step_streams)
            hipLaunchKernelGGL((k_global_step_tiled<8, true>), g, dim3(kTileX * 8), 0, s, a);
        else
            hipLaunchKernelGGL((k_global_step_tiled<8, false>), g, dim3(kTileX * 8), 0, s, a);
    }
    prof_end(c, tok);
    return hipGetLastError();
}

hipError_t seq_end(hmc_ctx_s* c, hipStream_t s, int n)
{
    if (n <= 0) return hipSuccess;
    const int64_t per = (int64_t)c->n_rep * kSumSlots;
    const int tok = s == c->stream ? prof_begin(c, kProfRefreshOther) : -1;
    hipLaunchKernelGGL(k_seq_fold, dim3(c->n_rep), dim3(64), 0, s, c->d.state,
                       c->d.seq_state + (int64_t)((n - 1) & 1) * c->n_rep * kSeqState,
                       c->d.sums + ((n - 1) % 3) * per, c->d.reps);
    prof_end(c, tok);
    return hipGetLastError();
}

hipError_t launch_global_steps(hmc_ctx_s* c, int n_steps)
{
    if (n_steps <= 0) return hipSuccess;
    hipError_t e = seq_begin(c, c->stream);
    for (int s = 0; s < n_steps && e == hipSuccess; ++s) {
        e = seq_step(c, c->stream, s, c->d.u[c->cur_u], c->d.u[1 - c->cur_u], nullptr);
        c->cur_u = 1 - c->cur_u;
    }
    if (e == hipSuccess) e = seq_end(c, c->stream, n_steps);
    return e;
}

hipError_t launch_global_final(hmc_ctx_s* c, bool write_sigma)
{
    FinalArgs a;
    a.spins = c->d.spins;
    a.Ctab = c->d.Ctab;
    a.u = c->d.u[c->cur_u];
    a.sigma = write_sigma ? c->d.sigma : nullptr;
    a.partials = c->d.partials;
    a.state = c->d.state;
    a.reps = c->d.reps;
    a.node_rep = c->d.node_rep;
    a.plane = c->total_sites;
    const int tok = prof_begin(c, kProfRefreshOther);
    hipLaunchKernelGGL(k_global_final, dim3(c->node_blocks), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL(k_sum_U, dim3(c->n_rep), dim3(256), 0, c->stream, c->d.state, c->d.partials, c->d.reps,
                       c->d.counters + kNonFinite);
    prof_end(c, tok);
    return hipGetLastError();
}

hipError_t launch_zero_wE(hmc_ctx_s* c)
{
    hipLaunchKernelGGL(k_zero_wE, dim3(c->n_rep < 1024 ? c->n_rep : 1024), dim3(64), 0, c->stream, c->d.state,
                       c->n_rep);
    return hipGetLastError();
}

hipError_t launch_unlike_bonds(hmc_ctx_s* c, int rep)
{
    const RepDev& R = c->reps[rep];
    int64_t g = (R.n3 + 255) / 256;
    if (g > 4096) g = 4096;
    const int16_t* sp = c->d.spins + R.site_off;
    if (c->p.neighbors == 26)
        hipLaunchKernelGGL(k_unlike<26>, dim3((unsigned)g), dim3(256), 0, c->stream, sp, R.K, R.n3, c->d.bonds);
    else
        hipLaunchKernelGGL(k_unlike<6>, dim3((unsigned)g), dim3(256), 0, c->stream, sp, R.K, R.n3, c->d.bonds);
    return hipGetLastError();
}

hipError_t launch_texture(hmc_ctx_s* c, int rep, int nbins)
{
    const RepDev& R = c->reps[rep];
    int64_t g = (R.n3 + 255) / 256;
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_texture, dim3((unsigned)g), dim3(256), 0, c->stream, c->d.spins + R.site_off,
                       c->d.tex_bin + R.grain_off, R.n3, nbins, c->d.hist);
    return hipGetLastError();
}

}  // namespace hmc
