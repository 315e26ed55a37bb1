// hmc_device.h -- device helpers shared by the global-solve and adjoint kernels.
#pragma once

#include "hmc_internal.h"

namespace hmc {

__device__ __forceinline__ int wrapk(int a, int K) { return a < 0 ? a + K : (a >= K ? a - K : a); }

// Periodic wrap of any a >= -K: a compare and an add for a < 2K (every coordinate of a
// large lattice), an exact remainder beyond (tile halos on lattices narrower than a tile).
__device__ __forceinline__ int wrap_tile(int a, int K)
{
    if (a < 0) return a + K;
    if (a < K) return a;
    a -= K;
    return a < K ? a : a % K;
}

template <class Tab>
__device__ __forceinline__ void symv21(Tab c, const float e[6], float s[6])
{
    s[0] = c[0] * e[0] + c[1] * e[1] + c[2] * e[2] + c[3] * e[3] + c[4] * e[4] + c[5] * e[5];
    s[1] = c[1] * e[0] + c[6] * e[1] + c[7] * e[2] + c[8] * e[3] + c[9] * e[4] + c[10] * e[5];
    s[2] = c[2] * e[0] + c[7] * e[1] + c[11] * e[2] + c[12] * e[3] + c[13] * e[4] + c[14] * e[5];
    s[3] = c[3] * e[0] + c[8] * e[1] + c[12] * e[2] + c[15] * e[3] + c[16] * e[4] + c[17] * e[5];
    s[4] = c[4] * e[0] + c[9] * e[1] + c[13] * e[2] + c[16] * e[3] + c[18] * e[4] + c[19] * e[5];
    s[5] = c[5] * e[0] + c[10] * e[1] + c[14] * e[2] + c[17] * e[3] + c[19] * e[4] + c[20] * e[5];
}

// The 21 entries of grain q's table when q is the same in every active lane (e.g. from
// readfirstlane), read through the scalar data cache: the constant address space lets the
// compiler use scalar loads, which leave the vector memory path (and its in-order wait
// counter) to the field data.  Tables are read-only while any kernel that reads them runs.
typedef const __attribute__((address_space(4))) float* UniformTab;
__device__ __forceinline__ void uniform_row(const float* tab, int q, float c[21])
{
    const UniformTab u = (UniformTab)(tab + (int64_t)q * kTab);
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(u[i])));
}

// s = C_q e over a wavefront whose lanes mostly share the grain q (neighbouring voxels of a
// polycrystal).  One grain in the wavefront: one product with its table from scalar loads.
// Two grains: a product with each (the second in its lanes only).  More: each lane gathers
// its own table.  Each lane's result is symv21 with its own table.
__device__ __forceinline__ void symv21_grains(const float* tab, int q, const float e[6], float s[6])
{
    const int q0 = __builtin_amdgcn_readfirstlane(q);
    const uint64_t other = __builtin_amdgcn_ballot_w64(q != q0);
    float c[21];
    if (other == 0) {
        uniform_row(tab, q0, c);
        symv21(c, e, s);
    } else {
        const int q1 = __builtin_amdgcn_readlane(q, (int)__builtin_ctzll(other));
        if (__builtin_amdgcn_ballot_w64(q != q0 && q != q1) == 0) {
            uniform_row(tab, q0, c);
            symv21(c, e, s);
            uniform_row(tab, q1, c);
            if (q == q1) symv21(c, e, s);
        } else {
            symv21(tab + (int64_t)q * kTab, e, s);
        }
    }
}

// Voxel positions of a 32 x TY node tile's layer (33 x (TY + 1) voxels, tile-relative; voxel
// (ix, iy) has the tile's nodes ix, ix+1 and iy, iy+1 as corners, node 0 being the low halo)
// in the order the 32 TY threads of a tiled step take them: first the 32 x TY voxels whose
// high corner is an own node, as 8 x 8 patches, one per wavefront (neighbouring voxels mostly
// share a grain), then the low halo row and column.  kStepVox counts them for TY = 8.
constexpr int kStepVox = (kTileX + 1) * (kTileY + 1);
static_assert(kTileX == 32 && kTileY == 8, "voxel patches assume 32-wide tiles of 8, 16 or 32 rows");
// For a 32 x TY tile (TY = 8, 16 or 32; 32 TY threads): wavefront w takes the 8 x 8 patch at x in
// [8 (w % 4) + 1, 8 (w % 4) + 8], y in [8 (w / 4) + 1, 8 (w / 4) + 8].
template <int TY = kTileY>
__device__ __forceinline__ void step_voxel_pos(int i, int& ix, int& iy)
{
    static_assert(TY == 8 || TY == 16 || TY == 32, "tile rows");
    constexpr int NI = kTileX * TY;
    if (i < NI) {                          // interior patches
        const int w = i >> 6;
        ix = 1 + 8 * (w & 3) + (i & 7);
        iy = 1 + 8 * (w >> 2) + ((i & 63) >> 3);
    } else if (i < NI + kTileX + 1) {      // halo row y = 0
        ix = i - NI;
        iy = 0;
    } else {                               // halo column x = 0
        ix = 0;
        iy = i - (NI + kTileX + 1) + 1;
    }
}

// Layer-pair sums of the tiled steps.  A node entry holds, for the pair of node layers
// (z, z+1), S = u(z+1) + u(z) and D = u(z+1) - u(z) of each component as (S0, D0, S1, D1) and
// (S2, D2); a voxel entry holds, for the pair of voxel layers (z-1, z), sums P = s(z) + s(z-1)
// and differences M = s(z) - s(z-1) of a symmetric tensor field as (P_xx, P_yy, P_yz, P_xz)
// and (P_xy, M_zz, M_yz, M_xz).
__device__ __forceinline__ void pair_node_entry(const float hi[3], const float lo[3], float4& na, float2& nb)
{
    na = make_float4(hi[0] + lo[0], hi[0] - lo[0], hi[1] + lo[1], hi[1] - lo[1]);
    nb = make_float2(hi[2] + lo[2], hi[2] - lo[2]);
}

__device__ __forceinline__ void pair_voxel_entry(const float s[6], const float sp[6], float4& pa, float4& pb)
{
    pa = make_float4(s[0] + sp[0], s[1] + sp[1], s[3] + sp[3], s[4] + sp[4]);
    pb = make_float4(s[5] + sp[5], s[2] - sp[2], s[3] - sp[3], s[4] - sp[4]);
}

// base + the symmetric gradient (engineering shears) of the trilinear field at the centre of
// voxel (ix, iy) between the two node layers: with S, D at the voxel's node columns 00, 10,
// 01, 11, 4 du/dx = (S10 - S00) + (S11 - S01), 4 du/dy = (S01 - S00) + (S11 - S10) and
// 4 du/dz = D00 + D10 + D01 + D11.
template <int NX>
__device__ __forceinline__ void pair_strain(const float4 (*Na)[NX], const float2 (*Nb)[NX], int ix, int iy,
                                            const float base[6], float e[6])
{
    float S[3][4], D[3][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float4 na = Na[iy + (c >> 1)][ix + (c & 1)];
        const float2 nb = Nb[iy + (c >> 1)][ix + (c & 1)];
        S[0][c] = na.x;
        D[0][c] = na.y;
        S[1][c] = na.z;
        D[1][c] = na.w;
        S[2][c] = nb.x;
        D[2][c] = nb.y;
    }
    float G[3][3];   // 4 du_j / dx_d
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        G[j][0] = (S[j][1] - S[j][0]) + (S[j][3] - S[j][2]);
        G[j][1] = (S[j][2] - S[j][0]) + (S[j][3] - S[j][1]);
        G[j][2] = (D[j][0] + D[j][1]) + (D[j][2] + D[j][3]);
    }
    e[0] = base[0] + 0.25f * G[0][0];
    e[1] = base[1] + 0.25f * G[1][1];
    e[2] = base[2] + 0.25f * G[2][2];
    e[3] = base[3] + 0.25f * (G[1][2] + G[2][1]);
    e[4] = base[4] + 0.25f * (G[0][2] + G[2][0]);
    e[5] = base[5] + 0.25f * (G[0][1] + G[1][0]);
}

// 4 x sum over the 8 voxels around tile node (lx+1, ly+1) of B_v(n)^T s_v, from the voxel
// pair entries: its voxel columns a = (lx, ly), b = (lx+1, ly), c = (lx, ly+1),
// d = (lx+1, ly+1) carry x weight + for a, c, y weight + for a, b and z weight + for the
// lower layer, i.e. - on M.
template <int VX>
__device__ __forceinline__ void pair_force(const float4 (*Pa)[VX], const float4 (*Pb)[VX], int lx, int ly,
                                           float F[3])
{
    const float4 pa = Pa[ly][lx], pb = Pa[ly][lx + 1], pc = Pa[ly + 1][lx], pd = Pa[ly + 1][lx + 1];
    const float4 qa = Pb[ly][lx], qb = Pb[ly][lx + 1], qc = Pb[ly + 1][lx], qd = Pb[ly + 1][lx + 1];
    F[0] = ((pa.x - pb.x) + (pc.x - pd.x)) + ((qa.x - qc.x) + (qb.x - qd.x)) - ((qa.w + qb.w) + (qc.w + qd.w));
    F[1] = ((qa.x - qb.x) + (qc.x - qd.x)) + ((pa.y - pc.y) + (pb.y - pd.y)) - ((qa.z + qb.z) + (qc.z + qd.z));
    F[2] = ((pa.w - pb.w) + (pc.w - pd.w)) + ((pa.z - pc.z) + (pb.z - pd.z)) - ((qa.y + qb.y) + (qc.y + qd.y));
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

// Sum over the 256 threads of a block of v[k], k < NVALS, in a fixed order: a butterfly
// within each wavefront (both lanes of a pair form the same sum), then the four wavefront
// sums in order.  Thread k < NVALS receives total k; the other threads receive 0.
template <int NVALS>
__device__ __forceinline__ double block_total(const double v[NVALS])
{
    __shared__ double red[NVALS][4];
    double s[NVALS];
#pragma unroll
    for (int k = 0; k < NVALS; ++k) s[k] = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < NVALS; ++k) s[k] += __shfl_xor(s[k], o, 64);
    const int t = threadIdx.x;
    if ((t & 63) == 0)
#pragma unroll
        for (int k = 0; k < NVALS; ++k) red[k][t >> 6] = s[k];
    __syncthreads();
    return t < NVALS ? (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]) : 0.0;
}

// block_total for blocks of 4 Q wavefronts, per group of four: thread 256 g + k (k < NVALS)
// receives the total k of wavefronts 4g .. 4g+3, summed exactly as block_total sums a block of
// four; the other threads receive 0.
template <int NVALS, int Q>
__device__ __forceinline__ double block_total_quads(const double v[NVALS])
{
    __shared__ double red[NVALS][4 * Q];
    double s[NVALS];
#pragma unroll
    for (int k = 0; k < NVALS; ++k) s[k] = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < NVALS; ++k) s[k] += __shfl_xor(s[k], o, 64);
    const int t = threadIdx.x;
    if ((t & 63) == 0)
#pragma unroll
        for (int k = 0; k < NVALS; ++k) red[k][t >> 6] = s[k];
    __syncthreads();
    const int k = t & 255, g = t >> 8;
    return k < NVALS ? (red[k][4 * g] + red[k][4 * g + 1]) + (red[k][4 * g + 2] + red[k][4 * g + 3]) : 0.0;
}

// Deterministic block sum of NVALS doubles per thread into partials[slot * 8 + k] (slot: the
// block's logical index, blockIdx.x by default).
template <int NVALS>
__device__ __forceinline__ void block_sum_to(double* __restrict__ partials, const double v[NVALS],
                                             int slot = -1)
{
    const double s = block_total<NVALS>(v);
    if (slot < 0) slot = (int)blockIdx.x;
    if (threadIdx.x < NVALS) partials[(int64_t)slot * 8 + threadIdx.x] = s;
}

// Node-parallel kernels: block b belongs to replica node_rep[b]; within a replica the
// blocks cover 256 consecutive nodes each (and stride by the replica's block count beyond
// 8192 blocks), so the per-block partial sums and their fixed-order folding do not depend
// on how many replicas share the launch.
struct NodeRange {
    RepDev R;
    int64_t first, stride;
};

__device__ __forceinline__ NodeRange node_range(const RepDev* reps, const int32_t* node_rep)
{
    NodeRange n;
    n.R = reps[node_rep[blockIdx.x]];
    n.first = (int64_t)(blockIdx.x - n.R.node_first) * blockDim.x + threadIdx.x;
    n.stride = (int64_t)n.R.node_blocks * blockDim.x;
    return n;
}

}  // namespace hmc
