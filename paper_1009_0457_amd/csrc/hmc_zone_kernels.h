// hmc_zone_kernels.h -- local elastic energy change of each real trial flip (Sec. 3, Eq. H_1
// second form and Fig. 1): the (2h+1)^3-voxel zone around the trial site keeps the
// traction on its boundary, so the flip's energy change is the zone's stored energy minus
// the work of that traction.  With eps_p = S_old sigma_p (the site's strain under its
// stored stress), dC = C_new - C_old and t = dC eps_p, it equals
//     1/2 eps_p.dC eps_p + Phi(du),   Phi(du) = t.(B_p du) + 1/2 sum_v (B_v du).C_v (B_v du),
// minimised over the extra displacement du of the zone's (2h+2)^3 corner nodes (outer
// boundary free) by n_r explicit heavy-ball steps from rest (no early exit).  B_v is the
// centre-point strain of voxel v from its 8 corners; C_v the stiffness of the pass's
// snapshot spin at v, except C_new at the trial site.
//
// Three kernels compute this solve with different layouts (hmc_params.zone_variant):
// k_zone (a wavefront per trial), k_zone_col (node columns of several trials across a
// 256-lane work-group) and k_zone_lane (whole trials inside one wavefront, x neighbours by
// cross-lane moves; the default for h = 1, 2, 3).  State and arithmetic are FP32; the final
// energy is accumulated in FP64.  The decision uses the same predicate as the integer
// path: accept iff dE <= 0 or r1 < 2^32 exp(-dE/kT).
//
// k_zone layout: one 64-lane wavefront (one work-group) owns one trial at a time.  Lane l
// owns voxels l, l+64, ... (their 21 stiffness entries stay in registers) and nodes l,
// l+64, ... (displacement and velocity in registers).  Each step is two phases exchanged
// through LDS:
//   A: every owned voxel reads its 8 corner displacements, forms strain and stress, and
//      publishes the stress;
//   B: every owned node gathers the forces of its (up to 8) voxels, takes the heavy-ball
//      step and publishes its new displacement.
#pragma once
#include "hmc_internal.h"

namespace hmc {

struct ZoneArgs {
    const int16_t* spins;           // all replicas, end to end
    const float* Ctab;
    const float* Stab;
    const float* sigma;             // 6 planes of `plane` floats
    const RepDev* reps;
    const TrialEntry* list;
    const uint32_t* count;
    uint8_t* acc;
    hmc_trial_record* rec;          // indexed by site_off + site, or null
    unsigned long long* stats;
    uint32_t* nonfinite;            // counters[kNonFinite]
    int nr;
    int order;                      // logical block order (hmc_set_block_order)
    int64_t plane;
    float alpha, beta;
};

// The trial's replica, its lattice, grain tables and decision constants.
struct TrialCtx {
    const int16_t* spins;
    const float* Ctab;
    const float* Stab;
    int64_t site_off;
    int K;
    double J, kT, lambda;
};

__device__ __forceinline__ TrialCtx trial_ctx(const ZoneArgs& a, uint32_t qr)
{
    const RepDev& R = a.reps[qr >> 16];
    TrialCtx c;
    c.spins = a.spins + R.site_off;
    c.Ctab = a.Ctab + R.grain_off * kTab;
    c.Stab = a.Stab + R.grain_off * kTab;
    c.site_off = R.site_off;
    c.K = R.K;
    c.J = R.J;
    c.kT = R.kT;
    c.lambda = R.lambda;
    return c;
}

__device__ __forceinline__ void load_sym(const float* __restrict__ t, float c[21])
{
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = t[i];
}

// s = C e for a symmetric Voigt matrix stored as its upper triangle.
__device__ __forceinline__ void symv(const float c[21], const float e[6], float s[6])
{
    s[0] = c[0] * e[0] + c[1] * e[1] + c[2] * e[2] + c[3] * e[3] + c[4] * e[4] + c[5] * e[5];
    s[1] = c[1] * e[0] + c[6] * e[1] + c[7] * e[2] + c[8] * e[3] + c[9] * e[4] + c[10] * e[5];
    s[2] = c[2] * e[0] + c[7] * e[1] + c[11] * e[2] + c[12] * e[3] + c[13] * e[4] + c[14] * e[5];
    s[3] = c[3] * e[0] + c[8] * e[1] + c[12] * e[2] + c[15] * e[3] + c[16] * e[4] + c[17] * e[5];
    s[4] = c[4] * e[0] + c[9] * e[1] + c[13] * e[2] + c[16] * e[3] + c[18] * e[4] + c[19] * e[5];
    s[5] = c[5] * e[0] + c[10] * e[1] + c[14] * e[2] + c[17] * e[3] + c[19] * e[4] + c[20] * e[5];
}

// Centre-point Voigt strain of a voxel from its corner displacements u[c], c = a + 2b + 4d.
__device__ __forceinline__ void corner_strain(const float4 u[8], float e[6])
{
    float gx[3], gy[3], gz[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        auto comp = [&](int c) { return j == 0 ? u[c].x : (j == 1 ? u[c].y : u[c].z); };
        const float s01 = comp(0) + comp(1), s23 = comp(2) + comp(3), s45 = comp(4) + comp(5),
                    s67 = comp(6) + comp(7);
        const float d01 = comp(1) - comp(0), d23 = comp(3) - comp(2), d45 = comp(5) - comp(4),
                    d67 = comp(7) - comp(6);
        gx[j] = 0.25f * ((d01 + d23) + (d45 + d67));
        gy[j] = 0.25f * ((s23 - s01) + (s67 - s45));
        gz[j] = 0.25f * ((s45 + s67) - (s01 + s23));
    }
    e[0] = gx[0];
    e[1] = gy[1];
    e[2] = gz[2];
    e[3] = gz[1] + gy[2];
    e[4] = gz[0] + gx[2];
    e[5] = gy[0] + gx[1];
}

template <int H>
__global__ __launch_bounds__(64) void k_zone(ZoneArgs a)
{
    constexpr int N = 2 * H + 1, NN = 2 * H + 2;
    constexpr int NV = N * N * N, NNODE = NN * NN * NN;
    constexpr int VPL = (NV + 63) / 64, NPL = (NNODE + 63) / 64;
    constexpr int CENTRE = H + N * (H + N * H);

    __shared__ float4 s_du[NNODE];
    __shared__ float4 s_sig[NV][2];

    const int lane = threadIdx.x;
    const uint32_t count = *a.count;

    for (uint32_t e = (uint32_t)stride_block((int)blockIdx.x, (int)gridDim.x, a.order); e < count; e += gridDim.x) {
        const TrialEntry ent = a.list[e];
        const TrialCtx tc = trial_ctx(a, ent.qr);
        const int K = tc.K;
        const int px = (int)(ent.site % (uint32_t)K);
        const int py = (int)((ent.site / (uint32_t)K) % (uint32_t)K);
        const int pz = (int)(ent.site / ((uint32_t)K * (uint32_t)K));
        const int q_old = tc.spins[ent.site];
        const int q_new = (int)(ent.qr & 0xffffu);

        // centre: eps_p = S_old sigma_p, t = (C_new - C_old) eps_p
        float sp[6], eps[6], t[6];
        {
            float c[21], s[6];
#pragma unroll
            for (int I = 0; I < 6; ++I) sp[I] = a.sigma[(int64_t)I * a.plane + tc.site_off + ent.site];
            load_sym(tc.Stab + (int64_t)q_old * kTab, c);
            symv(c, sp, eps);
            load_sym(tc.Ctab + (int64_t)q_new * kTab, c);
            symv(c, eps, t);
            load_sym(tc.Ctab + (int64_t)q_old * kTab, c);
            symv(c, eps, s);
#pragma unroll
            for (int I = 0; I < 6; ++I) t[I] -= s[I];
        }

        // owned voxels: stiffness in registers
        float Cv[VPL][21];
#pragma unroll
        for (int m = 0; m < VPL; ++m) {
            const int v = lane + 64 * m;
            if (v < NV) {
                const int i = v % N, j = (v / N) % N, k = v / (N * N);
                int g;
                if (v == CENTRE) {
                    g = q_new;
                } else {
                    int gx = px + i - H, gy = py + j - H, gz = pz + k - H;
                    gx = (gx % K + K) % K;
                    gy = (gy % K + K) % K;
                    gz = (gz % K + K) % K;
                    g = tc.spins[gx + K * (gy + K * gz)];
                }
                load_sym(tc.Ctab + (int64_t)g * kTab, Cv[m]);
            }
        }

        // owned nodes: displacement and velocity from rest
        float du[NPL][3], w[NPL][3];
#pragma unroll
        for (int m = 0; m < NPL; ++m) {
            du[m][0] = du[m][1] = du[m][2] = 0.f;
            w[m][0] = w[m][1] = w[m][2] = 0.f;
            const int n = lane + 64 * m;
            if (n < NNODE) s_du[n] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        __syncthreads();

        for (int step = 0; step < a.nr; ++step) {
            // phase A: voxel stresses
#pragma unroll
            for (int m = 0; m < VPL; ++m) {
                const int v = lane + 64 * m;
                if (v < NV) {
                    const int i = v % N, j = (v / N) % N, k = v / (N * N);
                    const int n0 = i + NN * (j + NN * k);
                    float4 u[8];
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        u[c] = s_du[n0 + (c & 1) + NN * (((c >> 1) & 1) + NN * (c >> 2))];
                    float ev[6], sv[6];
                    corner_strain(u, ev);
                    symv(Cv[m], ev, sv);
                    if (v == CENTRE) {
#pragma unroll
                        for (int I = 0; I < 6; ++I) sv[I] += t[I];
                    }
                    s_sig[v][0] = make_float4(sv[0], sv[1], sv[2], sv[3]);
                    s_sig[v][1] = make_float4(sv[4], sv[5], 0.f, 0.f);
                }
            }
            __syncthreads();
            // phase B: node forces and heavy-ball step
#pragma unroll
            for (int m = 0; m < NPL; ++m) {
                const int n = lane + 64 * m;
                if (n < NNODE) {
                    const int na = n % NN, nb = (n / NN) % NN, nc = n / (NN * NN);
                    float fx = 0.f, fy = 0.f, fz = 0.f;
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int ca = c & 1, cb = (c >> 1) & 1, cc = c >> 2;
                        const int vi = na - ca, vj = nb - cb, vk = nc - cc;
                        if (vi >= 0 && vi < N && vj >= 0 && vj < N && vk >= 0 && vk < N) {
                            const int v = vi + N * (vj + N * vk);
                            const float4 s0 = s_sig[v][0], s1 = s_sig[v][1];
                            const float sx = ca ? 0.25f : -0.25f, sy = cb ? 0.25f : -0.25f,
                                        sz = cc ? 0.25f : -0.25f;
                            fx += sx * s0.x + sy * s1.y + sz * s1.x;
                            fy += sx * s1.y + sy * s0.y + sz * s0.w;
                            fz += sx * s1.x + sy * s0.w + sz * s0.z;
                        }
                    }
                    w[m][0] = a.beta * w[m][0] - a.alpha * fx;
                    w[m][1] = a.beta * w[m][1] - a.alpha * fy;
                    w[m][2] = a.beta * w[m][2] - a.alpha * fz;
                    du[m][0] += w[m][0];
                    du[m][1] += w[m][1];
                    du[m][2] += w[m][2];
                    s_du[n] = make_float4(du[m][0], du[m][1], du[m][2], 0.f);
                }
            }
            __syncthreads();
        }

        // energy at the final displacement
        double part = 0.0;
#pragma unroll
        for (int m = 0; m < VPL; ++m) {
            const int v = lane + 64 * m;
            if (v < NV) {
                const int i = v % N, j = (v / N) % N, k = v / (N * N);
                const int n0 = i + NN * (j + NN * k);
                float4 u[8];
#pragma unroll
                for (int c = 0; c < 8; ++c) u[c] = s_du[n0 + (c & 1) + NN * (((c >> 1) & 1) + NN * (c >> 2))];
                float ev[6], sv[6];
                corner_strain(u, ev);
                symv(Cv[m], ev, sv);
                double d = 0.0;
#pragma unroll
                for (int I = 0; I < 6; ++I) d += 0.5 * (double)ev[I] * (double)sv[I];
                if (v == CENTRE) {
#pragma unroll
                    for (int I = 0; I < 6; ++I) d += (double)t[I] * (double)ev[I];
                }
                part += d;
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);

        if (lane == 0) {
            double base = 0.0;
#pragma unroll
            for (int I = 0; I < 6; ++I) base += 0.5 * (double)eps[I] * (double)t[I];
            const double dPi = base + part;
            if (!isfinite(dPi)) atomicOr(a.nonfinite, (uint32_t)kNfZone);
            const double dE = tc.J * (double)ent.gb + tc.lambda * dPi;
            const bool accept = (dE <= 0.0) || ((double)ent.r1 < ldexp(exp(-dE / tc.kT), 32));
            a.acc[e] = accept ? 1 : 0;
            if (a.rec) {
                a.rec[tc.site_off + ent.site].dPi = (float)dPi;
                a.rec[tc.site_off + ent.site].flags = 1 | 4 | (accept ? 2 : 0);
            }
            atomicAdd(&a.stats[stat_copy(blockIdx.x) + kStatSolves], 1ull);
            if (accept) atomicAdd(&a.stats[stat_copy(blockIdx.x) + kStatAccepted], 1ull);
        }
        __syncthreads();   // LDS is reused by the next trial
    }
}


// ------------------------------------------------------------------------------------
// Column variant.  A work-group of 256 lanes holds Z = 256 / (2h+2)^2 trials at once.
// Within a trial, lane (cx, cy) owns the z-column of (2h+2) nodes at (cx, cy) and, when
// cx, cy < 2h+1, the z-column of (2h+1) voxels whose lowest corner column it is.  The
// strain of a voxel needs the node columns (cx, cy), (cx+1, cy), (cx, cy+1), (cx+1, cy+1):
// per node layer the lane forms the x-difference, y-difference and sum of those four
// nodes, and two consecutive layers give the voxel's nine displacement gradients (all
// with the factor 1/4 left out).  The corner forces are the transpose: per node layer the
// lane sums its voxels' stress rows over the two voxels sharing the layer and splits the
// result into its four node columns; its own column stays in registers, the other three
// go through LDS to their owners.  Two barriers per step: after the displacements are
// published and after the forces are.
//
// Scaling: with B = B'/4, sigma'' = C (B' du) + 4 t = 4 (C B du + t) and the true
// gradient is B'^T sigma'' / 16, so the step uses alpha / 16.
// ------------------------------------------------------------------------------------
template <int H>
__global__ __launch_bounds__(256, 2) void k_zone_col(ZoneArgs a)
{
    constexpr int N = 2 * H + 1, NN = 2 * H + 2, NC = NN * NN;
    constexpr int Z = 256 / NC;
    static_assert(Z >= 1, "zone too large for one work-group");

    __shared__ float s_u[Z][3][NN][NC];          // node displacements
    __shared__ float s_f[3][Z][3][NN][NC];       // force contributions: from (x-1,y), (x,y-1), (x-1,y-1)
    __shared__ double s_red[256];
    __shared__ float s_ctr[Z][12];               // per trial: eps_p[6], t[6]

    const int t = threadIdx.x;
    const int zs = t / NC;
    const int col = t - zs * NC;
    const int cx = col % NN, cy = col / NN;
    const bool in_zone = zs < Z;
    const bool vox = in_zone && cx < N && cy < N;
    const bool centre_col = vox && cx == H && cy == H;
    const int zsafe = in_zone ? zs : 0;
    const uint32_t count = *a.count;
    const float alpha16 = a.alpha * 0.0625f, beta = a.beta;

    for (uint32_t base = (uint32_t)stride_block((int)blockIdx.x, (int)gridDim.x, a.order) * (uint32_t)Z; base < count;
         base += gridDim.x * (uint32_t)Z) {
        const uint32_t e = base + (uint32_t)zsafe;
        const bool active = in_zone && e < count;

        TrialEntry ent{0u, 0u, 0, 0u};
        TrialCtx tc{};
        float Cv[N][21];
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
            for (int i = 0; i < 21; ++i) Cv[k][i] = 0.f;
        if (active) {
            ent = a.list[e];
            tc = trial_ctx(a, ent.qr);
            const int K = tc.K;
            const int q_new = (int)(ent.qr & 0xffffu);
            const int px = (int)(ent.site % (uint32_t)K);
            const int py = (int)((ent.site / (uint32_t)K) % (uint32_t)K);
            const int pz = (int)(ent.site / ((uint32_t)K * (uint32_t)K));
            if (col == 0) {
                // eps_p = S_old sigma_p, t = (C_new - C_old) eps_p, shared through LDS
                const int q_old = tc.spins[ent.site];
                float c[21], sp[6], s[6], eps[6], tt[6];
#pragma unroll
                for (int I = 0; I < 6; ++I) sp[I] = a.sigma[(int64_t)I * a.plane + tc.site_off + ent.site];
                load_sym(tc.Stab + (int64_t)q_old * kTab, c);
                symv(c, sp, eps);
                load_sym(tc.Ctab + (int64_t)q_new * kTab, c);
                symv(c, eps, tt);
                load_sym(tc.Ctab + (int64_t)q_old * kTab, c);
                symv(c, eps, s);
#pragma unroll
                for (int I = 0; I < 6; ++I) {
                    s_ctr[zs][I] = eps[I];
                    s_ctr[zs][6 + I] = tt[I] - s[I];
                }
            }
            if (vox) {
                const int gx = ((px + cx - H) % K + K) % K, gy = ((py + cy - H) % K + K) % K;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const int gz = ((pz + k - H) % K + K) % K;
                    const int g = (centre_col && k == H) ? q_new : (int)tc.spins[gx + K * (gy + K * gz)];
                    load_sym(tc.Ctab + (int64_t)g * kTab, Cv[k]);
                }
            }
        }
        float du[NN][3], w[NN][3];
#pragma unroll
        for (int z = 0; z < NN; ++z)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                du[z][j] = 0.f;
                w[z][j] = 0.f;
                if (in_zone) {
                    s_u[zs][j][z][col] = 0.f;
                    s_f[0][zs][j][z][col] = 0.f;
                    s_f[1][zs][j][z][col] = 0.f;
                    s_f[2][zs][j][z][col] = 0.f;
                }
            }
        __syncthreads();

        const int cE = col + 1, cN = col + NN, cNE = col + NN + 1;
        for (int step = 0; step < a.nr; ++step) {
            // ---- voxels: strain, stress, corner forces ----
            float fo[NN][3];
            if (vox && active) {
                float Lp[3][3];     // previous node layer: (dx, dy, sum) x comp
                float Pp[3] = {0.f, 0.f, 0.f}, Qp[3] = {0.f, 0.f, 0.f}, Rp[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int z = 0; z < NN; ++z) {
                    float Lc[3][3];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const float ua = du[z][j];
                        const float ub = s_u[zs][j][z][cE];
                        const float uc = s_u[zs][j][z][cN];
                        const float ud = s_u[zs][j][z][cNE];
                        const float s1 = ua + ub, s2 = uc + ud, d1 = ub - ua, d2 = ud - uc;
                        Lc[0][j] = d1 + d2;   // x-difference
                        Lc[1][j] = s2 - s1;   // y-difference
                        Lc[2][j] = s1 + s2;   // sum
                    }
                    float P[3] = {0.f, 0.f, 0.f}, Q[3] = {0.f, 0.f, 0.f}, R[3] = {0.f, 0.f, 0.f};
                    if (z >= 1) {
                        const int k = z - 1;   // voxel between layers z-1 and z
                        float g[3][3];
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            g[j][0] = Lp[0][j] + Lc[0][j];
                            g[j][1] = Lp[1][j] + Lc[1][j];
                            g[j][2] = Lc[2][j] - Lp[2][j];
                        }
                        const float ev[6] = {g[0][0], g[1][1], g[2][2], g[1][2] + g[2][1], g[0][2] + g[2][0],
                                             g[0][1] + g[1][0]};
                        float sv[6];
                        symv(Cv[k], ev, sv);
                        if (centre_col && k == H) {
#pragma unroll
                            for (int I = 0; I < 6; ++I) sv[I] += 4.f * s_ctr[zs][6 + I];
                        }
                        P[0] = sv[0]; P[1] = sv[5]; P[2] = sv[4];
                        Q[0] = sv[5]; Q[1] = sv[1]; Q[2] = sv[3];
                        R[0] = sv[4]; R[1] = sv[3]; R[2] = sv[2];
                        // node layer k collects voxel k-1 (its upper corners) and voxel k (lower)
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            const float PL = Pp[j] + P[j], QL = Qp[j] + Q[j], RL = Rp[j] - R[j];
                            const float U = QL + RL, V = RL - QL;
                            fo[k][j] = V - PL;
                            s_f[0][zs][j][k][cE] = PL + V;
                            s_f[1][zs][j][k][cN] = U - PL;
                            s_f[2][zs][j][k][cNE] = PL + U;
                            Pp[j] = P[j];
                            Qp[j] = Q[j];
                            Rp[j] = R[j];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < 3; ++j)
#pragma unroll
                        for (int r = 0; r < 3; ++r) Lp[r][j] = Lc[r][j];
                }
                // top node layer: only voxel N-1 below it
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const float PL = Pp[j], QL = Qp[j], RL = Rp[j];
                    const float U = QL + RL, V = RL - QL;
                    fo[NN - 1][j] = V - PL;
                    s_f[0][zs][j][NN - 1][cE] = PL + V;
                    s_f[1][zs][j][NN - 1][cN] = U - PL;
                    s_f[2][zs][j][NN - 1][cNE] = PL + U;
                }
            } else {
#pragma unroll
                for (int z = 0; z < NN; ++z)
#pragma unroll
                    for (int j = 0; j < 3; ++j) fo[z][j] = 0.f;
            }
            __syncthreads();
            // ---- nodes: gather forces, heavy-ball step, publish displacement ----
            if (active) {
#pragma unroll
                for (int z = 0; z < NN; ++z)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const float f = ((fo[z][j] + s_f[0][zs][j][z][col]) + s_f[1][zs][j][z][col]) +
                                        s_f[2][zs][j][z][col];
                        w[z][j] = beta * w[z][j] - alpha16 * f;
                        du[z][j] += w[z][j];
                        s_u[zs][j][z][col] = du[z][j];
                    }
            }
            __syncthreads();
        }

        // ---- energy at the final displacement: 1/2 e.C e over the zone + t.e at the centre ----
        double part = 0.0;
        if (vox && active) {
            float Lp[3][3];
#pragma unroll
            for (int z = 0; z < NN; ++z) {
                float Lc[3][3];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const float ua = du[z][j];
                    const float ub = s_u[zs][j][z][cE];
                    const float uc = s_u[zs][j][z][cN];
                    const float ud = s_u[zs][j][z][cNE];
                    const float s1 = ua + ub, s2 = uc + ud, d1 = ub - ua, d2 = ud - uc;
                    Lc[0][j] = d1 + d2;
                    Lc[1][j] = s2 - s1;
                    Lc[2][j] = s1 + s2;
                }
                if (z >= 1) {
                    const int k = z - 1;
                    float g[3][3];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        g[j][0] = 0.25f * (Lp[0][j] + Lc[0][j]);
                        g[j][1] = 0.25f * (Lp[1][j] + Lc[1][j]);
                        g[j][2] = 0.25f * (Lc[2][j] - Lp[2][j]);
                    }
                    const float ev[6] = {g[0][0], g[1][1], g[2][2], g[1][2] + g[2][1], g[0][2] + g[2][0],
                                         g[0][1] + g[1][0]};
                    float sv[6];
                    symv(Cv[k], ev, sv);
                    double d = 0.0;
#pragma unroll
                    for (int I = 0; I < 6; ++I) d += 0.5 * (double)ev[I] * (double)sv[I];
                    if (centre_col && k == H) {
#pragma unroll
                        for (int I = 0; I < 6; ++I) d += (double)s_ctr[zs][6 + I] * (double)ev[I];
                    }
                    part += d;
                }
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int r = 0; r < 3; ++r) Lp[r][j] = Lc[r][j];
            }
        }
        s_red[t] = part;
        __syncthreads();
        if (active && col == 0) {
            double sum = 0.0;
            for (int i = 0; i < NC; ++i) sum += s_red[zs * NC + i];
            double base_e = 0.0;
#pragma unroll
            for (int I = 0; I < 6; ++I) base_e += 0.5 * (double)s_ctr[zs][I] * (double)s_ctr[zs][6 + I];
            const double dPi = base_e + sum;
            if (!isfinite(dPi)) atomicOr(a.nonfinite, (uint32_t)kNfZone);
            const double dE = tc.J * (double)ent.gb + tc.lambda * dPi;
            const bool accept = (dE <= 0.0) || ((double)ent.r1 < ldexp(exp(-dE / tc.kT), 32));
            a.acc[e] = accept ? 1 : 0;
            if (a.rec) {
                a.rec[tc.site_off + ent.site].dPi = (float)dPi;
                a.rec[tc.site_off + ent.site].flags = 1 | 4 | (accept ? 2 : 0);
            }
            atomicAdd(&a.stats[stat_copy(blockIdx.x) + kStatSolves], 1ull);
            if (accept) atomicAdd(&a.stats[stat_copy(blockIdx.x) + kStatAccepted], 1ull);
        }
        __syncthreads();   // LDS is reused by the next group of trials
    }
}

// ------------------------------------------------------------------------------------
// Lane-shift variant (1 <= h <= 3).  Each trial occupies LT = (2h+2)(2h+1) consecutive lanes
// (12, 30 and 56) of one wavefront, laid out as lane l = x + (2h+2) y over node columns x in [0, 2h+2),
// y in [0, 2h+1); a wavefront holds 64 / LT trials and never splits one.  Lane (x, y) owns
// node column (x, y) in registers and, for x < 2h+1, the voxel column (x, y); the top row
// of node columns (y = 2h+1) is split into (column, component) items held by the trial's
// first 3(2h+2) lanes, their displacements in LDS.
//
// Neighbours in x are the next lane, so they move through the wavefront with DPP shifts
// (no LDS):  the +x node column's displacement, the +x+y column's (the +x lane's +y
// read), the force a voxel sends to its +x node column, and the force it sends to its
// +x+y column, which the receiving lane folds into its own +y force.  Only the +y
// exchange goes through LDS: one read and one write per node and component per phase, at
// lane-consecutive addresses, with the trials of a wavefront placed 30 (mod 64) floats
// apart for h = 2 (12 for h = 1) so that no access has a bank conflict.  Lanes with
// x = 2h+1 and lanes beyond the last trial of a wavefront carry zero stiffness, so they
// run the same instructions and produce zero forces; the control flow is uniform across
// the work-group, which the cross-lane moves need.  A work-group is one wavefront, so its
// barriers never wait for another wavefront.  Stiffnesses are pre-scaled by
// -alpha/16 (see the column variant for the 1/16), so a stress evaluation
// yields the step's force directly and the heavy-ball update is w <- beta w + f; the final
// energy undoes the scale in FP64.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ float from_next_lane(float v)   // lane i receives lane i+1's v (0 at the end)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}

__device__ __forceinline__ float from_prev_lane(float v)   // lane i receives lane i-1's v (0 at lane 0)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}

// Corner forces of one node layer: the transpose of the strain pipeline.  L0, L1, L2 are
// the layer's weights on its x-difference, y-difference and sum (PL, QL, RL: the stress rows
// of the voxels below and above, summed or differenced).  Since the layer's x-difference and
// sum combine A = u(x,y) + u(x,y+1) of this lane and the next, and its y-difference
// D = u(x,y+1) - u(x,y) of both, A's weight is (L2 - L0) here plus (L2 + L0) of lane l-1 and
// D's weight is L1 here plus L1 of lane l-1.  The own node gets A^ - D^, the +y node A^ + D^
// (through LDS).
__device__ __forceinline__ void node_forces(float L0, float L1, float L2, float beta, float& w, float& ny)
{
    const float Ab = (L2 - L0) + from_prev_lane(L2 + L0);
    const float Db = L1 + from_prev_lane(L1);
    w = beta * w + (Ab - Db);
    ny = Ab + Db;
}

template <int H, int WAVES = 1>
struct LaneShiftShape {
    static constexpr int N = 2 * H + 1, NN = N + 1;
    static constexpr int LT = NN * N;                   // lanes per trial
    static constexpr int TW = 64 / LT;                  // trials per wavefront
    static constexpr int THREADS = 64 * WAVES;          // wavefronts per work-group
    static constexpr int Z = TW * WAVES;                // trials per work-group
    static constexpr int ROW = NN * NN;                 // floats per (component, layer) row
    static constexpr int BODY = 3 * NN * ROW;
    // block stride: >= BODY + NN (zero gap), and = LT (mod 64) for conflict-free addressing
    static constexpr int TB = BODY + NN + ((LT - (BODY + NN) % 64) % 64 + 64) % 64;
    static constexpr int PAD = 8;                       // leading zeros of the force array
};

// Wavefronts per SIMD, measured on the 128^3 workload: h = 1 (3^3 x 50 steps) runs 3 with a
// few registers spilled, 0.357 against 0.418 ms per colour launch at 2; h = 2 runs 2 (3 spill
// 131 registers and take 9.6 against 5.7 ms); h = 3 (7 x 21 stiffness registers per lane)
// spills some 34 registers at 2 and still beats 1 without spills (36.9 against 44.2 ms).
// WAVES wavefronts per work-group (1 by default; 2 and 4 are shapes for the autotuner): each
// wavefront holds its own trials, the work-group shares its barriers.
template <int H, int WAVES>
__global__ __launch_bounds__(64 * WAVES, H == 1 ? 3 : 2) void k_zone_lane(ZoneArgs a)
{
    using S = LaneShiftShape<H, WAVES>;
    constexpr int N = S::N, NN = S::NN, LT = S::LT, TW = S::TW, Z = S::Z, ROW = S::ROW, TB = S::TB;
    static_assert(H >= 1 && H <= 3 && TW >= 1 && 3 * NN <= LT, "lane-shift variant needs 1 <= h <= 3");
    static_assert(TB % 64 == LT % 64 && TB >= S::BODY + NN, "block stride");

    // blocks 0..Z-1 belong to trials, block Z to lanes outside every trial
    __shared__ float s_u[(Z + 1) * TB];                   // node displacements
    __shared__ __align__(16) float s_n[S::PAD + (Z + 1) * TB];   // forces sent to the +y neighbour
    __shared__ float s_ctr[Z][18];                        // eps_p[6], t[6], -alpha/4 t[6]
    static_assert(sizeof(s_n) >= S::THREADS * sizeof(double), "energy scratch does not fit");
    double* s_red = reinterpret_cast<double*>(s_n);

    const int t = threadIdx.x;
    const int wave = t >> 6, li = t & 63;
    const int slot = li / LT;
    const bool member = slot < TW;
    const int l = member ? li - slot * LT : li - TW * LT;
    const int zs = member ? wave * TW + slot : Z;
    const int x = l % NN, y = l / NN;
    const bool vox = member && x < N;
    const bool centre_col = vox && x == H && y == H;
    const uint32_t count = *a.count;
    const float alpha16 = a.alpha * 0.0625f, beta = a.beta;

    float* const ub = s_u + zs * TB;                      // this lane's trial block
    float* const nbk = s_n + S::PAD + zs * TB;
    // top-row item: node column (l % NN, N), component l / NN, for the first 3 NN lanes
    const bool xon = member && l < 3 * NN;
    const int xcol = l % NN + NN * N, xj = xon ? l / NN : 0;

    // solves and acceptances are counted per lane and added to the statistics once per
    // work-group at the end (same-address atomics per trial would serialise in L2)
    uint32_t n_solved = 0, n_accepted = 0;
    for (uint32_t base = (uint32_t)stride_block((int)blockIdx.x, (int)gridDim.x, a.order) * (uint32_t)Z; base < count;
         base += gridDim.x * (uint32_t)Z) {
        const uint32_t e = base + (uint32_t)(member ? zs : 0);
        const bool active = member && e < count;

        float Cv[N][21];
#pragma unroll
        for (int k = 0; k < N; ++k)
#pragma unroll
            for (int i = 0; i < 21; ++i) Cv[k][i] = 0.f;
        if (active) {
            const TrialEntry ent = a.list[e];
            const TrialCtx tc = trial_ctx(a, ent.qr);
            const int K = tc.K;
            const int q_new = (int)(ent.qr & 0xffffu);
            const int px = (int)(ent.site % (uint32_t)K);
            const int py = (int)((ent.site / (uint32_t)K) % (uint32_t)K);
            const int pz = (int)(ent.site / ((uint32_t)K * (uint32_t)K));
            if (l == 0) {
                const int q_old = tc.spins[ent.site];
                float c[21], sp[6], s[6], eps[6], tt[6];
#pragma unroll
                for (int I = 0; I < 6; ++I) sp[I] = a.sigma[(int64_t)I * a.plane + tc.site_off + ent.site];
                load_sym(tc.Stab + (int64_t)q_old * kTab, c);
                symv(c, sp, eps);
                load_sym(tc.Ctab + (int64_t)q_new * kTab, c);
                symv(c, eps, tt);
                load_sym(tc.Ctab + (int64_t)q_old * kTab, c);
                symv(c, eps, s);
#pragma unroll
                for (int I = 0; I < 6; ++I) {
                    const float ti = tt[I] - s[I];
                    s_ctr[zs][I] = eps[I];
                    s_ctr[zs][6 + I] = ti;
                    s_ctr[zs][12 + I] = (-4.f * alpha16) * ti;
                }
            }
            if (vox) {
                const int gx = ((px + x - H) % K + K) % K, gy = ((py + y - H) % K + K) % K;
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    const int gz = ((pz + k - H) % K + K) % K;
                    const int g = (centre_col && k == H) ? q_new : (int)tc.spins[gx + K * (gy + K * gz)];
                    load_sym(tc.Ctab + (int64_t)g * kTab, Cv[k]);
#pragma unroll
                    for (int i = 0; i < 21; ++i) Cv[k][i] *= -alpha16;
                }
            }
        }
        for (int i = t; i < (Z + 1) * TB; i += S::THREADS) s_u[i] = 0.f;
        for (int i = t; i < S::PAD + (Z + 1) * TB; i += S::THREADS) s_n[i] = 0.f;
        __syncthreads();
        float ts[6];
#pragma unroll
        for (int I = 0; I < 6; ++I) ts[I] = (active && centre_col) ? s_ctr[zs][12 + I] : 0.f;

        float du[NN][3], w[NN][3], xw[NN];
#pragma unroll
        for (int z = 0; z < NN; ++z) {
            xw[z] = 0.f;
#pragma unroll
            for (int j = 0; j < 3; ++j) du[z][j] = w[z][j] = 0.f;
        }

        for (int step = 0; step < a.nr; ++step) {
            // ---- voxels: strain, (scaled) stress, corner forces ----
            {
                float cn[3], cnn[3];
#pragma unroll
                for (int j = 0; j < 3; ++j) cn[j] = ub[(j * NN + 0) * ROW + l + NN];
                float Lp[3][3], Pp[3], Qp[3], Rp[3];
#pragma unroll
                for (int z = 0; z < NN; ++z) {
                    if (z + 1 < NN) {
#pragma unroll
                        for (int j = 0; j < 3; ++j) cnn[j] = ub[(j * NN + z + 1) * ROW + l + NN];
                    }
                    // with A = u(x,y) + u(x,y+1) and D = u(x,y+1) - u(x,y), the +x lane's A and D
                    // complete the four-column x-difference, y-difference and sum
                    float Lc[3][3];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const float A = du[z][j] + cn[j], D = cn[j] - du[z][j];
                        Lc[0][j] = from_next_lane(A) - A;
                        Lc[1][j] = D + from_next_lane(D);
                        Lc[2][j] = A + from_next_lane(A);
                    }
                    if (z >= 1) {
                        const int k = z - 1;
                        float g[3][3];
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            g[j][0] = Lp[0][j] + Lc[0][j];
                            g[j][1] = Lp[1][j] + Lc[1][j];
                            g[j][2] = Lc[2][j] - Lp[2][j];
                        }
                        const float ev[6] = {g[0][0], g[1][1], g[2][2], g[1][2] + g[2][1], g[0][2] + g[2][0],
                                             g[0][1] + g[1][0]};
                        float sv[6];
                        symv(Cv[k], ev, sv);
                        if (k == H) {
#pragma unroll
                            for (int I = 0; I < 6; ++I) sv[I] += ts[I];
                        }
                        const float P[3] = {sv[0], sv[5], sv[4]};
                        const float Q[3] = {sv[5], sv[1], sv[3]};
                        const float R[3] = {sv[4], sv[3], sv[2]};
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            const float PL = k == 0 ? P[j] : Pp[j] + P[j];
                            const float QL = k == 0 ? Q[j] : Qp[j] + Q[j];
                            const float RL = k == 0 ? -R[j] : Rp[j] - R[j];
                            node_forces(PL, QL, RL, beta, w[k][j], nbk[(j * NN + k) * ROW + l]);
                            Pp[j] = P[j];
                            Qp[j] = Q[j];
                            Rp[j] = R[j];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        cn[j] = cnn[j];
#pragma unroll
                        for (int r = 0; r < 3; ++r) Lp[r][j] = Lc[r][j];
                    }
                }
                // top node layer: only voxel N-1 below it
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    node_forces(Pp[j], Qp[j], Rp[j], beta, w[NN - 1][j],
                                nbk[(j * NN + NN - 1) * ROW + l]);
            }
            __syncthreads();
            // ---- nodes: add the force from the -y neighbour, step, publish ----
#pragma unroll
            for (int z = 0; z < NN; ++z)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    w[z][j] += nbk[(j * NN + z) * ROW + l - NN];
                    du[z][j] += w[z][j];
                    ub[(j * NN + z) * ROW + l] = du[z][j];
                }
            if (xon) {
#pragma unroll
                for (int z = 0; z < NN; ++z) {
                    xw[z] = beta * xw[z] + nbk[(xj * NN + z) * ROW + xcol - NN];
                    ub[(xj * NN + z) * ROW + xcol] += xw[z];
                }
            }
            __syncthreads();
        }

        // ---- energy at the final displacement: 1/2 e.C e over the zone + t.e at the centre ----
        double quad = 0.0, lin = 0.0;
        {
            float Lp[3][3];
#pragma unroll
            for (int z = 0; z < NN; ++z) {
                float Lc[3][3];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const float uc = ub[(j * NN + z) * ROW + l + NN];
                    const float A = du[z][j] + uc, D = uc - du[z][j];
                    Lc[0][j] = from_next_lane(A) - A;
                    Lc[1][j] = D + from_next_lane(D);
                    Lc[2][j] = A + from_next_lane(A);
                }
                if (z >= 1) {
                    const int k = z - 1;
                    float g[3][3];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        g[j][0] = 0.25f * (Lp[0][j] + Lc[0][j]);
                        g[j][1] = 0.25f * (Lp[1][j] + Lc[1][j]);
                        g[j][2] = 0.25f * (Lc[2][j] - Lp[2][j]);
                    }
                    const float ev[6] = {g[0][0], g[1][1], g[2][2], g[1][2] + g[2][1], g[0][2] + g[2][0],
                                         g[0][1] + g[1][0]};
                    float sv[6];
                    symv(Cv[k], ev, sv);
#pragma unroll
                    for (int I = 0; I < 6; ++I) quad += (double)ev[I] * (double)sv[I];
                    if (k == H && centre_col) {
#pragma unroll
                        for (int I = 0; I < 6; ++I) lin += (double)s_ctr[zs][6 + I] * (double)ev[I];
                    }
                }
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int r = 0; r < 3; ++r) Lp[r][j] = Lc[r][j];
            }
        }
        const double part = vox ? quad * (-0.5 / (double)alpha16) + lin : 0.0;
        __syncthreads();   // the force array becomes the reduction scratch
        s_red[t] = part;
        __syncthreads();
        if (active && l == 0) {
            const TrialEntry ent = a.list[e];
            const TrialCtx tc = trial_ctx(a, ent.qr);
            double sum = 0.0;
            for (int i = 0; i < LT; ++i) sum += s_red[t + i];
            double base_e = 0.0;
#pragma unroll
            for (int I = 0; I < 6; ++I) base_e += 0.5 * (double)s_ctr[zs][I] * (double)s_ctr[zs][6 + I];
            const double dPi = base_e + sum;
            if (!isfinite(dPi)) atomicOr(a.nonfinite, (uint32_t)kNfZone);
            const double dE = tc.J * (double)ent.gb + tc.lambda * dPi;
            const bool accept = (dE <= 0.0) || ((double)ent.r1 < ldexp(exp(-dE / tc.kT), 32));
            a.acc[e] = accept ? 1 : 0;
            if (a.rec) {
                a.rec[tc.site_off + ent.site].dPi = (float)dPi;
                a.rec[tc.site_off + ent.site].flags = 1 | 4 | (accept ? 2 : 0);
            }
            n_solved += 1;
            n_accepted += accept ? 1 : 0;
        }
        __syncthreads();   // LDS is reused by the next group of trials
    }
    // sum the lane counts across each wavefront; one atomic per wavefront
    for (int off = 32; off > 0; off >>= 1) {
        n_solved += __shfl_xor(n_solved, off);
        n_accepted += __shfl_xor(n_accepted, off);
    }
    if (li == 0 && n_solved) {
        atomicAdd(&a.stats[stat_copy(blockIdx.x) + kStatSolves], (unsigned long long)n_solved);
        if (n_accepted) atomicAdd(&a.stats[stat_copy(blockIdx.x) + kStatAccepted], (unsigned long long)n_accepted);
    }
}

// Launch k_zone_lane<2, waves> and k_zone_lane<3, waves> for waves = 1, 2 or 4 (else
// hipErrorInvalidValue) on the stream; a launch error stays pending for hipGetLastError.  The
// instances of the 5^3 and 7^3 zones live in translation units of their own so that the build
// can give each its own scheduling options.
hipError_t launch_zone_lane_h2(int waves, dim3 grid, dim3 block, hipStream_t stream, const ZoneArgs& a);
hipError_t launch_zone_lane_h3(int waves, dim3 grid, dim3 block, hipStream_t stream, const ZoneArgs& a);

}  // namespace hmc
