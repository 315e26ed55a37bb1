// hmc_mp8.hip -- the global quasi-static solve with 2 x 2 x 2 material points per background
// cell (the arrangement of the paper's MPM, Appendix: a fixed number of particles per cell, two
// per direction), a variant of the one-point-per-voxel default of hmc_elastic.hip.
//
// The mesh has (K/2)^3 periodic nodes at the corners of cells of 2 x 2 x 2 sites.  Every site is
// a material point with its own stiffness at local coordinates +-1/2 of its cell; its strain is
// the gradient of the trilinear interpolation of the cell's 8 corner displacements there (the
// cell edge is 2 sites, so d/dx = d/dxi), its nodal forces the transpose.  The relaxation is the
// default's: average-stress control of the macroscopic strain E, heavy-ball steps
//   w <- beta w + alpha r,  u <- u + w,   wE <- beta wE + alphaE (Sigma - <sigma>),  E <- E + wE,
// with the Reuss start and the warm start of the default.  Stable for alpha below the Polyak
// value of L = 8 x the largest Mandel eigenvalue of the stiffness (the identity material's
// Hessian peaks at 8 here, against 4 for one point per voxel).
//
// One step is three launches on the context's stream: a cell pass (one thread per cell: gather
// the 8 corner displacements, their differences along the cell's 12 edges, the 8 points'
// strains as bilinear interpolations of those and their stresses, the transpose back onto the
// edges and the cell's 24 corner forces written to a cell-major force array, and per-block
// sums of the point stresses), a node pass
// (one thread per node: the forces of its 8 cells, the heavy-ball update of u and w in place)
// and a fold of the stress sums into E (one block per replica); each launch covers every replica
// of a batch.  A replica's node fields occupy the first (K/2)^3 entries of its slice of each
// displacement plane; its corner forces use its slice of the second displacement buffer, which
// holds exactly 24 floats per cell.
#include <algorithm>

#include "hmc_device.h"

namespace hmc {

namespace {

// Weight of the edge at bit b (0 or 1) of a cell direction for the point at sub-position p
// there: the trilinear shape functions' factor 1 +- xi_p with xi_p = +-1/2.
__host__ __device__ constexpr float mp_w(int b, int p) { return b == p ? 1.5f : 0.5f; }

// Work-groups per replica of the cell and node passes: one per 256 cells, at most 4096 (the
// passes stride beyond).  The same count alone and in a batch, so each replica's partial sums
// are the same numbers in the same order either way.
__host__ __device__ inline int mp8_blocks(int K)
{
    const int64_t Kc = K / 2, nc = Kc * Kc * Kc;
    const int64_t b = (nc + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// All replicas in one launch: work-group (x, y) is block x of replica y; blocks beyond the
// replica's count return at once.  A replica's partial sums go to its own node-block slots
// (RepDev::node_first onwards, never fewer than its cell-pass blocks).
struct Mp8Args {
    const int16_t* spins;
    const float* Ctab;
    const float* u;        // 3 planes of `plane` floats; a replica's nodes first in its slice
    float* F;              // corner forces: row k of a replica's cells at plane k / 8, offset
                           // (k % 8) n_cells of its slice (3 planes of `plane`)
    float* sigma;          // final pass: 6 planes of point stresses (or null)
    double* partials;
    const double* state;
    const RepDev* reps;
    int64_t plane;
};

template <bool FINAL>
__global__ __launch_bounds__(256) void k_mp8_cells(Mp8Args a)
{
    const RepDev& R = a.reps[blockIdx.y];
    const int K = R.K, Kc = K >> 1, nb = mp8_blocks(K);
    if ((int)blockIdx.x >= nb) return;   // the whole work-group leaves together
    const int64_t nc = (int64_t)Kc * Kc * Kc;
    const int16_t* spins = a.spins + R.site_off;
    const float* Ctab = a.Ctab + R.grain_off * kTab;
    const float* u = a.u + R.site_off;
    float* F = a.F + R.site_off;
    const double* st = a.state + (int64_t)blockIdx.y * kStateDoubles;
    float E[6];
#pragma unroll
    for (int I = 0; I < 6; ++I) E[I] = (float)st[kE + I];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cell < nc;
         cell += (int64_t)nb * blockDim.x) {
        const int X = (int)(cell % Kc), Y = (int)((cell / Kc) % Kc), Z = (int)(cell / ((int64_t)Kc * Kc));
        const int X1 = X + 1 < Kc ? X + 1 : 0, Y1 = Y + 1 < Kc ? Y + 1 : 0, Z1 = Z + 1 < Kc ? Z + 1 : 0;
        float uc[8][3];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t node = (int64_t)((c & 1) ? X1 : X) +
                                 (int64_t)Kc * (((c >> 1) & 1 ? Y1 : Y) + (int64_t)Kc * ((c >> 2) & 1 ? Z1 : Z));
#pragma unroll
            for (int j = 0; j < 3; ++j) uc[c][j] = u[(int64_t)j * a.plane + node];
        }
        // Edge differences of the cell along each direction: D[d][e][j] for the 4 edges e
        // parallel to d (e = the other two bits, lower direction first).  The gradient at a
        // point is their bilinear interpolation, d/dx = 1/8 sum_e w w D (cell edge 2 sites).
        float D[3][4][3];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int b1 = e & 1, b2 = e >> 1;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                D[0][e][j] = uc[1 + 2 * b1 + 4 * b2][j] - uc[0 + 2 * b1 + 4 * b2][j];
                D[1][e][j] = uc[b1 + 2 + 4 * b2][j] - uc[b1 + 0 + 4 * b2][j];
                D[2][e][j] = uc[b1 + 2 * b2 + 4][j] - uc[b1 + 2 * b2 + 0][j];
            }
        }
        // per-edge force sums, the transpose: G[d][e][j] = 1/8 sum_p w w t_d(p)[j]
        float G[3][4][3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int e = 0; e < 4; ++e) G[d][e][0] = G[d][e][1] = G[d][e][2] = 0.f;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int px = p & 1, py = (p >> 1) & 1, pz = (p >> 2) & 1;
            const int64_t v = (int64_t)(2 * X + px) + (int64_t)K * ((2 * Y + py) + (int64_t)K * (2 * Z + pz));
            // point sub-positions along the two other directions of each d, lower first
            const int q1[3] = {py, px, px}, q2[3] = {pz, pz, py};
            float g[3][3];   // g[d][j] = d u_j / d x_d
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    float gs = 0.f;
#pragma unroll
                    for (int e = 0; e < 4; ++e) gs += (0.125f * mp_w(e & 1, q1[d]) * mp_w(e >> 1, q2[d])) * D[d][e][j];
                    g[d][j] = gs;
                }
            float e6[6], s[6];
            e6[0] = g[0][0] + E[0];
            e6[1] = g[1][1] + E[1];
            e6[2] = g[2][2] + E[2];
            e6[3] = (g[2][1] + g[1][2]) + E[3];
            e6[4] = (g[2][0] + g[0][2]) + E[4];
            e6[5] = (g[1][0] + g[0][1]) + E[5];
            symv21(Ctab + (int64_t)spins[v] * kTab, e6, s);
            if (FINAL) {
                double dd = 0.0;
#pragma unroll
                for (int I = 0; I < 6; ++I) dd += (double)s[I] * (double)e6[I];
                acc[0] += 0.5 * dd;
                if (a.sigma)
#pragma unroll
                    for (int I = 0; I < 6; ++I) a.sigma[(int64_t)I * a.plane + R.site_off + v] = s[I];
            } else {
#pragma unroll
                for (int I = 0; I < 6; ++I) acc[I] += (double)s[I];
                // traction rows t_d = sigma e_d (Voigt: xx yy zz yz xz xy)
                const float t[3][3] = {{s[0], s[5], s[4]}, {s[5], s[1], s[3]}, {s[4], s[3], s[2]}};
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float w = 0.125f * mp_w(e & 1, q1[d]) * mp_w(e >> 1, q2[d]);
#pragma unroll
                        for (int j = 0; j < 3; ++j) G[d][e][j] += w * t[d][j];
                    }
            }
        }
        // corner forces: + G at the upper end of every edge, - G at the lower end
        float f[8][3];
#pragma unroll
        for (int c = 0; c < 8; ++c) f[c][0] = f[c][1] = f[c][2] = 0.f;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int b1 = e & 1, b2 = e >> 1;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                f[1 + 2 * b1 + 4 * b2][j] += G[0][e][j];
                f[0 + 2 * b1 + 4 * b2][j] -= G[0][e][j];
                f[b1 + 2 + 4 * b2][j] += G[1][e][j];
                f[b1 + 0 + 4 * b2][j] -= G[1][e][j];
                f[b1 + 2 * b2 + 4][j] += G[2][e][j];
                f[b1 + 2 * b2 + 0][j] -= G[2][e][j];
            }
        }
        if (!FINAL)
#pragma unroll
            for (int c = 0; c < 8; ++c)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    F[(int64_t)((3 * c + j) >> 3) * a.plane + (int64_t)((3 * c + j) & 7) * nc + cell] = f[c][j];
    }
    if (FINAL)
        block_sum_to<1>(a.partials, acc, R.node_first + (int)blockIdx.x);
    else
        block_sum_to<6>(a.partials, acc, R.node_first + (int)blockIdx.x);
}

// Node n gathers corner c of cell n - c (bits x, y, z) from every one of its 8 cells.
__global__ __launch_bounds__(256) void k_mp8_nodes(const float* __restrict__ Fall, float* uall, float* wall,
                                                   const RepDev* reps, int64_t plane)
{
    const RepDev& R = reps[blockIdx.y];
    const int K = R.K, Kc = K >> 1, nb = mp8_blocks(K);
    if ((int)blockIdx.x >= nb) return;
    const int64_t nc = (int64_t)Kc * Kc * Kc;
    const float* F = Fall + R.site_off;
    float* u = uall + R.site_off;
    float* w = wall + R.site_off;
    const float alpha = R.glob_alpha, beta = R.glob_beta;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nc; n += (int64_t)nb * blockDim.x) {
        const int X = (int)(n % Kc), Y = (int)((n / Kc) % Kc), Z = (int)(n / ((int64_t)Kc * Kc));
        const int Xm = X > 0 ? X - 1 : Kc - 1, Ym = Y > 0 ? Y - 1 : Kc - 1, Zm = Z > 0 ? Z - 1 : Kc - 1;
        float r[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t cell = (int64_t)((c & 1) ? Xm : X) +
                                 (int64_t)Kc * (((c >> 1) & 1 ? Ym : Y) + (int64_t)Kc * ((c >> 2) & 1 ? Zm : Z));
#pragma unroll
            for (int j = 0; j < 3; ++j)
                r[j] -= F[(int64_t)((3 * c + j) >> 3) * plane + (int64_t)((3 * c + j) & 7) * nc + cell];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int64_t i = (int64_t)j * plane + n;
            const float wn = beta * w[i] + alpha * r[j];
            w[i] = wn;
            u[i] = u[i] + wn;
        }
    }
}

// One block per replica: fixed-order sum of its cell pass's stress sums, then its macroscopic
// update.
__global__ __launch_bounds__(256) void k_mp8_E(double* state, const double* partials, const RepDev* reps)
{
    const RepDev R = reps[blockIdx.x];
    const int nb = mp8_blocks(R.K);
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += 256)
#pragma unroll
        for (int I = 0; I < 6; ++I) s[I] += partials[(int64_t)(R.node_first + b) * 8 + I];
    const double tot = block_total<6>(s);
    if (threadIdx.x < 6) {
        double* st = state + (int64_t)blockIdx.x * kStateDoubles;
        const int I = threadIdx.x;
        const double rE = R.Sigma[I] - tot / (double)R.n3;
        const double wE = (double)R.glob_beta * st[kWE + I] + R.glob_alphaE * rE;
        st[kWE + I] = wE;
        st[kE + I] += wE;
    }
}

__global__ __launch_bounds__(256) void k_mp8_U(double* state, const double* partials, const RepDev* reps,
                                                uint32_t* nonfinite)
{
    const RepDev R = reps[blockIdx.x];
    const int nb = mp8_blocks(R.K);
    double s[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += 256) s[0] += partials[(int64_t)(R.node_first + b) * 8];
    const double tot = block_total<1>(s);
    if (threadIdx.x == 0) {
        state[(int64_t)blockIdx.x * kStateDoubles + kU] = tot;
        if (!isfinite(tot)) atomicOr(nonfinite, (uint32_t)kNfGlobal);   // a non-finite point stress
    }
}

Mp8Args mp8_args(hmc_ctx_s* c)
{
    Mp8Args a;
    a.spins = c->d.spins;
    a.Ctab = c->d.Ctab;
    a.u = c->d.u[0];
    a.F = c->d.u[1];
    a.sigma = nullptr;
    a.partials = c->d.partials;
    a.state = c->d.state;
    a.reps = c->d.reps;
    a.plane = c->total_sites;
    return a;
}

dim3 mp8_grid(const hmc_ctx_s* c)
{
    int nb = 1;
    for (const RepDev& R : c->reps) nb = std::max(nb, mp8_blocks(R.K));
    return dim3((unsigned)nb, (unsigned)c->n_rep);
}

}  // namespace

hipError_t launch_mp8_steps(hmc_ctx_s* c, int n_steps)
{
    const Mp8Args a = mp8_args(c);
    const dim3 grid = mp8_grid(c);
    for (int s = 0; s < n_steps; ++s) {
        const int tok = prof_begin(c, kProfRefreshStep);
        hipLaunchKernelGGL(k_mp8_cells<false>, grid, dim3(256), 0, c->stream, a);
        hipLaunchKernelGGL(k_mp8_nodes, grid, dim3(256), 0, c->stream, (const float*)c->d.u[1], c->d.u[0], c->d.w,
                           (const RepDev*)c->d.reps, c->total_sites);
        hipLaunchKernelGGL(k_mp8_E, dim3(c->n_rep), dim3(256), 0, c->stream, c->d.state, (const double*)c->d.partials,
                           (const RepDev*)c->d.reps);
        prof_end(c, tok);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_mp8_final(hmc_ctx_s* c, bool write_sigma)
{
    Mp8Args a = mp8_args(c);
    a.sigma = write_sigma ? c->d.sigma : nullptr;
    const int tok = prof_begin(c, kProfRefreshOther);
    hipLaunchKernelGGL(k_mp8_cells<true>, mp8_grid(c), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL(k_mp8_U, dim3(c->n_rep), dim3(256), 0, c->stream, c->d.state, (const double*)c->d.partials,
                       (const RepDev*)c->d.reps, c->d.counters + kNonFinite);
    prof_end(c, tok);
    return hipGetLastError();
}

}  // namespace hmc
