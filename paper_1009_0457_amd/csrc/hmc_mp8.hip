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
// the 8 corner displacements, the 8 points' strains and stresses, the cell's 24 corner forces
// written to a cell-major force array, and per-block sums of the point stresses), a node pass
// (one thread per node: the forces of its 8 cells, the heavy-ball update of u and w in place)
// and a one-block fold of the stress sums into E.  Single-lattice contexts only.  Node fields
// occupy the first (K/2)^3 entries of each displacement plane; the corner forces use the second
// displacement buffer, which holds exactly 24 floats per cell.
#include "hmc_device.h"

namespace hmc {

namespace {

// d N_c / d x_dir at material point p of a cell (c, p: bits x, y, z), times 8.
__host__ __device__ constexpr float mp_w8(int c, int p, int dir)
{
    float f = 1.0f;
    for (int d = 0; d < 3; ++d) {
        const float xc = ((c >> d) & 1) ? 1.0f : -1.0f;
        const float xp = ((p >> d) & 1) ? 0.5f : -0.5f;
        f *= (d == dir) ? xc : (1.0f + xc * xp);
    }
    return f;
}

struct Mp8Args {
    const int16_t* spins;
    const float* Ctab;
    const float* u;        // 3 planes of `plane` floats, nodes first
    float* F;              // 24 x n_cells corner forces (cell-major per component)
    float* sigma;          // final pass: 6 planes of point stresses (or null)
    double* partials;
    const double* state;
    int K;
    int64_t plane;
};

template <bool FINAL>
__global__ __launch_bounds__(256) void k_mp8_cells(Mp8Args a)
{
    const int K = a.K, Kc = K >> 1;
    const int64_t nc = (int64_t)Kc * Kc * Kc;
    float E[6];
#pragma unroll
    for (int I = 0; I < 6; ++I) E[I] = (float)a.state[kE + I];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cell < nc;
         cell += (int64_t)gridDim.x * blockDim.x) {
        const int X = (int)(cell % Kc), Y = (int)((cell / Kc) % Kc), Z = (int)(cell / ((int64_t)Kc * Kc));
        const int X1 = X + 1 < Kc ? X + 1 : 0, Y1 = Y + 1 < Kc ? Y + 1 : 0, Z1 = Z + 1 < Kc ? Z + 1 : 0;
        float uc[8][3];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t node = (int64_t)((c & 1) ? X1 : X) +
                                 (int64_t)Kc * (((c >> 1) & 1 ? Y1 : Y) + (int64_t)Kc * ((c >> 2) & 1 ? Z1 : Z));
#pragma unroll
            for (int j = 0; j < 3; ++j) uc[c][j] = a.u[(int64_t)j * a.plane + node];
        }
        float f[8][3];
#pragma unroll
        for (int c = 0; c < 8; ++c) f[c][0] = f[c][1] = f[c][2] = 0.f;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int64_t v = (int64_t)(2 * X + (p & 1)) +
                              (int64_t)K * ((2 * Y + ((p >> 1) & 1)) + (int64_t)K * (2 * Z + ((p >> 2) & 1)));
            float g[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};   // g[j][i] = d u_j / d x_i
#pragma unroll
            for (int c = 0; c < 8; ++c)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const float w = 0.125f * mp_w8(c, p, i);
#pragma unroll
                    for (int j = 0; j < 3; ++j) g[j][i] += w * uc[c][j];
                }
            float e[6], s[6];
            e[0] = g[0][0] + E[0];
            e[1] = g[1][1] + E[1];
            e[2] = g[2][2] + E[2];
            e[3] = (g[1][2] + g[2][1]) + E[3];
            e[4] = (g[0][2] + g[2][0]) + E[4];
            e[5] = (g[0][1] + g[1][0]) + E[5];
            symv21(a.Ctab + (int64_t)a.spins[v] * kTab, e, s);
            if (FINAL) {
                double d = 0.0;
#pragma unroll
                for (int I = 0; I < 6; ++I) d += (double)s[I] * (double)e[I];
                acc[0] += 0.5 * d;
                if (a.sigma)
#pragma unroll
                    for (int I = 0; I < 6; ++I) a.sigma[(int64_t)I * a.plane + v] = s[I];
            } else {
#pragma unroll
                for (int I = 0; I < 6; ++I) acc[I] += (double)s[I];
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const float gx = 0.125f * mp_w8(c, p, 0), gy = 0.125f * mp_w8(c, p, 1),
                                gz = 0.125f * mp_w8(c, p, 2);
                    f[c][0] += gx * s[0] + gy * s[5] + gz * s[4];
                    f[c][1] += gx * s[5] + gy * s[1] + gz * s[3];
                    f[c][2] += gx * s[4] + gy * s[3] + gz * s[2];
                }
            }
        }
        if (!FINAL)
#pragma unroll
            for (int c = 0; c < 8; ++c)
#pragma unroll
                for (int j = 0; j < 3; ++j) a.F[(int64_t)(3 * c + j) * nc + cell] = f[c][j];
    }
    if (FINAL)
        block_sum_to<1>(a.partials, acc);
    else
        block_sum_to<6>(a.partials, acc);
}

// Node n gathers corner c of cell n - c (bits x, y, z) from every one of its 8 cells.
__global__ __launch_bounds__(256) void k_mp8_nodes(const float* __restrict__ F, float* u, float* w, int K,
                                                   int64_t plane, float alpha, float beta)
{
    const int Kc = K >> 1;
    const int64_t nc = (int64_t)Kc * Kc * Kc;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nc; n += (int64_t)gridDim.x * blockDim.x) {
        const int X = (int)(n % Kc), Y = (int)((n / Kc) % Kc), Z = (int)(n / ((int64_t)Kc * Kc));
        const int Xm = X > 0 ? X - 1 : Kc - 1, Ym = Y > 0 ? Y - 1 : Kc - 1, Zm = Z > 0 ? Z - 1 : Kc - 1;
        float r[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t cell = (int64_t)((c & 1) ? Xm : X) +
                                 (int64_t)Kc * (((c >> 1) & 1 ? Ym : Y) + (int64_t)Kc * ((c >> 2) & 1 ? Zm : Z));
#pragma unroll
            for (int j = 0; j < 3; ++j) r[j] -= F[(int64_t)(3 * c + j) * nc + cell];
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

// One block: fixed-order sum of the cell pass's stress sums, then the macroscopic update.
__global__ __launch_bounds__(256) void k_mp8_E(double* state, const double* partials, int nblocks, const RepDev* reps)
{
    const RepDev R = reps[0];
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256)
#pragma unroll
        for (int I = 0; I < 6; ++I) s[I] += partials[(int64_t)b * 8 + I];
    const double tot = block_total<6>(s);
    if (threadIdx.x < 6) {
        const int I = threadIdx.x;
        const double rE = R.Sigma[I] - tot / (double)R.n3;
        const double wE = (double)R.glob_beta * state[kWE + I] + R.glob_alphaE * rE;
        state[kWE + I] = wE;
        state[kE + I] += wE;
    }
}

__global__ __launch_bounds__(256) void k_mp8_U(double* state, const double* partials, int nblocks)
{
    double s[1] = {0.0};
    for (int b = threadIdx.x; b < nblocks; b += 256) s[0] += partials[(int64_t)b * 8];
    const double tot = block_total<1>(s);
    if (threadIdx.x == 0) state[kU] = tot;
}

int mp8_blocks(const hmc_ctx_s* c)
{
    const int64_t Kc = c->reps[0].K / 2, nc = Kc * Kc * Kc;
    const int64_t b = (nc + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
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
    a.K = c->reps[0].K;
    a.plane = c->total_sites;
    return a;
}

}  // namespace

hipError_t launch_mp8_steps(hmc_ctx_s* c, int n_steps)
{
    const RepDev& R = c->reps[0];
    const Mp8Args a = mp8_args(c);
    const int nb = mp8_blocks(c);
    for (int s = 0; s < n_steps; ++s) {
        const int tok = prof_begin(c, kProfRefreshStep);
        hipLaunchKernelGGL(k_mp8_cells<false>, dim3(nb), dim3(256), 0, c->stream, a);
        hipLaunchKernelGGL(k_mp8_nodes, dim3(nb), dim3(256), 0, c->stream, (const float*)c->d.u[1], c->d.u[0], c->d.w,
                           R.K, c->total_sites, R.glob_alpha, R.glob_beta);
        hipLaunchKernelGGL(k_mp8_E, dim3(1), dim3(256), 0, c->stream, c->d.state, (const double*)c->d.partials, nb,
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
    const int nb = mp8_blocks(c);
    const int tok = prof_begin(c, kProfRefreshOther);
    hipLaunchKernelGGL(k_mp8_cells<true>, dim3(nb), dim3(256), 0, c->stream, a);
    hipLaunchKernelGGL(k_mp8_U, dim3(1), dim3(256), 0, c->stream, c->d.state, (const double*)c->d.partials, nb);
    prof_end(c, tok);
    return hipGetLastError();
}

}  // namespace hmc
