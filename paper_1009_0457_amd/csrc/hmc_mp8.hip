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
// and a one-block fold of the stress sums into E, per replica.  A replica's node fields occupy
// the first (K/2)^3 entries of its slice of each displacement plane; its corner forces use its
// slice of the second displacement buffer, which holds exactly 24 floats per cell.
#include "hmc_device.h"

namespace hmc {

namespace {

// Weight of the edge at bit b (0 or 1) of a cell direction for the point at sub-position p
// there: the trilinear shape functions' factor 1 +- xi_p with xi_p = +-1/2.
__host__ __device__ constexpr float mp_w(int b, int p) { return b == p ? 1.5f : 0.5f; }

struct Mp8Args {
    const int16_t* spins;
    const float* Ctab;
    const float* u;        // 3 planes of `plane` floats, nodes first
    float* F;              // 24 x n_cells corner forces: row k of the cells at plane k / 8,
                           // offset (k % 8) n_cells (a replica's slice of 3 planes of `plane`)
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
            symv21(a.Ctab + (int64_t)a.spins[v] * kTab, e6, s);
            if (FINAL) {
                double dd = 0.0;
#pragma unroll
                for (int I = 0; I < 6; ++I) dd += (double)s[I] * (double)e6[I];
                acc[0] += 0.5 * dd;
                if (a.sigma)
#pragma unroll
                    for (int I = 0; I < 6; ++I) a.sigma[(int64_t)I * a.plane + v] = s[I];
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
                    a.F[(int64_t)((3 * c + j) >> 3) * a.plane + (int64_t)((3 * c + j) & 7) * nc + cell] = f[c][j];
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

// One block: fixed-order sum of the cell pass's stress sums, then the macroscopic update.
__global__ __launch_bounds__(256) void k_mp8_E(double* state, const double* partials, int nblocks, const RepDev* reps,
                                               int rep)
{
    const RepDev R = reps[rep];
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

int mp8_blocks(const RepDev& R)
{
    const int64_t Kc = R.K / 2, nc = Kc * Kc * Kc;
    const int64_t b = (nc + 255) / 256;
    return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// Replica r's slices: its spins, grain tables, node fields, force rows and state.
Mp8Args mp8_args(hmc_ctx_s* c, int r)
{
    const RepDev& R = c->reps[r];
    Mp8Args a;
    a.spins = c->d.spins + R.site_off;
    a.Ctab = c->d.Ctab + R.grain_off * kTab;
    a.u = c->d.u[0] + R.site_off;
    a.F = c->d.u[1] + R.site_off;
    a.sigma = nullptr;
    a.partials = c->d.partials;
    a.state = c->d.state + (int64_t)r * kStateDoubles;
    a.K = R.K;
    a.plane = c->total_sites;
    return a;
}

}  // namespace

// Replicas of a batch run one after another within each step (their cell passes share the
// partial-sum buffer, which each replica's fold reads before the next replica's pass).
hipError_t launch_mp8_steps(hmc_ctx_s* c, int n_steps)
{
    for (int s = 0; s < n_steps; ++s) {
        const int tok = prof_begin(c, kProfRefreshStep);
        for (int r = 0; r < c->n_rep; ++r) {
            const RepDev& R = c->reps[r];
            const Mp8Args a = mp8_args(c, r);
            const int nb = mp8_blocks(R);
            hipLaunchKernelGGL(k_mp8_cells<false>, dim3(nb), dim3(256), 0, c->stream, a);
            hipLaunchKernelGGL(k_mp8_nodes, dim3(nb), dim3(256), 0, c->stream, (const float*)a.F,
                               c->d.u[0] + R.site_off, c->d.w + R.site_off, R.K, c->total_sites, R.glob_alpha,
                               R.glob_beta);
            hipLaunchKernelGGL(k_mp8_E, dim3(1), dim3(256), 0, c->stream, c->d.state + (int64_t)r * kStateDoubles,
                               (const double*)c->d.partials, nb, (const RepDev*)c->d.reps, r);
        }
        prof_end(c, tok);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_mp8_final(hmc_ctx_s* c, bool write_sigma)
{
    const int tok = prof_begin(c, kProfRefreshOther);
    for (int r = 0; r < c->n_rep; ++r) {
        Mp8Args a = mp8_args(c, r);
        a.sigma = write_sigma ? c->d.sigma + c->reps[r].site_off : nullptr;
        const int nb = mp8_blocks(c->reps[r]);
        hipLaunchKernelGGL(k_mp8_cells<true>, dim3(nb), dim3(256), 0, c->stream, a);
        hipLaunchKernelGGL(k_mp8_U, dim3(1), dim3(256), 0, c->stream, c->d.state + (int64_t)r * kStateDoubles,
                           (const double*)c->d.partials, nb);
    }
    prof_end(c, tok);
    return hipGetLastError();
}

}  // namespace hmc
