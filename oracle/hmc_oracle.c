/*
 * hmc_oracle.c -- serial FP64 CPU oracle for the hybrid Monte Carlo (HMC) hot path of
 * Zhang, Bartel & Lusk, "Parallelized Hybrid Monte Carlo Simulation of Stress-Induced
 * Texture Evolution" (arXiv:1009.0457).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this file's library.  It shares no code, header, table or
 * helper with the HIP library; it is written to be read against the paper, not to be
 * fast: plain loops, double precision, one thread, no blocking or fusion.
 *
 * What each part follows:
 *   - Potts grain-boundary energy and the Metropolis rule: Sec. 3, Eqs. (H_1) and
 *     (metrop_1).  H_gb = J * (number of unlike neighbour bonds), each bond once; for a
 *     trial flip of site i only the bonds of i change.
 *   - Red/black (here: 2- or 8-colour) checkerboard with updates deferred to the end of
 *     each half step: Sec. 6.  The Gauss-Seidel scheme Sec. 6 compares it with (every site
 *     in turn, each accepted change written at once) is here too, at zero load.
 *   - Global solve with 2 x 2 x 2 material points per background cell (Appendix), as a
 *     variant of the one-point default.
 *   - Local elastic energy change from a zone Omega_1 under constant boundary traction,
 *     "stored energy minus boundary work": Sec. 3, Eq. (H_1, second form) and Fig. 1;
 *     the point-zone limit is Eq. (eladriv).
 *   - Rotated cubic stiffness C'_ijkl = A_im A_jn A_ko A_lp C_mnop with A built from
 *     three Euler angles: Sec. 5, Eq. (stiffrot).
 *   - Global quasi-static elastic state by time-explicit damped relaxation of a
 *     background-grid discretisation with one material point per lattice site: Sec. 5.
 *   - The trial random numbers come from Philox4x32-10 (Salmon et al., SC'11), which
 *     the paper does not specify; its keying on (seed, sweep, site) is this library's.
 *
 * Conventions (shared with the HIP path by specification, not by code):
 *   site index i = x + K*(y + K*z); Voigt order xx,yy,zz,yz,xz,xy with engineering
 *   shear strains; stiffness in GPa, stress in GPa, energies in GPa*voxel.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------ */
/* Philox4x32-10: ten rounds of two 32x32->64 multiplies, key bumped by the Weyl        */
/* constants between rounds.                                                              */
/* ------------------------------------------------------------------------------------ */
void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t mult0 = 0xD2511F53u, mult1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint64_t prod0 = (uint64_t)mult0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)mult1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* The four words drawn for one site-trial: key = (seed low, seed high), counter =
 * (site, sweep, 0, 0).  r0 picks the trial state, r1 is the Metropolis variate.         */
void ora_draw(uint64_t seed, uint32_t site, uint32_t sweep, uint32_t out[4])
{
    uint32_t ctr[4] = {site, sweep, 0u, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    ora_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------------------ */
/* Lattice geometry                                                                      */
/* ------------------------------------------------------------------------------------ */
static int64_t wrap(int64_t a, int64_t K)
{
    a %= K;
    return a < 0 ? a + K : a;
}

static int64_t site_of(int64_t x, int64_t y, int64_t z, int64_t K)
{
    return wrap(x, K) + K * (wrap(y, K) + K * wrap(z, K));
}

/* Neighbour slot k of a site as an offset.  6 neighbours: -x,+x,-y,+y,-z,+z.
 * 26 neighbours: (dz,dy,dx) in lexicographic order over {-1,0,1}^3 without (0,0,0).      */
void ora_slot_offset(int M, int k, int off[3])
{
    if (M == 6) {
        static const int tab[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                                      {0, 1, 0},  {0, 0, -1}, {0, 0, 1}};
        off[0] = tab[k][0]; off[1] = tab[k][1]; off[2] = tab[k][2];
        return;
    }
    int n = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                if (n == k) { off[0] = dx; off[1] = dy; off[2] = dz; return; }
                ++n;
            }
}

int64_t ora_neighbour(int K, int M, int64_t site, int k)
{
    int off[3];
    ora_slot_offset(M, k, off);
    int64_t x = site % K, y = (site / K) % K, z = site / ((int64_t)K * K);
    return site_of(x + off[0], y + off[1], z + off[2], K);
}

/* Colour classes: with 6 neighbours the red/black parity of x+y+z; with 26 neighbours
 * the 2x2x2 sublattice (x&1) + 2(y&1) + 4(z&1).  No two sites of one class are
 * neighbours, so the trials of a class only read sites of other classes.               */
int ora_colour(int M, int64_t x, int64_t y, int64_t z)
{
    if (M == 6) return (int)((x + y + z) & 1);
    return (int)((x & 1) | ((y & 1) << 1) | ((z & 1) << 2));
}

int ora_num_colours(int M) { return M == 6 ? 2 : 8; }

/* ------------------------------------------------------------------------------------ */
/* Grain-boundary term                                                                   */
/* ------------------------------------------------------------------------------------ */
/* Change in the number of unlike bonds of site i when its spin goes q_old -> q_new:
 * sum over neighbour slots of [delta(q_n, q_old) - delta(q_n, q_new)].  The energy change
 * is J times this count.                                                                */
int ora_gb_count(int K, int M, const int32_t* q, int64_t site, int32_t q_new)
{
    int32_t q_old = q[site];
    int count = 0;
    for (int k = 0; k < M; ++k) {
        int32_t qn = q[ora_neighbour(K, M, site, k)];
        count += (qn == q_old) - (qn == q_new);
    }
    return count;
}

/* Number of unlike bonds: unlike neighbour slots summed over all sites, halved. */
int64_t ora_unlike_bonds(int K, int M, const int32_t* q)
{
    int64_t n = (int64_t)K * K * K, slots = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < M; ++k)
            slots += (q[ora_neighbour(K, M, i, k)] != q[i]);
    return slots / 2;
}

/* Trial state.  proposal 0: the spin of a random neighbour slot, slot = floor(r0*M/2^32).
 * proposal 1: a uniformly random state other than the current one.                      */
int32_t ora_propose(int K, int M, int Q, int proposal, const int32_t* q, int64_t site, uint32_t r0)
{
    if (proposal == 0) {
        int k = (int)(((uint64_t)r0 * (uint64_t)M) >> 32);
        return q[ora_neighbour(K, M, site, k)];
    }
    uint32_t step = (uint32_t)(((uint64_t)r0 * (uint64_t)(Q - 1)) >> 32);
    return (int32_t)((q[site] + 1 + (int64_t)step) % Q);
}

/* ------------------------------------------------------------------------------------ */
/* Stiffness tables (Sec. 5)                                                             */
/* ------------------------------------------------------------------------------------ */
static const int voigt_i[6] = {0, 1, 2, 1, 0, 0};
static const int voigt_j[6] = {0, 1, 2, 2, 2, 1};

static int voigt_index(int i, int j)
{
    if (i == j) return i;
    int s = i + j;               /* (1,2)->3, (0,2)->4, (0,1)->5 */
    return s == 3 ? 3 : (s == 2 ? 4 : 5);
}

/* Active rotation crystal -> lab, A = Rz(phi1) Rx(Phi) Rz(phi2). */
void ora_rotation(double phi1, double Phi, double phi2, double A[9])
{
    double c1 = cos(phi1), s1 = sin(phi1), c = cos(Phi), s = sin(Phi), c2 = cos(phi2), s2 = sin(phi2);
    double Rz1[3][3] = {{c1, -s1, 0}, {s1, c1, 0}, {0, 0, 1}};
    double Rx[3][3] = {{1, 0, 0}, {0, c, -s}, {0, s, c}};
    double Rz2[3][3] = {{c2, -s2, 0}, {s2, c2, 0}, {0, 0, 1}};
    double T[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            T[i][j] = 0;
            for (int k = 0; k < 3; ++k) T[i][j] += Rz1[i][k] * Rx[k][j];
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double v = 0;
            for (int k = 0; k < 3; ++k) v += T[i][k] * Rz2[k][j];
            A[3 * i + j] = v;
        }
}

/* C'_ijkl = sum_mnop A_im A_jn A_ko A_lp C_mnop (Eq. stiffrot with the summed indices on
 * the crystal tensor), written out as the 4-index sum. Both tensors in Voigt 6x6 form.    */
void ora_rotate_stiffness(const double A[9], const double Ccrys[36], double Clab[36])
{
    double C4[3][3][3][3], R4[3][3][3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l)
                    C4[i][j][k][l] = Ccrys[6 * voigt_index(i, j) + voigt_index(k, l)];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) {
                    double v = 0;
                    for (int m = 0; m < 3; ++m)
                        for (int n = 0; n < 3; ++n)
                            for (int o = 0; o < 3; ++o)
                                for (int p = 0; p < 3; ++p)
                                    v += A[3 * i + m] * A[3 * j + n] * A[3 * k + o] * A[3 * l + p] *
                                         C4[m][n][o][p];
                    R4[i][j][k][l] = v;
                }
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J)
            Clab[6 * I + J] = R4[voigt_i[I]][voigt_j[I]][voigt_i[J]][voigt_j[J]];
}

/* Inverse of a 6x6 matrix by Gauss-Jordan elimination with partial pivoting.
 * Returns 0 on success, -1 if singular.                                                 */
int ora_invert6(const double Min[36], double Mout[36])
{
    double a[6][12];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 12; ++j) a[i][j] = j < 6 ? Min[6 * i + j] : (j - 6 == i ? 1.0 : 0.0);
    for (int col = 0; col < 6; ++col) {
        int piv = col;
        for (int r = col + 1; r < 6; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (a[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int j = 0; j < 12; ++j) { double t = a[col][j]; a[col][j] = a[piv][j]; a[piv][j] = t; }
        double d = a[col][col];
        for (int j = 0; j < 12; ++j) a[col][j] /= d;
        for (int r = 0; r < 6; ++r) {
            if (r == col) continue;
            double f = a[r][col];
            if (f != 0.0)
                for (int j = 0; j < 12; ++j) a[r][j] -= f * a[col][j];
        }
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) Mout[6 * i + j] = a[i][j + 6];
    return 0;
}

/* Per-grain lab-frame stiffness C (Q x 36), compliance S = C^-1 (Q x 36) and rotation
 * (Q x 9) from Bunge Euler angles (Q x 3, radians) and cubic constants (GPa).
 * Returns 0, or -1 if some stiffness is singular.                                       */
int ora_tables(int Q, const double* euler, double C11, double C12, double C44,
               double* Ctab, double* Stab, double* Arot)
{
    double Cc[36];
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J) {
            double v = 0;
            if (I < 3 && J < 3) v = (I == J) ? C11 : C12;
            else if (I == J) v = C44;
            Cc[6 * I + J] = v;
        }
    for (int g = 0; g < Q; ++g) {
        double A[9];
        ora_rotation(euler[3 * g], euler[3 * g + 1], euler[3 * g + 2], A);
        if (Arot) memcpy(Arot + 9 * g, A, sizeof A);
        ora_rotate_stiffness(A, Cc, Ctab + 36 * g);
        if (ora_invert6(Ctab + 36 * g, Stab + 36 * g) != 0) return -1;
    }
    return 0;
}

/* Angle (degrees) between a unit lab axis and the nearest crystal <100> direction. */
double ora_texture_angle(const double A[9], const double axis[3])
{
    double n = sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    double best = 0;
    for (int m = 0; m < 3; ++m) {
        /* component of the axis on crystal direction m: (A^T d)_m */
        double c = (A[m] * axis[0] + A[3 + m] * axis[1] + A[6 + m] * axis[2]) / n;
        if (fabs(c) > best) best = fabs(c);
    }
    if (best > 1.0) best = 1.0;
    return acos(best) * (180.0 / M_PI);
}

/* Volume-weighted histogram of that angle over all sites. */
void ora_texture_counts(int K, const int32_t* q, int Q, const double* Arot, const double axis[3],
                        double bin_deg, int nbins, int64_t* counts)
{
    int* bin = (int*)malloc(sizeof(int) * (size_t)Q);
    for (int g = 0; g < Q; ++g) {
        int b = (int)floor(ora_texture_angle(Arot + 9 * g, axis) / bin_deg);
        bin[g] = b < nbins - 1 ? b : nbins - 1;
    }
    for (int b = 0; b < nbins; ++b) counts[b] = 0;
    int64_t n = (int64_t)K * K * K;
    for (int64_t i = 0; i < n; ++i) counts[bin[q[i]]] += 1;
    free(bin);
}

/* ------------------------------------------------------------------------------------ */
/* Element operator: one material point at the centre of a voxel, corners as nodes.      */
/* Corner c = a + 2b + 4d for offsets (a,b,d) along x,y,z.  The shape-function gradient   */
/* at the centre is (+-1/4, +-1/4, +-1/4), + on the high side.                          */
/* ------------------------------------------------------------------------------------ */
static double corner_grad(int c, int dir)
{
    return ((c >> dir) & 1) ? 0.25 : -0.25;
}

/* Voigt engineering strain of the corner displacements u[8][3]. */
static void voxel_strain(const double u[8][3], double e[6])
{
    double g[3][3] = {{0}};   /* g[j][i] = d u_j / d x_i */
    for (int c = 0; c < 8; ++c)
        for (int j = 0; j < 3; ++j)
            for (int i = 0; i < 3; ++i) g[j][i] += corner_grad(c, i) * u[c][j];
    e[0] = g[0][0];
    e[1] = g[1][1];
    e[2] = g[2][2];
    e[3] = g[1][2] + g[2][1];
    e[4] = g[0][2] + g[2][0];
    e[5] = g[0][1] + g[1][0];
}

/* Corner forces f[c][j] = sum_i dN_c/dx_i sigma_ij: the transpose of voxel_strain. */
static void voxel_forces(const double s[6], double f[8][3])
{
    for (int c = 0; c < 8; ++c) {
        double gx = corner_grad(c, 0), gy = corner_grad(c, 1), gz = corner_grad(c, 2);
        f[c][0] = gx * s[0] + gy * s[5] + gz * s[4];
        f[c][1] = gx * s[5] + gy * s[1] + gz * s[3];
        f[c][2] = gx * s[4] + gy * s[3] + gz * s[2];
    }
}

static void matvec6(const double* M, const double* x, double* y)
{
    for (int I = 0; I < 6; ++I) {
        double v = 0;
        for (int J = 0; J < 6; ++J) v += M[6 * I + J] * x[J];
        y[I] = v;
    }
}

static double dot6(const double* a, const double* b)
{
    double v = 0;
    for (int I = 0; I < 6; ++I) v += a[I] * b[I];
    return v;
}

/* ------------------------------------------------------------------------------------ */
/* Global elastic state (Sec. 5): periodic K^3 grid of corner nodes, one material point   */
/* per site, unknowns = nodal displacement fluctuation u (3 x K^3, component-major) and   */
/* the macroscopic strain E (Voigt).  Strain at site v: E + B_v u; stress C_{q_v} times   */
/* it.  The applied load is the average stress Sigma.  Each explicit step:                */
/*   r_n = -sum_{v at n} B_v(n)^T sigma_v,   r_E = Sigma - mean_v sigma_v                 */
/*   w <- beta w + alpha r,   u <- u + w;   wE <- beta wE + alphaE r_E,  E <- E + wE       */
/* which is damped explicit dynamics (alpha = dt^2/m, beta = 1 - c dt).                  */
/* cold != 0: start from u = 0 and the uniform-stress (Reuss) strain E = mean(S_q) Sigma. */
/* Outputs: sigma_out (6 x K^3, component-major, may be NULL), info[0] = stored energy    */
/* U = 1/2 sum sigma.eps, info[1] = |r| (2-norm of nodal residual), info[2] = |r_E|.      */
/* ------------------------------------------------------------------------------------ */
static void gather_corners(int K, const double* u, int64_t x, int64_t y, int64_t z, double uc[8][3])
{
    int64_t n3 = (int64_t)K * K * K;
    for (int c = 0; c < 8; ++c) {
        int64_t node = site_of(x + (c & 1), y + ((c >> 1) & 1), z + ((c >> 2) & 1), K);
        for (int j = 0; j < 3; ++j) uc[c][j] = u[j * n3 + node];
    }
}

static void global_residual(int K, const int32_t* q, const double* Ctab, const double* u, const double* E,
                            double* r, double* sig_sum, double* sig_out, double* energy)
{
    int64_t n3 = (int64_t)K * K * K;
    if (r) memset(r, 0, sizeof(double) * 3 * (size_t)n3);
    for (int I = 0; I < 6; ++I) sig_sum[I] = 0;
    double U = 0;
    for (int64_t z = 0; z < K; ++z)
        for (int64_t y = 0; y < K; ++y)
            for (int64_t x = 0; x < K; ++x) {
                int64_t v = x + K * (y + K * z);
                double uc[8][3], e[6], s[6], f[8][3];
                gather_corners(K, u, x, y, z, uc);
                voxel_strain(uc, e);
                for (int I = 0; I < 6; ++I) e[I] += E[I];
                matvec6(Ctab + 36 * (int64_t)q[v], e, s);
                for (int I = 0; I < 6; ++I) sig_sum[I] += s[I];
                if (sig_out)
                    for (int I = 0; I < 6; ++I) sig_out[I * n3 + v] = s[I];
                U += 0.5 * dot6(s, e);
                if (r) {
                    voxel_forces(s, f);
                    for (int c = 0; c < 8; ++c) {
                        int64_t node = site_of(x + (c & 1), y + ((c >> 1) & 1), z + ((c >> 2) & 1), K);
                        for (int j = 0; j < 3; ++j) r[j * n3 + node] -= f[c][j];
                    }
                }
            }
    if (energy) *energy = U;
}

void ora_global(int K, const int32_t* q, const double* Ctab, const double* Stab, const double Sigma[6],
                int nsteps, int cold, double alpha, double beta, double alphaE,
                double* u, double* E, double* sigma_out, double* info)
{
    int64_t n3 = (int64_t)K * K * K;
    if (cold) {
        memset(u, 0, sizeof(double) * 3 * (size_t)n3);
        double Sm[36] = {0};
        for (int64_t v = 0; v < n3; ++v)
            for (int a = 0; a < 36; ++a) Sm[a] += Stab[36 * (int64_t)q[v] + a];
        for (int a = 0; a < 36; ++a) Sm[a] /= (double)n3;
        matvec6(Sm, Sigma, E);
    }
    double* w = (double*)calloc(3 * (size_t)n3, sizeof(double));
    double* r = (double*)malloc(sizeof(double) * 3 * (size_t)n3);
    double wE[6] = {0}, ssum[6];
    for (int t = 0; t < nsteps; ++t) {
        global_residual(K, q, Ctab, u, E, r, ssum, NULL, NULL);
        for (int64_t a = 0; a < 3 * n3; ++a) {
            w[a] = beta * w[a] + alpha * r[a];
            u[a] += w[a];
        }
        for (int I = 0; I < 6; ++I) {
            double rE = Sigma[I] - ssum[I] / (double)n3;
            wE[I] = beta * wE[I] + alphaE * rE;
            E[I] += wE[I];
        }
    }
    double U;
    global_residual(K, q, Ctab, u, E, r, ssum, sigma_out, &U);
    if (info) {
        double rn = 0, re = 0;
        for (int64_t a = 0; a < 3 * n3; ++a) rn += r[a] * r[a];
        for (int I = 0; I < 6; ++I) {
            double d = Sigma[I] - ssum[I] / (double)n3;
            re += d * d;
        }
        info[0] = U;
        info[1] = sqrt(rn);
        info[2] = sqrt(re);
    }
    free(w);
    free(r);
}

/* Stored elastic energy 1/2 sum_v eps_v . C_{q_v} eps_v of a given state (u, E). */
/* Variant with 2 x 2 x 2 material points per background cell (the arrangement of the
 * paper's MPM, Appendix: particles per cell fixed, two per direction).  The mesh has
 * (K/2)^3 periodic nodes at the corners of cells of 2 x 2 x 2 sites; every site is a material
 * point at local coordinates +-1/2 of its cell, with its own stiffness.  Its strain is the
 * gradient of the trilinear interpolation of the cell's 8 corner displacements there (cell
 * edge 2 sites, so d/dx = d/dxi), its nodal forces the transpose.  Otherwise the relaxation is
 * the one of ora_global: average-stress control, heavy ball, Reuss cold start. */
static double mp_grad(int c, int p, int dir)
{
    double f = 0.125;
    for (int d = 0; d < 3; ++d) {
        const double xc = ((c >> d) & 1) ? 1.0 : -1.0;
        const double xp = ((p >> d) & 1) ? 0.5 : -0.5;
        f *= (d == dir) ? xc : (1.0 + xc * xp);
    }
    return f;
}

static void global_residual_mp8(int K, const int32_t* q, const double* Ctab, const double* u, const double* E,
                                double* r, double* sig_sum, double* sig_out, double* energy)
{
    const int64_t Kc = K / 2, nn = Kc * Kc * Kc, n3 = (int64_t)K * K * K;
    if (r) memset(r, 0, sizeof(double) * 3 * (size_t)nn);
    for (int I = 0; I < 6; ++I) sig_sum[I] = 0;
    double U = 0;
    for (int64_t Z = 0; Z < Kc; ++Z)
        for (int64_t Y = 0; Y < Kc; ++Y)
            for (int64_t X = 0; X < Kc; ++X) {
                int64_t node[8];
                double uc[8][3], f[8][3] = {{0}};
                for (int c = 0; c < 8; ++c) {
                    node[c] = site_of(X + (c & 1), Y + ((c >> 1) & 1), Z + ((c >> 2) & 1), (int)Kc);
                    for (int j = 0; j < 3; ++j) uc[c][j] = u[j * nn + node[c]];
                }
                for (int p = 0; p < 8; ++p) {
                    const int64_t v = site_of(2 * X + (p & 1), 2 * Y + ((p >> 1) & 1), 2 * Z + ((p >> 2) & 1), K);
                    double g[3][3] = {{0}}, e[6], s[6];
                    for (int c = 0; c < 8; ++c)
                        for (int i = 0; i < 3; ++i) {
                            const double w = mp_grad(c, p, i);
                            for (int j = 0; j < 3; ++j) g[j][i] += w * uc[c][j];
                        }
                    e[0] = g[0][0] + E[0];
                    e[1] = g[1][1] + E[1];
                    e[2] = g[2][2] + E[2];
                    e[3] = g[1][2] + g[2][1] + E[3];
                    e[4] = g[0][2] + g[2][0] + E[4];
                    e[5] = g[0][1] + g[1][0] + E[5];
                    matvec6(Ctab + 36 * (int64_t)q[v], e, s);
                    for (int I = 0; I < 6; ++I) sig_sum[I] += s[I];
                    if (sig_out)
                        for (int I = 0; I < 6; ++I) sig_out[I * n3 + v] = s[I];
                    U += 0.5 * dot6(s, e);
                    for (int c = 0; c < 8; ++c) {
                        const double gx = mp_grad(c, p, 0), gy = mp_grad(c, p, 1), gz = mp_grad(c, p, 2);
                        f[c][0] += gx * s[0] + gy * s[5] + gz * s[4];
                        f[c][1] += gx * s[5] + gy * s[1] + gz * s[3];
                        f[c][2] += gx * s[4] + gy * s[3] + gz * s[2];
                    }
                }
                if (r)
                    for (int c = 0; c < 8; ++c)
                        for (int j = 0; j < 3; ++j) r[j * nn + node[c]] -= f[c][j];
            }
    if (energy) *energy = U;
}

/* u: 3 x (K/2)^3 node displacements (K even). */
void ora_global_mp8(int K, const int32_t* q, const double* Ctab, const double* Stab, const double Sigma[6],
                    int nsteps, int cold, double alpha, double beta, double alphaE,
                    double* u, double* E, double* sigma_out, double* info)
{
    const int64_t n3 = (int64_t)K * K * K, nn = n3 / 8;
    if (cold) {
        memset(u, 0, sizeof(double) * 3 * (size_t)nn);
        double Sm[36] = {0};
        for (int64_t v = 0; v < n3; ++v)
            for (int a = 0; a < 36; ++a) Sm[a] += Stab[36 * (int64_t)q[v] + a];
        for (int a = 0; a < 36; ++a) Sm[a] /= (double)n3;
        matvec6(Sm, Sigma, E);
    }
    double* w = (double*)calloc(3 * (size_t)nn, sizeof(double));
    double* r = (double*)malloc(sizeof(double) * 3 * (size_t)nn);
    double wE[6] = {0}, ssum[6];
    for (int t = 0; t < nsteps; ++t) {
        global_residual_mp8(K, q, Ctab, u, E, r, ssum, NULL, NULL);
        for (int64_t a = 0; a < 3 * nn; ++a) {
            w[a] = beta * w[a] + alpha * r[a];
            u[a] += w[a];
        }
        for (int I = 0; I < 6; ++I) {
            const double rE = Sigma[I] - ssum[I] / (double)n3;
            wE[I] = beta * wE[I] + alphaE * rE;
            E[I] += wE[I];
        }
    }
    double U;
    global_residual_mp8(K, q, Ctab, u, E, r, ssum, sigma_out, &U);
    if (info) {
        double rn = 0, re = 0;
        for (int64_t a = 0; a < 3 * nn; ++a) rn += r[a] * r[a];
        for (int I = 0; I < 6; ++I) {
            const double d = Sigma[I] - ssum[I] / (double)n3;
            re += d * d;
        }
        info[0] = U;
        info[1] = sqrt(rn);
        info[2] = sqrt(re);
    }
    free(w);
    free(r);
}

/* Residual forces (3 x (K/2)^3) and the point stresses of the variant above at (u, E). */
void ora_residual_mp8(int K, const int32_t* q, const double* Ctab, const double* u, const double* E, double* r,
                      double* sig_out, double* U)
{
    double ssum[6];
    global_residual_mp8(K, q, Ctab, u, E, r, ssum, sig_out, U);
}

double ora_elastic_energy(int K, const int32_t* q, const double* Ctab, const double* u, const double* E)
{
    double ssum[6], U;
    global_residual(K, q, Ctab, u, E, NULL, ssum, NULL, &U);
    return U;
}

/* ------------------------------------------------------------------------------------ */
/* Zone solve (Sec. 3, Eq. H_1 second form): the trial flip of site p from q_old to q_new */
/* inside a zone of (2h+1)^3 voxels centred at p whose outer boundary keeps its traction. */
/* With eps_p = S_{q_old} sigma_p the strain of p under its current stress, dC =          */
/* C_new - C_old and t = dC eps_p, the change of (stored energy - boundary work) is       */
/*   dPi = 1/2 eps_p.dC eps_p + min over du of [ t.(B_p du) + 1/2 sum_v (B_v du).C_v(B_v du) ] */
/* where du is the extra displacement of the zone's (2h+2)^3 nodes (free outer boundary), */
/* C_v the stiffness of the snapshot spin at voxel v and C_new at p.  The minimisation is */
/* n_r heavy-ball steps w <- beta w - alpha grad, du <- du + w from du = w = 0, with no   */
/* early exit; dPi is evaluated at the final du.  For h = 0 and n_r -> infinity this is   */
/* the point-zone result 1/2 sigma_p.(S_old - S_new) sigma_p (Eq. eladriv, with the sign */
/* that makes the softer grain grow).                                                    */
/* ------------------------------------------------------------------------------------ */
double ora_zone(int K, const int32_t* q, const double* Ctab, const double* Stab,
                int64_t p, int32_t q_new, const double sigma_p[6], int h, int nr,
                double alpha, double beta)
{
    int n = 2 * h + 1, nn = 2 * h + 2;
    int nv = n * n * n, nnodes = nn * nn * nn;
    int64_t px = p % K, py = (p / K) % K, pz = p / ((int64_t)K * K);
    int32_t q_old = q[p];
    const double* Cold = Ctab + 36 * (int64_t)q_old;
    const double* Cnew = Ctab + 36 * (int64_t)q_new;
    double eps[6], dC[36], t[6];
    matvec6(Stab + 36 * (int64_t)q_old, sigma_p, eps);
    for (int a = 0; a < 36; ++a) dC[a] = Cnew[a] - Cold[a];
    matvec6(dC, eps, t);

    const double** Cv = (const double**)malloc(sizeof(double*) * (size_t)nv);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int v = i + n * (j + n * k);
                if (i == h && j == h && k == h) Cv[v] = Cnew;
                else Cv[v] = Ctab + 36 * (int64_t)q[site_of(px + i - h, py + j - h, pz + k - h, K)];
            }
    int centre = h + n * (h + n * h);

    double* du = (double*)calloc(3 * (size_t)nnodes, sizeof(double));
    double* w = (double*)calloc(3 * (size_t)nnodes, sizeof(double));
    double* grad = (double*)malloc(sizeof(double) * 3 * (size_t)nnodes);

    for (int step = 0; step < nr; ++step) {
        memset(grad, 0, sizeof(double) * 3 * (size_t)nnodes);
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int v = i + n * (j + n * k);
                    double uc[8][3], e[6], s[6], f[8][3];
                    for (int c = 0; c < 8; ++c) {
                        int node = (i + (c & 1)) + nn * ((j + ((c >> 1) & 1)) + nn * (k + ((c >> 2) & 1)));
                        for (int d = 0; d < 3; ++d) uc[c][d] = du[3 * node + d];
                    }
                    voxel_strain(uc, e);
                    matvec6(Cv[v], e, s);
                    if (v == centre)
                        for (int I = 0; I < 6; ++I) s[I] += t[I];
                    voxel_forces(s, f);
                    for (int c = 0; c < 8; ++c) {
                        int node = (i + (c & 1)) + nn * ((j + ((c >> 1) & 1)) + nn * (k + ((c >> 2) & 1)));
                        for (int d = 0; d < 3; ++d) grad[3 * node + d] += f[c][d];
                    }
                }
        for (int a = 0; a < 3 * nnodes; ++a) {
            w[a] = beta * w[a] - alpha * grad[a];
            du[a] += w[a];
        }
    }

    double dPi = 0.5 * dot6(eps, t);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int v = i + n * (j + n * k);
                double uc[8][3], e[6], s[6];
                for (int c = 0; c < 8; ++c) {
                    int node = (i + (c & 1)) + nn * ((j + ((c >> 1) & 1)) + nn * (k + ((c >> 2) & 1)));
                    for (int d = 0; d < 3; ++d) uc[c][d] = du[3 * node + d];
                }
                voxel_strain(uc, e);
                matvec6(Cv[v], e, s);
                dPi += 0.5 * dot6(e, s);
                if (v == centre) dPi += dot6(t, e);
            }
    free(Cv);
    free(du);
    free(w);
    free(grad);
    return dPi;
}

/* The same energy change taken literally from Fig. 1 and Eq. (H_1, second form): nodal   */
/* displacements of the zone u_old = E.x + u_global, boundary loads f = the forces that  */
/* the voxels outside the zone exert on the zone's nodes, Pi(u) = sum_{v in zone}         */
/* 1/2 (B_v u).C_v (B_v u) - f.u, and dPi_A = Pi_new(u_n) - Pi_old(u_old) with u_n after  */
/* n_r heavy-ball steps on Pi_new from u_old.  Used only to check the form above.         */
double ora_zone_literal(int K, const int32_t* q, const double* Ctab, const double* u, const double* E,
                        int64_t p, int32_t q_new, int h, int nr, double alpha, double beta)
{
    int n = 2 * h + 1, nn = 2 * h + 2;
    int nv = n * n * n, nnodes = nn * nn * nn;
    int64_t n3 = (int64_t)K * K * K;
    int64_t px = p % K, py = (p / K) % K, pz = p / ((int64_t)K * K);
    int64_t x0 = px - h, y0 = py - h, z0 = pz - h;   /* lowest zone node, unwrapped */

    /* macro strain as a tensor, for the affine part E.x of the displacement */
    double Et[3][3] = {{E[0], 0.5 * E[5], 0.5 * E[4]},
                       {0.5 * E[5], E[1], 0.5 * E[3]},
                       {0.5 * E[4], 0.5 * E[3], E[2]}};
    double* uold = (double*)malloc(sizeof(double) * 3 * (size_t)nnodes);
    double* fb = (double*)calloc(3 * (size_t)nnodes, sizeof(double));
    int64_t* gnode = (int64_t*)malloc(sizeof(int64_t) * (size_t)nnodes);
    for (int c = 0; c < nn; ++c)
        for (int b = 0; b < nn; ++b)
            for (int a = 0; a < nn; ++a) {
                int node = a + nn * (b + nn * c);
                double X[3] = {(double)(x0 + a), (double)(y0 + b), (double)(z0 + c)};
                gnode[node] = site_of(x0 + a, y0 + b, z0 + c, K);
                for (int d = 0; d < 3; ++d)
                    uold[3 * node + d] = Et[d][0] * X[0] + Et[d][1] * X[1] + Et[d][2] * X[2] +
                                         u[d * n3 + gnode[node]];
            }
    /* boundary loads: forces from every voxel outside the zone that touches a zone node */
    for (int c = 0; c < nn; ++c)
        for (int b = 0; b < nn; ++b)
            for (int a = 0; a < nn; ++a) {
                int node = a + nn * (b + nn * c);
                for (int corner = 0; corner < 8; ++corner) {
                    /* voxel whose corner `corner` is this node */
                    int vi = a - (corner & 1), vj = b - ((corner >> 1) & 1), vk = c - ((corner >> 2) & 1);
                    if (vi >= 0 && vi < n && vj >= 0 && vj < n && vk >= 0 && vk < n) continue;
                    int64_t gx = x0 + vi, gy = y0 + vj, gz = z0 + vk;
                    double uc[8][3], e[6], s[6], f[8][3];
                    gather_corners(K, u, wrap(gx, K), wrap(gy, K), wrap(gz, K), uc);
                    voxel_strain(uc, e);
                    for (int I = 0; I < 6; ++I) e[I] += E[I];
                    matvec6(Ctab + 36 * (int64_t)q[site_of(gx, gy, gz, K)], e, s);
                    voxel_forces(s, f);
                    for (int d = 0; d < 3; ++d) fb[3 * node + d] -= f[corner][d];
                }
            }
    const double** Cold = (const double**)malloc(sizeof(double*) * (size_t)nv);
    const double** Cnew = (const double**)malloc(sizeof(double*) * (size_t)nv);
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int v = i + n * (j + n * k);
                Cold[v] = Ctab + 36 * (int64_t)q[site_of(x0 + i, y0 + j, z0 + k, K)];
                Cnew[v] = (i == h && j == h && k == h) ? Ctab + 36 * (int64_t)q_new : Cold[v];
            }

    double* uu = (double*)malloc(sizeof(double) * 3 * (size_t)nnodes);
    double* w = (double*)calloc(3 * (size_t)nnodes, sizeof(double));
    double* grad = (double*)malloc(sizeof(double) * 3 * (size_t)nnodes);
    memcpy(uu, uold, sizeof(double) * 3 * (size_t)nnodes);

    for (int step = 0; step <= nr; ++step) {
        int last = (step == nr);
        for (int a = 0; a < 3 * nnodes; ++a) grad[a] = -fb[a];
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int v = i + n * (j + n * k);
                    double uc[8][3], e[6], s[6], f[8][3];
                    for (int c = 0; c < 8; ++c) {
                        int node = (i + (c & 1)) + nn * ((j + ((c >> 1) & 1)) + nn * (k + ((c >> 2) & 1)));
                        for (int d = 0; d < 3; ++d) uc[c][d] = uu[3 * node + d];
                    }
                    voxel_strain(uc, e);
                    matvec6(Cnew[v], e, s);
                    voxel_forces(s, f);
                    for (int c = 0; c < 8; ++c) {
                        int node = (i + (c & 1)) + nn * ((j + ((c >> 1) & 1)) + nn * (k + ((c >> 2) & 1)));
                        for (int d = 0; d < 3; ++d) grad[3 * node + d] += f[c][d];
                    }
                }
        if (last) break;
        for (int a = 0; a < 3 * nnodes; ++a) {
            w[a] = beta * w[a] - alpha * grad[a];
            uu[a] += w[a];
        }
    }
    /* Pi_new(uu) - Pi_old(uold) */
    double Pnew = 0, Pold = 0;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int v = i + n * (j + n * k);
                double un[8][3], uo[8][3], en[6], eo[6], sn[6], so[6];
                for (int c = 0; c < 8; ++c) {
                    int node = (i + (c & 1)) + nn * ((j + ((c >> 1) & 1)) + nn * (k + ((c >> 2) & 1)));
                    for (int d = 0; d < 3; ++d) {
                        un[c][d] = uu[3 * node + d];
                        uo[c][d] = uold[3 * node + d];
                    }
                }
                voxel_strain(un, en);
                voxel_strain(uo, eo);
                matvec6(Cnew[v], en, sn);
                matvec6(Cold[v], eo, so);
                Pnew += 0.5 * dot6(en, sn);
                Pold += 0.5 * dot6(eo, so);
            }
    for (int a = 0; a < 3 * nnodes; ++a) {
        Pnew -= fb[a] * uu[a];
        Pold -= fb[a] * uold[a];
    }
    free(uold); free(fb); free(gnode); free(Cold); free(Cnew); free(uu); free(w); free(grad);
    return Pnew - Pold;
}

/* ------------------------------------------------------------------------------------ */
/* Monte Carlo trial, colour pass and sweep (Secs. 3 and 6)                             */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int32_t K, M, Q, proposal, h, nr, elastic, R, n_warm;
    int32_t pad_;
    double J, kT, lambda_el, zone_alpha, zone_beta, glob_alpha, glob_beta, glob_alphaE;
    double Sigma[6];          /* GPa */
    uint64_t seed;
} ora_params;

typedef struct {
    int32_t q_new;            /* trial state */
    int32_t gb;               /* change in unlike-bond count (energy J*gb) */
    double dPi;               /* elastic zone energy change, GPa*voxel */
    double dE;                /* total energy change, MC units */
    uint32_t r1;              /* Metropolis variate */
    int32_t flags;            /* 1: the trial changes the spin, 2: accepted */
} ora_record;

/* One trial of site `site` in sweep `sweep` against the snapshot `snap`; sigma is the
 * stored stress field (6 x K^3 component-major, GPa) or NULL when elasticity is off.
 * Accept iff dE <= 0 or r1 < 2^32 exp(-dE/kT) (Eq. metrop_1 with u = r1 / 2^32).      */
void ora_trial(const ora_params* P, const int32_t* snap, const double* Ctab, const double* Stab,
               const double* sigma, int64_t site, uint32_t sweep, ora_record* rec)
{
    uint32_t r[4];
    ora_draw(P->seed, (uint32_t)site, sweep, r);
    int32_t q_new = ora_propose(P->K, P->M, P->Q, P->proposal, snap, site, r[0]);
    rec->q_new = q_new;
    rec->r1 = r[1];
    rec->gb = 0;
    rec->dPi = 0;
    rec->dE = 0;
    rec->flags = 0;
    if (q_new == snap[site]) return;
    rec->flags = 1;
    rec->gb = ora_gb_count(P->K, P->M, snap, site, q_new);
    double dE = P->J * rec->gb;
    if (P->elastic) {
        int64_t n3 = (int64_t)P->K * P->K * P->K;
        double sp[6];
        for (int I = 0; I < 6; ++I) sp[I] = sigma[I * n3 + site];
        rec->dPi = ora_zone(P->K, snap, Ctab, Stab, site, q_new, sp, P->h, P->nr,
                            P->zone_alpha, P->zone_beta);
        dE += P->lambda_el * rec->dPi;
    }
    rec->dE = dE;
    int accept = (dE <= 0.0) || ((double)r[1] < ldexp(exp(-dE / P->kT), 32));
    if (accept) rec->flags |= 2;
}

/* One colour pass: every site of colour `colour` is tried against the state at the start
 * of the pass, and all accepted changes are written afterwards.  recs (K^3, may be
 * NULL) receives the record of each tried site at its site index.                      */
void ora_pass(const ora_params* P, int32_t* q, const double* Ctab, const double* Stab,
              const double* sigma, uint32_t sweep, int colour, ora_record* recs)
{
    int K = P->K;
    int64_t n3 = (int64_t)K * K * K;
    int32_t* snap = (int32_t*)malloc(sizeof(int32_t) * (size_t)n3);
    memcpy(snap, q, sizeof(int32_t) * (size_t)n3);
    for (int64_t z = 0; z < K; ++z)
        for (int64_t y = 0; y < K; ++y)
            for (int64_t x = 0; x < K; ++x) {
                if (ora_colour(P->M, x, y, z) != colour) continue;
                int64_t i = x + K * (y + K * z);
                ora_record rec;
                ora_trial(P, snap, Ctab, Stab, sigma, i, sweep, &rec);
                if (rec.flags & 2) q[i] = rec.q_new;
                if (recs) recs[i] = rec;
            }
    free(snap);
}

/* Trials of a subset of sites of one colour pass (for timing samples): tries sites
 * list[0..n) against `snap` and returns the number accepted.                            */
int64_t ora_trials(const ora_params* P, const int32_t* snap, const double* Ctab, const double* Stab,
                   const double* sigma, uint32_t sweep, const int64_t* list, int64_t n, ora_record* recs)
{
    int64_t acc = 0;
    for (int64_t a = 0; a < n; ++a) {
        ora_record rec;
        ora_trial(P, snap, Ctab, Stab, sigma, list[a], sweep, &rec);
        acc += (rec.flags & 2) != 0;
        if (recs) recs[a] = rec;
    }
    return acc;
}

/* n sweeps starting at sweep index s0.  With elasticity on, sweep s begins with a warm
 * refresh of the global state (u, E -> sigma) whenever s is a multiple of R.            */
void ora_sweeps(const ora_params* P, int32_t* q, const double* Ctab, const double* Stab,
                double* u, double* E, double* sigma, uint32_t s0, int n)
{
    int C = ora_num_colours(P->M);
    for (int a = 0; a < n; ++a) {
        uint32_t s = s0 + (uint32_t)a;
        if (P->elastic && P->R > 0 && (s % (uint32_t)P->R) == 0)
            ora_global(P->K, q, Ctab, Stab, P->Sigma, P->n_warm, 0, P->glob_alpha, P->glob_beta,
                       P->glob_alphaE, u, E, sigma, NULL);
        for (int c = 0; c < C; ++c) ora_pass(P, q, Ctab, Stab, P->elastic ? sigma : NULL, s, c, NULL);
    }
}

/* Gauss-Seidel sweeps at zero load (Sec. 6, the scheme the checkerboard is compared with):
 * every site in turn, x fastest, tried against the current state and updated at once.  The
 * trial of site i in sweep s uses the same draws as in the colour passes.                */
void ora_gs_sweeps(const ora_params* P, int32_t* q, uint32_t s0, int n)
{
    int64_t n3 = (int64_t)P->K * P->K * P->K;
    for (int a = 0; a < n; ++a) {
        uint32_t s = s0 + (uint32_t)a;
        for (int64_t i = 0; i < n3; ++i) {
            ora_record rec;
            ora_trial(P, q, NULL, NULL, NULL, i, s, &rec);
            if (rec.flags & 2) q[i] = rec.q_new;
        }
    }
}
