// hmc_api.hip -- host side of the C ABI declared in include/hmc.h: parameter defaults and
// validation, per-grain stiffness tables (Sec. 5), workspace carving for one lattice or a
// batch of replicas, and the order in which the kernels of a sweep are enqueued (optionally
// captured once into HIP graphs and replayed).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "hmc_internal.h"

using namespace hmc;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int colours_of(int neighbors) { return neighbors == 26 ? 8 : 2; }

// ------------------------------------------------------------------------------------
// validation
// ------------------------------------------------------------------------------------
hmc_status check_common(const hmc_params* p)
{
    if (!p) return HMC_EINVAL;
    if (p->neighbors != 6 && p->neighbors != 26) return HMC_EINVAL;
    if (p->proposal != 0 && p->proposal != 1) return HMC_EINVAL;
    if (p->zone_h < 0 || p->zone_h > 3) return HMC_EINVAL;
    if (p->zone_variant < 0 || p->zone_variant > 5 || (p->zone_variant == 2 && p->zone_h > 2) ||
        (p->zone_variant >= 3 && p->zone_h < 1))
        return HMC_EINVAL;
    if (p->zone_screen != 0 && p->zone_screen != 1) return HMC_EINVAL;
    if (p->refresh_tile_z != 0 && p->refresh_tile_z != 1 && p->refresh_tile_z != 2 && p->refresh_tile_z != 4 &&
        p->refresh_tile_z != 8 && p->refresh_tile_z != 16 && p->refresh_tile_z != 32)
        return HMC_EINVAL;
    if (p->material_points != 0 && p->material_points != 1 && p->material_points != 8) return HMC_EINVAL;
    if (p->zone_steps < 0 || p->refresh_steps < 0 || p->cold_steps < 0 || p->refresh_every < 1) return HMC_EINVAL;
    const double vals[] = {p->J, p->kT, p->C11, p->C12, p->C44, p->lambda_el, p->zone_alpha, p->zone_beta,
                           p->glob_alpha, p->glob_beta, p->glob_alphaE};
    for (double v : vals)
        if (!std::isfinite(v)) return HMC_ENUMERIC;
    if (!(p->C11 - p->C12 > 0) || !(p->C11 + 2 * p->C12 > 0) || !(p->C44 > 0)) return HMC_ENUMERIC;
    return HMC_OK;
}

// The explicit step's fixed-point stress sums (2^-26 GPa per voxel, 64-bit) hold the whole
// lattice's sum for mean stresses up to 128 GPa at K = 1024; loads are held to 50 GPa, which
// leaves room for the relaxation's overshoot.
constexpr double kMaxLoadMPa = 5.0e4;
bool load_in_range(const double s[6])
{
    for (int I = 0; I < 6; ++I)
        if (!(std::fabs(s[I]) <= kMaxLoadMPa)) return false;
    return true;
}

hmc_status check_replica(const hmc_params* p, const hmc_replica* r)
{
    if (r->K < 2 || r->K > 1024 || (r->K & 1)) return HMC_ESHAPE;
    if (r->Q < 1 || r->Q > 32767) return HMC_ESHAPE;
    if (p->proposal == 1 && r->Q < 2) return HMC_EINVAL;
    const double vals[] = {r->kT, r->lambda_el, r->glob_alpha, r->glob_beta, r->glob_alphaE, r->sigma_MPa[0],
                           r->sigma_MPa[1], r->sigma_MPa[2], r->sigma_MPa[3], r->sigma_MPa[4], r->sigma_MPa[5]};
    for (double v : vals)
        if (!std::isfinite(v)) return HMC_ENUMERIC;
    if (!(r->kT > 0)) return HMC_EINVAL;
    if (!load_in_range(r->sigma_MPa)) return HMC_EINVAL;
    if (r->lambda_el != 0.0 && r->K < 2 * p->zone_h + 2) return HMC_ESHAPE;
    if (p->material_points == 8 && r->K < 4) return HMC_ESHAPE;
    return HMC_OK;
}

hmc_replica replica_of_params(const hmc_params* p, int32_t Q)
{
    hmc_replica r{};
    r.K = p->K;
    r.Q = Q;
    r.kT = p->kT;
    r.lambda_el = p->lambda_el;
    r.glob_alpha = p->glob_alpha;
    r.glob_beta = p->glob_beta;
    r.glob_alphaE = p->glob_alphaE;
    r.seed = p->seed;
    return r;
}

// ------------------------------------------------------------------------------------
// workspace layout
// ------------------------------------------------------------------------------------
struct Layout {
    size_t spins, Ctab, Stab, sigma, u0, u1, w, list, accept, state, partials, sums, seq_state, counters, stats,
        thr, tex, hist, bonds, reps, pass_rep, node_rep, tile_rep, sweep, total;
    int64_t sites, grains, max_list;
    int pass_blocks, node_blocks, tile_blocks, tile_z, tile_y;
    bool elastic;
};

int64_t n3_of(int K) { return (int64_t)K * K * K; }

// Node layers per block of one replica's explicit step: as many z-tiles as depth t gives, made
// equal (a 100-layer lattice at t = 32 takes four tiles of 25 layers instead of 32, 32, 32 and
// 4), so that no block marches further than it has to.
int balanced_depth(int t, int K)
{
    const int n = (K + t - 1) / t;
    return (K + n - 1) / n;
}

// Node rows per block of the forward explicit step at depth tz: the tallest of 32 (1024-thread
// blocks, one per compute unit), 16 (512 threads, two) and 8 (256 threads, four) that divides
// every replica's edge and still launches at least 512 blocks; taller tiles re-read fewer halo
// rows per owned node (512^3: 1.77, 1.73 and 1.62 ms per step on 8, 16 and 32 rows; 256^3:
// 262, 250 and 231 us), but a launch short of blocks leaves compute units idle (64^3 at depth
// 2: 15.1 us per step on 256 blocks of 16 rows against 14.6 us on 512 of 8).
int tile_rows_of(int n, const hmc_replica* r, int tz)
{
    for (int ty = 32; ty >= 16; ty /= 2) {
        int64_t blocks = 0;
        bool fits = true;
        for (int i = 0; i < n && fits; ++i) {
            fits = r[i].K % ty == 0;
            blocks += tile_blocks_of(r[i].K, balanced_depth(tz, r[i].K), ty);
        }
        if (fits && blocks >= 512) return ty;
    }
    return 8;
}

// Whether the explicit step streams its own nodes' u and w past the caches: when the arrays a
// step reads and writes (u in, u out, w: 36 bytes per node, and the 2-byte grain ids) are
// more than twice the 256 MB Infinity Cache, which then keeps little of them from one step to
// the next.  Below that, ordinary accesses let the next step find much of them there.
// Measured: 128^3 (80 MB, 32 x 16 tiles) 37.0 us plain against 42.2 us non-temporal; ten 100^3
// runs (380 MB, 32 x 8 tiles) 234 against 281 us; 256^3 (640 MB) 250 against 238 us; 512^3
// 1.73 against 1.66 ms.
bool step_streams_of(int64_t sites) { return sites * 38 > (int64_t)512 << 20; }

// Node layers per block of the tiled explicit step: the caller's choice, else the deepest
// tile that still launches at least 1024 blocks of 32 x 8 nodes over all replicas (4 per
// compute unit), but 2 rather than 1 (a block's first layer is redone by
// its neighbour, which one-layer tiles pay on every layer), and 1 when no depth reaches it.
// Measured with 32 x 8 tiles: 32 at 256^3 and 512^3 (64 is within 1 %), 8 at 128^3, 2 at 64^3
// are the fastest depths there.
int tile_depth_of(const hmc_params* p, int n, const hmc_replica* r)
{
    if (p->refresh_tile_z > 0) return p->refresh_tile_z;
    for (int tz = kTileZMax; tz >= 1; tz /= 2) {
        int64_t blocks = 0;
        for (int i = 0; i < n; ++i) blocks += tile_blocks_of(r[i].K, tz, 8);
        if (blocks >= 1024) return tz > 1 ? tz : 2;
    }
    return 1;
}

Layout layout_of(const hmc_params* p, int n, const hmc_replica* r)
{
    Layout L{};
    const int C = colours_of(p->neighbors);
    L.tile_z = tile_depth_of(p, n, r);
    L.tile_y = tile_rows_of(n, r, L.tile_z);
    for (int i = 0; i < n; ++i) {
        const int64_t n3 = n3_of(r[i].K);
        L.sites += n3;
        L.grains += r[i].Q;
        L.max_list += n3 / C;
        L.pass_blocks += (int)((n3 / C + kPassSites - 1) / kPassSites);
        int64_t nb = (n3 + kSiteBlock - 1) / kSiteBlock;
        if (nb > kMaxChunkBlocks) nb = kMaxChunkBlocks;
        L.node_blocks += (int)nb;
        L.tile_blocks += tile_blocks_of(r[i].K, balanced_depth(L.tile_z, r[i].K), L.tile_y);
        L.elastic = L.elastic || r[i].lambda_el != 0.0;
    }
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const size_t S = (size_t)L.sites;
    L.spins = take(S * sizeof(int16_t));
    L.Ctab = take((size_t)L.grains * kTab * sizeof(float));
    L.Stab = take((size_t)L.grains * kTab * sizeof(float));
    L.sigma = L.elastic ? take(6 * S * sizeof(float)) : 0;
    L.u0 = L.elastic ? take(3 * S * sizeof(float)) : 0;
    L.u1 = L.elastic ? take(3 * S * sizeof(float)) : 0;
    L.w = L.elastic ? take(3 * S * sizeof(float)) : 0;
    L.list = L.elastic ? take((size_t)L.max_list * sizeof(TrialEntry)) : 0;
    L.accept = L.elastic ? take((size_t)L.max_list) : 0;
    L.state = take((size_t)n * kStateDoubles * sizeof(double));
    const int pblocks = L.node_blocks > L.tile_blocks ? L.node_blocks : L.tile_blocks;
    L.partials = take((size_t)pblocks * 8 * sizeof(double));
    L.sums = take((size_t)3 * n * kSumSlots * sizeof(unsigned long long));
    L.seq_state = take((size_t)2 * n * kSeqState * sizeof(double));
    L.counters = take(kCounters * sizeof(uint32_t));
    L.stats = take(kStats * kStatCopies * sizeof(unsigned long long));
    L.thr = take((size_t)n * 64 * sizeof(uint64_t));
    L.tex = take((size_t)L.grains * sizeof(int32_t));
    L.hist = take(64 * sizeof(unsigned long long));
    L.bonds = take(sizeof(unsigned long long));
    L.reps = take((size_t)n * sizeof(RepDev));
    L.pass_rep = take((size_t)L.pass_blocks * sizeof(int32_t));
    L.node_rep = take((size_t)L.node_blocks * sizeof(int32_t));
    L.tile_rep = take((size_t)L.tile_blocks * sizeof(int32_t));
    L.sweep = take(sizeof(int64_t));
    L.total = o;
    return L;
}

// ------------------------------------------------------------------------------------
// per-grain tables (Sec. 5)
// ------------------------------------------------------------------------------------
// Rotation A = Rz(phi1) Rx(Phi) Rz(phi2), crystal -> lab.
void bunge(const double e[3], double A[3][3])
{
    const double c1 = std::cos(e[0]), s1 = std::sin(e[0]);
    const double c = std::cos(e[1]), s = std::sin(e[1]);
    const double c2 = std::cos(e[2]), s2 = std::sin(e[2]);
    A[0][0] = c1 * c2 - s1 * c * s2;
    A[0][1] = -c1 * s2 - s1 * c * c2;
    A[0][2] = s1 * s;
    A[1][0] = s1 * c2 + c1 * c * s2;
    A[1][1] = -s1 * s2 + c1 * c * c2;
    A[1][2] = -c1 * s;
    A[2][0] = s * s2;
    A[2][1] = s * c2;
    A[2][2] = c;
}

// Lab tables by the 6x6 transformation route: with Voigt pairs (i,j) for row I and (k,l)
// for column J, T[I][J] = A_ik A_jk (k == l) or A_ik A_jl + A_il A_jk (k != l).  Stress
// transforms as sigma' = T sigma, so C' = T C T^T; engineering strain transforms with
// N = D T D^-1 (D = diag(1,1,1,2,2,2)), so S' = N S N^T with the closed-form cubic S.
void grain_tables(const double e[3], double C11, double C12, double C44, double Cl[36], double Sl[36])
{
    static const int pi[6] = {0, 1, 2, 1, 0, 0}, pj[6] = {0, 1, 2, 2, 2, 1};
    double A[3][3];
    bunge(e, A);
    double T[6][6], N[6][6];
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J) {
            const int i = pi[I], j = pj[I], k = pi[J], l = pj[J];
            const double t = (k == l) ? A[i][k] * A[j][k] : A[i][k] * A[j][l] + A[i][l] * A[j][k];
            T[I][J] = t;
            N[I][J] = t * (I >= 3 ? 2.0 : 1.0) * (J >= 3 ? 0.5 : 1.0);
        }
    const double d = (C11 - C12) * (C11 + 2.0 * C12);
    const double S11 = (C11 + C12) / d, S12 = -C12 / d, S44 = 1.0 / C44;
    double Cc[6][6] = {}, Sc[6][6] = {};
    for (int I = 0; I < 3; ++I)
        for (int J = 0; J < 3; ++J) {
            Cc[I][J] = (I == J) ? C11 : C12;
            Sc[I][J] = (I == J) ? S11 : S12;
        }
    for (int I = 3; I < 6; ++I) {
        Cc[I][I] = C44;
        Sc[I][I] = S44;
    }
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J) {
            double c = 0.0, s = 0.0;
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b) {
                    c += T[I][a] * Cc[a][b] * T[J][b];
                    s += N[I][a] * Sc[a][b] * N[J][b];
                }
            Cl[6 * I + J] = c;
            Sl[6 * I + J] = s;
        }
}

// Derivatives of the lab tables with respect to the three Euler angles (phi1, Phi, phi2):
// dA by differentiating one factor of Rz(phi1) Rx(Phi) Rz(phi2), then the product rule on
// the quadratic transformation entries and on C' = T C T^T, S' = N S N^T.
void grain_table_derivatives(const double e[3], double C11, double C12, double C44, double dCl[3][36],
                             double dSl[3][36])
{
    static const int pi[6] = {0, 1, 2, 1, 0, 0}, pj[6] = {0, 1, 2, 2, 2, 1};
    const double c1 = std::cos(e[0]), s1 = std::sin(e[0]);
    const double c = std::cos(e[1]), s = std::sin(e[1]);
    const double c2 = std::cos(e[2]), s2 = std::sin(e[2]);
    const double Rz1[3][3] = {{c1, -s1, 0}, {s1, c1, 0}, {0, 0, 1}}, dRz1[3][3] = {{-s1, -c1, 0}, {c1, -s1, 0}, {0, 0, 0}};
    const double Rx[3][3] = {{1, 0, 0}, {0, c, -s}, {0, s, c}}, dRx[3][3] = {{0, 0, 0}, {0, -s, -c}, {0, c, -s}};
    const double Rz2[3][3] = {{c2, -s2, 0}, {s2, c2, 0}, {0, 0, 1}}, dRz2[3][3] = {{-s2, -c2, 0}, {c2, -s2, 0}, {0, 0, 0}};
    auto mul3 = [](const double X[3][3], const double Y[3][3], const double Z[3][3], double out[3][3]) {
        double T[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                T[i][j] = 0;
                for (int k = 0; k < 3; ++k) T[i][j] += X[i][k] * Y[k][j];
            }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                out[i][j] = 0;
                for (int k = 0; k < 3; ++k) out[i][j] += T[i][k] * Z[k][j];
            }
    };
    double A[3][3], dA[3][3][3];
    mul3(Rz1, Rx, Rz2, A);
    mul3(dRz1, Rx, Rz2, dA[0]);
    mul3(Rz1, dRx, Rz2, dA[1]);
    mul3(Rz1, Rx, dRz2, dA[2]);
    double T[6][6], N[6][6];
    for (int I = 0; I < 6; ++I)
        for (int J = 0; J < 6; ++J) {
            const int i = pi[I], j = pj[I], k = pi[J], l = pj[J];
            const double t = (k == l) ? A[i][k] * A[j][k] : A[i][k] * A[j][l] + A[i][l] * A[j][k];
            T[I][J] = t;
            N[I][J] = t * (I >= 3 ? 2.0 : 1.0) * (J >= 3 ? 0.5 : 1.0);
        }
    const double d = (C11 - C12) * (C11 + 2.0 * C12);
    const double S11 = (C11 + C12) / d, S12 = -C12 / d, S44 = 1.0 / C44;
    double Cc[6][6] = {}, Sc[6][6] = {};
    for (int I = 0; I < 3; ++I)
        for (int J = 0; J < 3; ++J) {
            Cc[I][J] = (I == J) ? C11 : C12;
            Sc[I][J] = (I == J) ? S11 : S12;
        }
    for (int I = 3; I < 6; ++I) {
        Cc[I][I] = C44;
        Sc[I][I] = S44;
    }
    for (int q = 0; q < 3; ++q) {
        double dT[6][6], dN[6][6];
        const double (&G)[3][3] = dA[q];
        for (int I = 0; I < 6; ++I)
            for (int J = 0; J < 6; ++J) {
                const int i = pi[I], j = pj[I], k = pi[J], l = pj[J];
                const double t = (k == l) ? G[i][k] * A[j][k] + A[i][k] * G[j][k]
                                          : G[i][k] * A[j][l] + A[i][k] * G[j][l] + G[i][l] * A[j][k] + A[i][l] * G[j][k];
                dT[I][J] = t;
                dN[I][J] = t * (I >= 3 ? 2.0 : 1.0) * (J >= 3 ? 0.5 : 1.0);
            }
        for (int I = 0; I < 6; ++I)
            for (int J = 0; J < 6; ++J) {
                double vc = 0.0, vs = 0.0;
                for (int a = 0; a < 6; ++a)
                    for (int b = 0; b < 6; ++b) {
                        vc += dT[I][a] * Cc[a][b] * T[J][b] + T[I][a] * Cc[a][b] * dT[J][b];
                        vs += dN[I][a] * Sc[a][b] * N[J][b] + N[I][a] * Sc[a][b] * dN[J][b];
                    }
                dCl[q][6 * I + J] = vc;
                dSl[q][6 * I + J] = vs;
            }
    }
}

// ------------------------------------------------------------------------------------
// error helpers
// ------------------------------------------------------------------------------------
hmc_status device_fail(hmc_ctx c, hipError_t e, const char* where)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    c->err = buf;
    return HMC_EDEVICE;
}

#define HMC_TRY(ctx, expr, where)                                 \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return device_fail(ctx, e_, where); \
    } while (0)

hmc_status state_fail(hmc_ctx c, hmc_status s, const char* m)
{
    c->err = m;
    return s;
}

void drop_graphs(hmc_ctx c)
{
    for (int i = 0; i < 2; ++i) {
        if (c->graph[i]) (void)hipGraphExecDestroy(c->graph[i]);
        c->graph[i] = nullptr;
        c->graph_u[i] = -1;
    }
}

hmc_status upload_reps(hmc_ctx c)
{
    HMC_TRY(c, hipMemcpyAsync(c->d.reps, c->reps.data(), c->reps.size() * sizeof(RepDev), hipMemcpyHostToDevice,
                              c->stream),
            "replica table");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "replica table");
    drop_graphs(c);
    return HMC_OK;
}

bool elastic_on(const hmc_ctx c) { return c->elastic_buffers && c->any_elastic(); }

// ------------------------------------------------------------------------------------
// the enqueue order of a refresh and a sweep
// ------------------------------------------------------------------------------------
hmc_status refresh(hmc_ctx c, int n_steps, bool cold)
{
    TraceRange range(cold ? "hmc stress refresh (cold)" : "hmc stress refresh");
    if (c->p.material_points == 8) {
        // nodes and velocities in place in the first displacement buffer, corner forces in
        // the second
        if (cold) {
            HMC_TRY(c, launch_fill_f32(c->d.u[0], 0.f, 3 * c->total_sites, c->stream), "refresh: clear u");
            HMC_TRY(c, launch_reuss(c), "refresh: uniform-stress start");
        } else {
            HMC_TRY(c, launch_zero_wE(c), "refresh: clear wE");
        }
        HMC_TRY(c, launch_fill_f32(c->d.w, 0.f, 3 * c->total_sites, c->stream), "refresh: clear w");
        c->cur_u = 0;
        HMC_TRY(c, launch_mp8_steps(c, n_steps), "refresh: explicit steps (8 points per cell)");
        HMC_TRY(c, launch_mp8_final(c, true), "refresh: point stresses");
        c->host_refresh_steps += n_steps;
        c->have_state = true;
        c->have_stress = true;
        return HMC_OK;
    }
    if (cold) {
        HMC_TRY(c, launch_fill_f32(c->d.u[0], 0.f, 3 * c->total_sites, c->stream), "refresh: clear u");
        HMC_TRY(c, launch_fill_f32(c->d.w, 0.f, 3 * c->total_sites, c->stream), "refresh: clear w");
        c->cur_u = 0;
        HMC_TRY(c, launch_reuss(c), "refresh: uniform-stress start");
    } else {
        HMC_TRY(c, launch_fill_f32(c->d.w, 0.f, 3 * c->total_sites, c->stream), "refresh: clear w");
        HMC_TRY(c, launch_zero_wE(c), "refresh: clear wE");
    }
    HMC_TRY(c, launch_global_steps(c, n_steps), "refresh: explicit steps");
    HMC_TRY(c, launch_global_final(c, true), "refresh: stress field");
    c->host_refresh_steps += n_steps;
    c->have_state = true;
    c->have_stress = true;
    return HMC_OK;
}

hmc_status run_pass(hmc_ctx c, int colour, hmc_trial_record* rec)
{
    static const char* const kPassName[8] = {"hmc colour pass 0", "hmc colour pass 1", "hmc colour pass 2",
                                             "hmc colour pass 3", "hmc colour pass 4", "hmc colour pass 5",
                                             "hmc colour pass 6", "hmc colour pass 7"};
    TraceRange range(kPassName[colour & 7]);
    // Only trials that need a zone solve enter the colour's trial list; with the elastic term
    // off for every replica the list stays empty and its count is neither read nor written.
    const bool el = elastic_on(c);
    if (el) HMC_TRY(c, launch_fill_u32(c->d.counters + kListCount + colour, 0u, 1, c->stream), "pass: reset list");
    HMC_TRY(c, launch_potts_pass(c, colour, rec), "pass: potts");
    if (el) {
        HMC_TRY(c, launch_zone_pass(c, colour, rec), "pass: zone solves");
        HMC_TRY(c, launch_apply_pass(c, colour), "pass: apply");
    }
    c->host_site_trials += c->total_sites / c->colours;
    return HMC_OK;
}

// one sweep without host synchronisation: [refresh], colour passes, sweep index + 1
hmc_status enqueue_sweep(hmc_ctx c, bool with_refresh)
{
    TraceRange range("hmc sweep");
    if (with_refresh) {
        hmc_status st = refresh(c, c->p.refresh_steps, false);
        if (st != HMC_OK) return st;
    }
    for (int col = 0; col < c->colours; ++col) {
        hmc_status st = run_pass(c, col, nullptr);
        if (st != HMC_OK) return st;
    }
    HMC_TRY(c, launch_add_i64(c->d.sweep, 1, c->stream), "sweep: advance index");
    return HMC_OK;
}

// Replays (capturing first if needed) the graph of one sweep.  The graph is tied to the
// parity of the displacement ping-pong buffer it was captured with.
hmc_status graph_sweep(hmc_ctx c, bool with_refresh)
{
    const int k = with_refresh ? 1 : 0;
    if (!c->graph[k] || c->graph_u[k] != c->cur_u) {
        if (c->graph[k]) (void)hipGraphExecDestroy(c->graph[k]);
        c->graph[k] = nullptr;
        const int u0 = c->cur_u;
        const int64_t trials0 = c->host_site_trials, steps0 = c->host_refresh_steps;
        HMC_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal), "graph: begin capture");
        hmc_status st = enqueue_sweep(c, with_refresh);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &g);
        c->cur_u = u0;   // nothing ran yet: restore the host mirrors
        c->host_site_trials = trials0;
        c->host_refresh_steps = steps0;
        if (st != HMC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return device_fail(c, e, "graph: end capture");
        e = hipGraphInstantiate(&c->graph[k], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return device_fail(c, e, "graph: instantiate");
        c->graph_u[k] = u0;
    }
    {
        TraceRange range("hmc sweep (graph replay)");
        HMC_TRY(c, hipGraphLaunch(c->graph[k], c->stream), "graph: launch");
    }
    // mirror what the replayed sweep did
    if (with_refresh) {
        // what refresh() leaves: the 8-point solve always ends in buffer 0, the one-point
        // steps alternate the ping-pong buffers
        if (c->p.material_points == 8)
            c->cur_u = 0;
        else if (c->p.refresh_steps & 1)
            c->cur_u = 1 - c->cur_u;
        c->host_refresh_steps += c->p.refresh_steps;
        c->have_state = c->have_stress = true;
    }
    c->host_site_trials += c->total_sites;
    return HMC_OK;
}

// Message of this thread's last failed context creation (there is no context to hold it).
thread_local std::string t_create_err;

hmc_status create_fail(hmc_status st, const char* what, hipError_t e = hipSuccess)
{
    t_create_err = what;
    if (e != hipSuccess) {
        t_create_err += ": ";
        t_create_err += hipGetErrorString(e);
    }
    return st;
}

hmc_status build_context(const hmc_params* p, int n, const hmc_replica* r, void* ws, size_t ws_bytes,
                         hipStream_t stream, bool batch, hmc_ctx* out)
{
    const Layout L = layout_of(p, n, r);
    if (!ws || ((uintptr_t)ws % kAlign) != 0) return create_fail(HMC_EINVAL, "workspace null or not 256-byte aligned");
    if (ws_bytes < L.total) return create_fail(HMC_ESHAPE, "workspace smaller than the layout needs");
    hmc_ctx c = new (std::nothrow) hmc_ctx_s();
    if (!c) return create_fail(HMC_EINVAL, "out of host memory");
    c->p = *p;
    c->n_rep = n;
    c->is_batch = batch;
    c->Q = (int32_t)L.grains;
    c->stream = stream;
    if (hipError_t e = hipGetDevice(&c->device); e != hipSuccess) {
        delete c;
        return create_fail(HMC_EDEVICE, "hipGetDevice", e);
    }
    c->total_sites = L.sites;
    c->colours = colours_of(p->neighbors);
    c->max_list = L.max_list;
    c->pass_blocks = L.pass_blocks;
    c->node_blocks = L.node_blocks;
    c->tile_blocks = L.tile_blocks;
    c->step_streams = step_streams_of(L.sites);
    c->elastic_buffers = L.elastic;
    char* b = (char*)ws;
    c->d.spins = (int16_t*)(b + L.spins);
    c->d.Ctab = (float*)(b + L.Ctab);
    c->d.Stab = (float*)(b + L.Stab);
    if (L.elastic) {
        c->d.sigma = (float*)(b + L.sigma);
        c->d.u[0] = (float*)(b + L.u0);
        c->d.u[1] = (float*)(b + L.u1);
        c->d.w = (float*)(b + L.w);
        c->d.list = (TrialEntry*)(b + L.list);
        c->d.accept = (uint8_t*)(b + L.accept);
    }
    c->d.state = (double*)(b + L.state);
    c->d.partials = (double*)(b + L.partials);
    c->d.sums = (unsigned long long*)(b + L.sums);
    c->d.seq_state = (double*)(b + L.seq_state);
    c->d.counters = (uint32_t*)(b + L.counters);
    c->d.stats = (unsigned long long*)(b + L.stats);
    c->d.thr = (uint64_t*)(b + L.thr);
    c->d.tex_bin = (int32_t*)(b + L.tex);
    c->d.hist = (unsigned long long*)(b + L.hist);
    c->d.bonds = (unsigned long long*)(b + L.bonds);
    c->d.reps = (RepDev*)(b + L.reps);
    c->d.pass_rep = (int32_t*)(b + L.pass_rep);
    c->d.node_rep = (int32_t*)(b + L.node_rep);
    c->d.tile_rep = (int32_t*)(b + L.tile_rep);
    c->d.sweep = (int64_t*)(b + L.sweep);

    const int M = p->neighbors;
    const int C = c->colours;
    std::vector<uint64_t> thr((size_t)n * 64, 0);
    std::vector<int32_t> pass_rep((size_t)L.pass_blocks), node_rep((size_t)L.node_blocks),
        tile_rep((size_t)L.tile_blocks);
    int64_t site_off = 0, grain_off = 0;
    int pf = 0, nf = 0, tf = 0;
    c->reps.resize(n);
    c->rep_euler_off.resize(n);
    for (int i = 0; i < n; ++i) {
        RepDev R{};
        R.K = r[i].K;
        R.Kh = r[i].K / 2;
        R.Q = r[i].Q;
        R.proposal = p->proposal;
        R.n3 = n3_of(r[i].K);
        R.site_off = site_off;
        R.grain_off = grain_off;
        R.pass_first = pf;
        R.pass_blocks = (int)((R.n3 / C + kPassSites - 1) / kPassSites);
        R.node_first = nf;
        int64_t nb = (R.n3 + kSiteBlock - 1) / kSiteBlock;
        R.node_blocks = (int)(nb > kMaxChunkBlocks ? kMaxChunkBlocks : nb);
        R.tile_first = tf;
        R.tile_z = balanced_depth(L.tile_z, R.K);
        R.tile_y = L.tile_y;
        R.tile_blocks = tile_blocks_of(R.K, R.tile_z, R.tile_y);
        R.J = p->J;
        R.kT = r[i].kT;
        R.lambda = r[i].lambda_el;
        R.glob_alpha = (float)r[i].glob_alpha;
        R.glob_beta = (float)r[i].glob_beta;
        R.glob_alphaE = r[i].glob_alphaE;
        bool nz = false;
        for (int I = 0; I < 6; ++I) {
            R.Sigma[I] = r[i].sigma_MPa[I] * 1e-3;
            nz = nz || r[i].sigma_MPa[I] != 0.0;
        }
        R.elastic = (nz && R.lambda != 0.0) ? 1 : 0;
        R.key0 = (uint32_t)(r[i].seed & 0xffffffffu);
        R.key1 = (uint32_t)(r[i].seed >> 32);
        for (int k = 0; k < R.pass_blocks; ++k) pass_rep[(size_t)pf + k] = i;
        for (int k = 0; k < R.node_blocks; ++k) node_rep[(size_t)nf + k] = i;
        for (int k = 0; k < R.tile_blocks; ++k) tile_rep[(size_t)tf + k] = i;
        tf += R.tile_blocks;
        pf += R.pass_blocks;
        nf += R.node_blocks;
        // integer Metropolis thresholds for dE = J*gb: accept iff r1 < thr[gb + M] with
        // thr = 2^32 when dE <= 0, else ceil(2^32 exp(-dE/kT)) (the predicate r1 < 2^32 P)
        for (int g = -M; g <= M; ++g) {
            const double dE = p->J * g;
            thr[(size_t)i * 64 + g + M] =
                dE <= 0.0 ? (1ull << 32) : (uint64_t)std::ceil(std::ldexp(std::exp(-dE / R.kT), 32));
        }
        c->reps[i] = R;
        c->rep_euler_off[i] = grain_off;
        site_off += R.n3;
        grain_off += R.Q;
    }
    c->euler.assign((size_t)3 * L.grains, 0.0);
    std::vector<double> state0((size_t)n * kStateDoubles, 0.0);
    std::vector<uint32_t> ctr0(kCounters, 0u);
    std::vector<unsigned long long> st0((size_t)kStats * kStatCopies, 0ull);
    const int64_t zero = 0;
    hipError_t e = hipMemcpyAsync(c->d.thr, thr.data(), thr.size() * sizeof(uint64_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d.state, state0.data(), state0.size() * sizeof(double), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d.counters, ctr0.data(), kCounters * sizeof(uint32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d.stats, st0.data(), st0.size() * sizeof(unsigned long long), hipMemcpyHostToDevice,
                           stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d.pass_rep, pass_rep.data(), pass_rep.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d.node_rep, node_rep.data(), node_rep.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d.tile_rep, tile_rep.data(), tile_rep.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d.reps, c->reps.data(), c->reps.size() * sizeof(RepDev), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->d.sweep, &zero, sizeof zero, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
        delete c;
        return create_fail(HMC_EDEVICE, "copying the replica tables to the workspace", e);
    }
    if (e = hipStreamSynchronize(stream); e != hipSuccess) {
        delete c;
        return create_fail(HMC_EDEVICE, "synchronising the stream after set-up", e);
    }
    // batches carry their loads from creation; a single lattice gets one from hmc_set_load
    c->have_load = batch;
    *out = c;
    return HMC_OK;
}

hmc_status upload_tables(hmc_ctx c, int rep, const double* euler)
{
    const RepDev& R = c->reps[rep];
    std::vector<float> Ct((size_t)R.Q * kTab, 0.f), St((size_t)R.Q * kTab, 0.f);
    for (int64_t g = 0; g < R.Q; ++g) {
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(euler[3 * g + k])) return state_fail(c, HMC_ENUMERIC, "non-finite Euler angle");
        double Cl[36], Sl[36];
        grain_tables(euler + 3 * g, c->p.C11, c->p.C12, c->p.C44, Cl, Sl);
        for (int i = 0; i < 6; ++i)
            for (int j = i; j < 6; ++j) {
                Ct[(size_t)g * kTab + sym_index(i, j)] = (float)Cl[6 * i + j];
                St[(size_t)g * kTab + sym_index(i, j)] = (float)Sl[6 * i + j];
            }
    }
    HMC_TRY(c, hipMemcpyAsync(c->d.Ctab + R.grain_off * kTab, Ct.data(), Ct.size() * sizeof(float),
                              hipMemcpyHostToDevice, c->stream),
            "orientations");
    HMC_TRY(c, hipMemcpyAsync(c->d.Stab + R.grain_off * kTab, St.data(), St.size() * sizeof(float),
                              hipMemcpyHostToDevice, c->stream),
            "orientations");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "orientations");
    std::memcpy(&c->euler[3 * (size_t)c->rep_euler_off[rep]], euler, sizeof(double) * 3 * (size_t)R.Q);
    return HMC_OK;
}

hmc_status upload_spins(hmc_ctx c, int rep, const int32_t* spins_dev)
{
    const RepDev& R = c->reps[rep];
    uint32_t* err = c->d.counters + kErrFlag;
    HMC_TRY(c, launch_fill_u32(err, 0u, 1, c->stream), "spins");
    HMC_TRY(c, launch_convert_spins(spins_dev, c->d.spins + R.site_off, R.n3, R.Q, err, c->stream), "spins");
    uint32_t flag = 0;
    HMC_TRY(c, hipMemcpyAsync(&flag, err, sizeof flag, hipMemcpyDeviceToHost, c->stream), "spins");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "spins");
    if (flag) return state_fail(c, HMC_EINVAL, "spin value outside [0, Q)");
    return HMC_OK;
}

hmc_status energy_of(hmc_ctx c, int rep, int64_t* unlike, double* U)
{
    if (!unlike || !U) return state_fail(c, HMC_EINVAL, "null output");
    if (!c->have_spins) return state_fail(c, HMC_ESTATE, "no spins set");
    HMC_TRY(c, hipMemsetAsync(c->d.bonds, 0, sizeof(unsigned long long), c->stream), "energy");
    HMC_TRY(c, launch_unlike_bonds(c, rep), "energy");
    unsigned long long slots = 0;
    HMC_TRY(c, hipMemcpyAsync(&slots, c->d.bonds, sizeof slots, hipMemcpyDeviceToHost, c->stream), "energy");
    double u = 0.0;
    if (c->elastic_buffers && c->have_state && c->have_orient) {
        if (c->p.material_points == 8)
            HMC_TRY(c, launch_mp8_final(c, false), "energy");
        else
            HMC_TRY(c, launch_global_final(c, false), "energy");
        HMC_TRY(c, hipMemcpyAsync(&u, c->d.state + (int64_t)rep * kStateDoubles + kU, sizeof u, hipMemcpyDeviceToHost,
                                  c->stream),
                "energy");
    }
    HMC_TRY(c, hipStreamSynchronize(c->stream), "energy");
    *unlike = (int64_t)(slots / 2);
    *U = u;
    return report_nonfinite(c);
}

hmc_status texture_of(hmc_ctx c, int rep, const double axis[3], double bin_deg, int32_t nbins, int64_t* counts)
{
    if (!axis || !counts) return state_fail(c, HMC_EINVAL, "null argument");
    if (nbins < 1 || nbins > 64 || !(bin_deg > 0) || !std::isfinite(bin_deg))
        return state_fail(c, HMC_EINVAL, "need 1 <= nbins <= 64 and bin_deg > 0");
    if (!c->have_spins || !c->have_orient) return state_fail(c, HMC_ESTATE, "no spins/orientations");
    const double nrm = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    if (!(nrm > 0) || !std::isfinite(nrm)) return state_fail(c, HMC_EINVAL, "axis must be finite and non-zero");
    const RepDev& R = c->reps[rep];
    std::vector<int32_t> bins((size_t)R.Q);
    texture_bins(&c->euler[3 * (size_t)R.grain_off], R.Q, axis, bin_deg, nbins, bins.data());
    std::vector<unsigned long long> h(64, 0ull);
    HMC_TRY(c, hipMemcpyAsync(c->d.tex_bin + R.grain_off, bins.data(), bins.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, c->stream),
            "texture");
    HMC_TRY(c, hipMemsetAsync(c->d.hist, 0, 64 * sizeof(unsigned long long), c->stream), "texture");
    HMC_TRY(c, launch_texture(c, rep, nbins), "texture");
    HMC_TRY(c, hipMemcpyAsync(h.data(), c->d.hist, 64 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream),
            "texture");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "texture");
    for (int b = 0; b < nbins; ++b) counts[b] = (int64_t)h[b];
    return report_nonfinite(c);
}

// Copies `planes` component planes of replica `rep` between a shared field and a dense
// caller array: out to `dst` when dst is given, else in from `src`.
hmc_status copy_field(hmc_ctx c, int rep, int planes, float* base, float* dst, const float* src, const char* what)
{
    const RepDev& R = c->reps[rep];
    for (int I = 0; I < planes; ++I) {
        float* fld = base + (int64_t)I * c->total_sites + R.site_off;
        float* to = dst ? dst + (int64_t)I * R.n3 : fld;
        const float* from = dst ? fld : src + (int64_t)I * R.n3;
        HMC_TRY(c, hipMemcpyAsync(to, from, R.n3 * sizeof(float), hipMemcpyDeviceToDevice, c->stream), what);
    }
    return HMC_OK;
}

bool bad_rep(hmc_ctx c, int32_t r) { return r < 0 || r >= c->n_rep; }

}  // namespace

// ------------------------------------------------------------------------------------
// kernel timing hooks
// ------------------------------------------------------------------------------------
namespace hmc {

static hipEvent_t take_event(hmc_ctx_s* c)
{
    if (!c->prof_free.empty()) {
        hipEvent_t e = c->prof_free.back();
        c->prof_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int prof_begin(hmc_ctx_s* c, int cls)
{
    if (!c->profiling) return -1;
    hipEvent_t a = take_event(c), b = take_event(c);
    if (!a || !b) return -1;
    if (hipEventRecord(a, c->stream) != hipSuccess) return -1;
    c->prof_pending.push_back({cls, a, b});
    return (int)c->prof_pending.size() - 1;
}

void prof_end(hmc_ctx_s* c, int token)
{
    if (token < 0 || token >= (int)c->prof_pending.size()) return;
    (void)hipEventRecord(c->prof_pending[token].b, c->stream);
}

void texture_bins(const double* euler, int64_t Q, const double axis[3], double bin_deg, int nbins, int32_t* bins)
{
    // angle = acos(max_m |(A^T d)_m|) between the unit axis d and the nearest crystal <100>
    const double nrm = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    for (int64_t g = 0; g < Q; ++g) {
        double A[3][3];
        bunge(euler + 3 * g, A);
        double best = 0.0;
        for (int m = 0; m < 3; ++m) {
            const double cm = (A[0][m] * axis[0] + A[1][m] * axis[1] + A[2][m] * axis[2]) / nrm;
            best = std::fmax(best, std::fabs(cm));
        }
        const double ang = std::acos(std::fmin(best, 1.0)) * (180.0 / M_PI);
        const int b = (int)std::floor(ang / bin_deg);
        bins[g] = b < nbins - 1 ? b : nbins - 1;
    }
}

void set_thread_error(const char* msg) { t_create_err = msg; }

// Reads (and clears) the device's non-finite flag.  Called by the entry points that
// synchronise the stream anyway; returns HMC_ENUMERIC with a message naming the kernels that
// met a non-finite value since the last report.
hmc_status report_nonfinite(hmc_ctx_s* c)
{
    uint32_t* dflag = c->d.counters + kNonFinite;
    uint32_t flag = 0;
    HMC_TRY(c, hipMemcpyAsync(&flag, dflag, sizeof flag, hipMemcpyDeviceToHost, c->stream), "non-finite flag");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "non-finite flag");
    if (!flag) return HMC_OK;
    HMC_TRY(c, launch_fill_u32(dflag, 0u, 1, c->stream), "non-finite flag");
    std::string m = "non-finite value met on the device:";
    if (flag & kNfInjected) m += " an injected stress field (hmc_set_stress);";
    if (flag & kNfGlobal) m += " the global solve's stress field or stored energy;";
    if (flag & kNfZone) m += " a zone solve's energy change (its trial was rejected);";
    c->err = m;
    return HMC_ENUMERIC;
}

}  // namespace hmc

// ------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------
extern "C" {

hmc_status hmc_default_params(hmc_params* p, int32_t K, int32_t neighbors, int32_t zone_h)
{
    if (!p || K < 2 || (neighbors != 6 && neighbors != 26) || zone_h < 0 || zone_h > 3) return HMC_EINVAL;
    std::memset(p, 0, sizeof *p);
    p->K = K;
    p->neighbors = neighbors;
    p->proposal = 0;
    p->zone_h = zone_h;
    p->zone_steps = zone_h <= 1 ? 50 : 200;
    p->refresh_every = 10;
    p->refresh_steps = 200;
    p->cold_steps = 2000;
    p->J = 1.0;
    p->kT = 0.5;
    p->C11 = 246.5;
    p->C12 = 147.3;
    p->C44 = 124.7;
    const double lam = std::fmax(p->C11 + 2 * p->C12, std::fmax(p->C11 - p->C12, 2 * p->C44));
    const double L = 4.0 * lam, shear = 0.5 * (p->C11 - p->C12);
    const double mu = shear / ((2.0 * zone_h + 1) * (2.0 * zone_h + 1));
    const double sl = std::sqrt(L), sm = std::sqrt(mu);
    p->zone_alpha = 4.0 / ((sl + sm) * (sl + sm));
    p->zone_beta = ((sl - sm) / (sl + sm)) * ((sl - sm) / (sl + sm));
    p->seed = 1;
    hmc_replica r;
    hmc_default_replica(&r, p, K, 1);
    p->lambda_el = r.lambda_el;
    p->glob_alpha = r.glob_alpha;
    p->glob_beta = r.glob_beta;
    p->glob_alphaE = r.glob_alphaE;
    return HMC_OK;
}

hmc_status hmc_set_material_points(hmc_params* p, int32_t n)
{
    if (!p || (n != 0 && n != 1 && n != 8) || p->K < 2) return HMC_EINVAL;
    p->material_points = n;
    hmc_replica r;
    const hmc_status st = hmc_default_replica(&r, p, p->K, 1);
    if (st != HMC_OK) return st;
    p->glob_alpha = r.glob_alpha;
    p->glob_beta = r.glob_beta;
    p->glob_alphaE = r.glob_alphaE;
    return HMC_OK;
}

hmc_status hmc_default_replica(hmc_replica* r, const hmc_params* common, int32_t K, int32_t Q)
{
    if (!r || !common || K < 2) return HMC_EINVAL;
    std::memset(r, 0, sizeof *r);
    r->K = K;
    r->Q = Q;
    r->kT = common->kT;
    // Sec. 4: lambda = 1e9 (l0/K)^3 / (2 E0), E0 = gamma_s l0^2 / (K^2 gamma*), Table 1, l0 = 1 mm
    const double l0 = 1.0e-3, gamma_s = 0.45, gamma_mc = 2.4;
    const double E0 = gamma_s * l0 * l0 / ((double)K * K) / gamma_mc;
    r->lambda_el = 1.0e9 * std::pow(l0 / K, 3) / (2.0 * E0);
    const double lam = std::fmax(common->C11 + 2 * common->C12, std::fmax(common->C11 - common->C12, 2 * common->C44));
    const bool mp8 = common->material_points == 8;
    const double L = (mp8 ? 8.0 : 4.0) * lam, shear = 0.5 * (common->C11 - common->C12);
    const double sK = 2.0 * std::sin(M_PI / (mp8 ? 0.5 * K : (double)K));
    const double sl = std::sqrt(L), sm = std::sqrt(shear * sK * sK);
    r->glob_alpha = 4.0 / ((sl + sm) * (sl + sm));
    r->glob_beta = ((sl - sm) / (sl + sm)) * ((sl - sm) / (sl + sm));
    r->glob_alphaE = r->glob_alpha;
    r->seed = common->seed;
    return HMC_OK;
}

size_t hmc_workspace_bytes(const hmc_params* p, int32_t Q)
{
    if (check_common(p) != HMC_OK) return 0;
    const hmc_replica r = replica_of_params(p, Q);
    if (check_replica(p, &r) != HMC_OK) return 0;
    return layout_of(p, 1, &r).total;
}

size_t hmc_batch_workspace_bytes(const hmc_params* common, int32_t n, const hmc_replica* reps)
{
    if (check_common(common) != HMC_OK || n < 1 || n > kMaxReplicas || !reps) return 0;
    for (int i = 0; i < n; ++i)
        if (check_replica(common, &reps[i]) != HMC_OK) return 0;
    return layout_of(common, n, reps).total;
}

hmc_status hmc_create(const hmc_params* p, int32_t Q, void* ws, size_t ws_bytes, hipStream_t stream, hmc_ctx* out)
{
    t_create_err.clear();
    if (!out) return create_fail(HMC_EINVAL, "null output handle");
    *out = nullptr;
    hmc_status st = check_common(p);
    if (st != HMC_OK) return create_fail(st, "invalid parameters");
    const hmc_replica r = replica_of_params(p, Q);
    st = check_replica(p, &r);
    if (st != HMC_OK) return create_fail(st, "invalid lattice size, grain count or physics constants");
    return build_context(p, 1, &r, ws, ws_bytes, stream, false, out);
}

hmc_status hmc_batch_create(const hmc_params* common, int32_t n, const hmc_replica* reps, void* ws, size_t ws_bytes,
                            hipStream_t stream, hmc_ctx* out)
{
    t_create_err.clear();
    if (!out) return create_fail(HMC_EINVAL, "null output handle");
    *out = nullptr;
    hmc_status st = check_common(common);
    if (st != HMC_OK) return create_fail(st, "invalid common parameters");
    if (n < 1 || n > kMaxReplicas || !reps) return create_fail(HMC_EINVAL, "replica count out of range");
    for (int i = 0; i < n; ++i) {
        st = check_replica(common, &reps[i]);
        if (st != HMC_OK) return create_fail(st, "invalid replica description");
    }
    return build_context(common, n, reps, ws, ws_bytes, stream, true, out);
}

void hmc_destroy(hmc_ctx c)
{
    if (!c) return;
    drop_graphs(c);
    for (auto& pp : c->prof_pending) {
        (void)hipEventDestroy(pp.a);
        (void)hipEventDestroy(pp.b);
    }
    for (auto e : c->prof_free) (void)hipEventDestroy(e);
    for (auto e : c->aux_ev)
        if (e) (void)hipEventDestroy(e);
    if (c->aux_stream) (void)hipStreamDestroy(c->aux_stream);
    delete c;
}

const char* hmc_last_error(hmc_ctx c) { return c ? c->err.c_str() : t_create_err.c_str(); }

hmc_status hmc_grain_tables(const double* euler, int32_t Q, double C11, double C12, double C44, double* C_out,
                            double* S_out)
{
    if (!euler || !C_out || !S_out || Q < 1) return HMC_EINVAL;
    for (int64_t g = 0; g < Q; ++g) {
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(euler[3 * g + k])) return HMC_ENUMERIC;
        grain_tables(euler + 3 * g, C11, C12, C44, C_out + 36 * g, S_out + 36 * g);
    }
    return HMC_OK;
}

hmc_status hmc_grain_table_derivatives(const double* euler, int32_t Q, double C11, double C12, double C44,
                                       double* dC_out, double* dS_out)
{
    if (!euler || !dC_out || !dS_out || Q < 1) return HMC_EINVAL;
    for (int64_t g = 0; g < Q; ++g) {
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(euler[3 * g + k])) return HMC_ENUMERIC;
        double dC[3][36], dS[3][36];
        grain_table_derivatives(euler + 3 * g, C11, C12, C44, dC, dS);
        std::memcpy(dC_out + 108 * g, dC, sizeof dC);
        std::memcpy(dS_out + 108 * g, dS, sizeof dS);
    }
    return HMC_OK;
}

hmc_status hmc_set_orientations(hmc_ctx c, const double* euler)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!euler) return state_fail(c, HMC_EINVAL, "null orientations");
    if (c->is_batch) return state_fail(c, HMC_ESTATE, "batches take orientations per replica");
    c->adj_steps = 0;   // a recorded adjoint forward no longer matches the orientations
    hmc_status st = upload_tables(c, 0, euler);
    if (st != HMC_OK) return st;
    drop_graphs(c);
    c->have_orient = true;
    c->have_stress = false;
    return HMC_OK;
}

hmc_status hmc_set_spins(hmc_ctx c, const int32_t* spins_dev)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!spins_dev) return state_fail(c, HMC_EINVAL, "null spins");
    if (c->is_batch) return state_fail(c, HMC_ESTATE, "batches take spins per replica");
    c->adj_steps = 0;
    hmc_status st = upload_spins(c, 0, spins_dev);
    c->have_spins = st == HMC_OK;
    return st;
}

hmc_status hmc_get_spins(hmc_ctx c, int32_t* spins_dev) { return hmc_batch_get_spins(c, 0, spins_dev); }

hmc_status hmc_set_load(hmc_ctx c, const double sigma_MPa[6])
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!sigma_MPa) return state_fail(c, HMC_EINVAL, "null load");
    for (int I = 0; I < 6; ++I)
        if (!std::isfinite(sigma_MPa[I])) return state_fail(c, HMC_ENUMERIC, "non-finite load");
    if (!load_in_range(sigma_MPa)) return state_fail(c, HMC_EINVAL, "load component beyond 5e4 MPa");
    c->adj_steps = 0;
    for (auto& R : c->reps) {
        bool nz = false;
        for (int I = 0; I < 6; ++I) {
            R.Sigma[I] = sigma_MPa[I] * 1e-3;
            nz = nz || sigma_MPa[I] != 0.0;
        }
        R.elastic = (nz && R.lambda != 0.0) ? 1 : 0;
    }
    hmc_status st = upload_reps(c);
    if (st != HMC_OK) return st;
    c->have_load = true;
    c->have_stress = false;
    return HMC_OK;
}

hmc_status hmc_stress_refresh(hmc_ctx c, int32_t n_steps, int32_t cold_start)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!c->elastic_buffers) return state_fail(c, HMC_ESTATE, "elastic term disabled (lambda_el == 0)");
    if (!c->have_orient || !c->have_spins || !c->have_load)
        return state_fail(c, HMC_ESTATE, "refresh needs orientations, spins and a load");
    if (!cold_start && !c->have_state) return state_fail(c, HMC_ESTATE, "warm refresh without a prior state");
    if (n_steps < 0) n_steps = cold_start ? c->p.cold_steps : c->p.refresh_steps;
    return refresh(c, n_steps, cold_start != 0);
}

hmc_status hmc_sweep(hmc_ctx c, int32_t n_sweeps)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (n_sweeps < 0) return state_fail(c, HMC_EINVAL, "negative sweep count");
    if (!c->have_orient || !c->have_spins) return state_fail(c, HMC_ESTATE, "sweep needs orientations and spins");
    const bool el = elastic_on(c);
    if (el && !c->have_stress) return state_fail(c, HMC_ESTATE, "elastic sweep needs a stress field (refresh first)");
    const bool graphs = c->use_graphs && !c->profiling && c->stream != nullptr;
    if (n_sweeps > 0) c->adj_steps = 0;   // spins change
    for (int32_t a = 0; a < n_sweeps; ++a) {
        const int64_t s = c->sweep;
        const bool with_refresh = el && (s % c->p.refresh_every) == 0 && c->p.refresh_steps > 0;
        hmc_status st = graphs ? graph_sweep(c, with_refresh) : enqueue_sweep(c, with_refresh);
        if (st != HMC_OK) return st;
        c->sweep = s + 1;
    }
    return HMC_OK;
}

hmc_status hmc_set_graphs(hmc_ctx c, int32_t enable)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (enable && c->stream == nullptr) return state_fail(c, HMC_EINVAL, "graph capture needs a non-null stream");
    c->use_graphs = enable != 0;
    if (!c->use_graphs) drop_graphs(c);
    return HMC_OK;
}

hmc_status hmc_colour_pass(hmc_ctx c, int32_t colour, hmc_trial_record* rec)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (colour < 0 || colour >= c->colours) return state_fail(c, HMC_EINVAL, "colour out of range");
    if (!c->have_orient || !c->have_spins) return state_fail(c, HMC_ESTATE, "pass needs orientations and spins");
    if (elastic_on(c) && !c->have_stress) return state_fail(c, HMC_ESTATE, "elastic pass needs a stress field");
    c->adj_steps = 0;   // spins change
    return run_pass(c, colour, rec);
}

hmc_status hmc_energy(hmc_ctx c, int64_t* unlike, double* U) { return hmc_batch_energy(c, 0, unlike, U); }

hmc_status hmc_texture_histogram(hmc_ctx c, const double axis[3], double bin_deg, int32_t nbins, int64_t* counts)
{
    return hmc_batch_texture_histogram(c, 0, axis, bin_deg, nbins, counts);
}

hmc_status hmc_get_stress(hmc_ctx c, float* out) { return hmc_batch_get_stress(c, 0, out); }

hmc_status hmc_set_stress(hmc_ctx c, const float* in)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!in) return state_fail(c, HMC_EINVAL, "null input");
    if (!c->elastic_buffers) return state_fail(c, HMC_ESTATE, "elastic term disabled (lambda_el == 0)");
    if (c->is_batch) return state_fail(c, HMC_ESTATE, "not available on batches");
    hmc_status st = copy_field(c, 0, 6, c->d.sigma, nullptr, in, "set_stress");
    if (st != HMC_OK) return st;
    HMC_TRY(c, launch_check_finite(c->d.sigma, 6 * c->total_sites, c->d.counters + kNonFinite, kNfInjected, c->stream),
            "set_stress");
    c->have_stress = true;
    return HMC_OK;
}

hmc_status hmc_get_displacement(hmc_ctx c, float* out)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!out) return state_fail(c, HMC_EINVAL, "null output");
    if (!c->elastic_buffers || !c->have_state) return state_fail(c, HMC_ESTATE, "no elastic state");
    if (c->p.material_points == 8) return state_fail(c, HMC_ESTATE, "displacements live on the coarse mesh");
    return copy_field(c, 0, 3, c->d.u[c->cur_u], out, nullptr, "get_displacement");
}

hmc_status hmc_get_macro_strain(hmc_ctx c, double E[6])
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!E) return state_fail(c, HMC_EINVAL, "null output");
    if (!c->elastic_buffers || !c->have_state) return state_fail(c, HMC_ESTATE, "no elastic state");
    double tmp[6];
    HMC_TRY(c, hipMemcpyAsync(tmp, c->d.state + kE, sizeof tmp, hipMemcpyDeviceToHost, c->stream), "get_macro_strain");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "get_macro_strain");
    std::memcpy(E, tmp, sizeof tmp);
    return report_nonfinite(c);
}

hmc_status hmc_set_elastic_state(hmc_ctx c, const float* u_dev, const double E_host[6])
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!u_dev || !E_host) return state_fail(c, HMC_EINVAL, "null argument");
    if (!c->elastic_buffers) return state_fail(c, HMC_ESTATE, "elastic term disabled (lambda_el == 0)");
    if (c->is_batch) return state_fail(c, HMC_ESTATE, "not available on batches");
    if (c->p.material_points == 8) return state_fail(c, HMC_ESTATE, "displacements live on the coarse mesh");
    for (int I = 0; I < 6; ++I)
        if (!std::isfinite(E_host[I])) return state_fail(c, HMC_ENUMERIC, "non-finite strain");
    double st[12];
    for (int I = 0; I < 6; ++I) {
        st[I] = E_host[I];
        st[6 + I] = 0.0;
    }
    c->cur_u = 0;
    drop_graphs(c);
    hmc_status s = copy_field(c, 0, 3, c->d.u[0], nullptr, u_dev, "set_elastic_state");
    if (s != HMC_OK) return s;
    HMC_TRY(c, hipMemcpyAsync(c->d.state + kE, st, sizeof st, hipMemcpyHostToDevice, c->stream), "set_elastic_state");
    HMC_TRY(c, launch_fill_f32(c->d.w, 0.f, 3 * c->total_sites, c->stream), "set_elastic_state");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "set_elastic_state");
    c->have_state = true;
    return HMC_OK;
}

hmc_status hmc_set_sweep_index(hmc_ctx c, int64_t s)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (s < 0) return state_fail(c, HMC_EINVAL, "negative sweep index");
    HMC_TRY(c, launch_set_i64(c->d.sweep, s, c->stream), "set_sweep_index");
    c->sweep = s;
    return HMC_OK;
}

hmc_status hmc_get_sweep_index(hmc_ctx c, int64_t* s)
{
    if (!c || !s) return HMC_EINVAL;
    *s = c->sweep;
    return HMC_OK;
}

hmc_status hmc_get_stats(hmc_ctx c, hmc_stats* out)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!out) return state_fail(c, HMC_EINVAL, "null output");
    unsigned long long all[kStats * kStatCopies];
    HMC_TRY(c, hipMemcpyAsync(all, c->d.stats, sizeof all, hipMemcpyDeviceToHost, c->stream), "get_stats");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "get_stats");
    unsigned long long s[kStats] = {};
    for (int k = 0; k < kStatCopies; ++k)
        for (int i = 0; i < kStats; ++i) s[i] += all[k * kStats + i];
    out->site_trials = c->host_site_trials;
    out->real_flips = (int64_t)s[kStatReal];
    out->zone_solves = (int64_t)s[kStatSolves];
    out->accepted = (int64_t)s[kStatAccepted];
    out->screened = (int64_t)s[kStatScreened];
    out->refresh_steps = c->host_refresh_steps;
    return report_nonfinite(c);
}

hmc_status hmc_reset_stats(hmc_ctx c)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    HMC_TRY(c, hipMemsetAsync(c->d.stats, 0, kStats * kStatCopies * sizeof(unsigned long long), c->stream),
            "reset_stats");
    c->host_site_trials = 0;
    c->host_refresh_steps = 0;
    return HMC_OK;
}

hmc_status hmc_set_zone_screen(hmc_ctx c, int32_t enable)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (enable != 0 && enable != 1) return state_fail(c, HMC_EINVAL, "enable must be 0 or 1");
    c->p.zone_screen = enable;
    drop_graphs(c);
    return HMC_OK;
}

hmc_status hmc_set_zone_variant(hmc_ctx c, int32_t variant)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    hmc_params q = c->p;
    q.zone_variant = variant;
    if (check_common(&q) != HMC_OK) return state_fail(c, HMC_EINVAL, "zone variant not allowed for this zone size");
    c->p.zone_variant = variant;
    drop_graphs(c);
    return HMC_OK;
}

hmc_status hmc_set_block_order(hmc_ctx c, int32_t order)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (order < 0 || order > 2) return state_fail(c, HMC_EINVAL, "block order must be 0, 1 or 2");
    c->block_order = order;
    drop_graphs(c);
    return HMC_OK;
}

hmc_status hmc_set_profiling(hmc_ctx c, int32_t enable)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    c->profiling = enable != 0;
    return HMC_OK;
}

hmc_status hmc_get_kernel_times(hmc_ctx c, hmc_kernel_times* out)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!out) return state_fail(c, HMC_EINVAL, "null output");
    std::memset(out, 0, sizeof *out);
    hmc_kernel_time* slot[kProfClasses] = {&out->potts, &out->zone, &out->apply, &out->refresh_step,
                                           &out->refresh_other};
    HMC_TRY(c, hipStreamSynchronize(c->stream), "get_kernel_times");
    for (auto& pp : c->prof_pending) {
        float ms = 0.f;
        HMC_TRY(c, hipEventElapsedTime(&ms, pp.a, pp.b), "get_kernel_times");
        slot[pp.cls]->launches += 1;
        slot[pp.cls]->total_ms += ms;
        c->prof_free.push_back(pp.a);
        c->prof_free.push_back(pp.b);
    }
    c->prof_pending.clear();
    return HMC_OK;
}

// ---- batches ----

hmc_status hmc_batch_set_replica(hmc_ctx c, int32_t r, const double* euler_host, const int32_t* spins_dev)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (bad_rep(c, r) || !euler_host || !spins_dev) return state_fail(c, HMC_EINVAL, "bad replica or null input");
    c->adj_steps = 0;
    hmc_status st = upload_tables(c, r, euler_host);
    if (st != HMC_OK) return st;
    st = upload_spins(c, r, spins_dev);
    if (st != HMC_OK) return st;
    drop_graphs(c);
    c->have_orient = c->have_spins = true;
    c->have_stress = false;
    return HMC_OK;
}

hmc_status hmc_batch_get_spins(hmc_ctx c, int32_t r, int32_t* spins_dev)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (bad_rep(c, r) || !spins_dev) return state_fail(c, HMC_EINVAL, "bad replica or null output");
    if (!c->have_spins) return state_fail(c, HMC_ESTATE, "no spins set");
    const RepDev& R = c->reps[r];
    HMC_TRY(c, launch_export_spins(c->d.spins + R.site_off, spins_dev, R.n3, c->stream), "get_spins");
    return HMC_OK;
}

hmc_status hmc_batch_get_stress(hmc_ctx c, int32_t r, float* dev_out)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (bad_rep(c, r) || !dev_out) return state_fail(c, HMC_EINVAL, "bad replica or null output");
    if (!c->elastic_buffers || !c->have_stress) return state_fail(c, HMC_ESTATE, "no stress field");
    return copy_field(c, r, 6, c->d.sigma, dev_out, nullptr, "get_stress");
}

hmc_status hmc_batch_energy(hmc_ctx c, int32_t r, int64_t* unlike, double* U)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (bad_rep(c, r)) return state_fail(c, HMC_EINVAL, "bad replica");
    return energy_of(c, r, unlike, U);
}

hmc_status hmc_grain_labels(hmc_ctx c, int32_t r, int32_t* labels_dev, int64_t* n_grains)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (bad_rep(c, r) || !labels_dev || !n_grains) return state_fail(c, HMC_EINVAL, "bad replica or null argument");
    if (!c->have_spins) return state_fail(c, HMC_ESTATE, "no spins set");
    int rounds = 0;
    HMC_TRY(c, launch_grain_labels(c, r, labels_dev, n_grains, &rounds), "grain labels");
    return HMC_OK;
}

hmc_status hmc_batch_texture_histogram(hmc_ctx c, int32_t r, const double axis[3], double bin_deg, int32_t nbins,
                                       int64_t* counts)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (bad_rep(c, r)) return state_fail(c, HMC_EINVAL, "bad replica");
    return texture_of(c, r, axis, bin_deg, nbins, counts);
}

}  // extern "C"
