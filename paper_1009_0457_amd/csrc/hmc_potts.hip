// hmc_potts.hip -- colour-pass kernels of the Potts sweep (Sec. 3 Eqs. H_1 and metrop_1,
// Sec. 6 checkerboard with deferred updates) and small utility kernels.
//
// Four sites of the active colour class per thread.  Every trial draws its two Philox
// words and forms the trial state; the real flips (new state differs) are compacted per
// wavefront, count the change of unlike neighbour bonds and either decide at once (elastic
// term off: exact integer threshold table) or go to a compacted list for the zone-solve
// kernel (elastic term on).  Because no two sites of one class are neighbours, the
// decide-at-once path may write spins in place: every read of the pass touches other
// classes only.
#include "hmc_internal.h"

namespace hmc {

// ------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds; in each, the first and
// third words are multiplied by fixed odd constants, the high halves are mixed with the
// other two words and the key, and the key is advanced by the golden-ratio Weyl steps.
// ------------------------------------------------------------------------------------
struct Philox4 {
    uint32_t v[4];
};

// a ^ b ^ k in one instruction (gfx950's three-input bitwise op with truth table 0x96; the
// compiler emits two XORs for it); k is the round key, uniform across the wavefront.
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product gives both halves (a single v_mad_u64_u32)
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t a = (uint32_t)pa, ah = (uint32_t)(pa >> 32);
        const uint32_t b = (uint32_t)pb, bh = (uint32_t)(pb >> 32);
        const uint32_t n0 = xor3_key(bh, c1, k0);
        const uint32_t n2 = xor3_key(ah, c3, k1);
        c0 = n0;
        c1 = b;
        c2 = n2;
        c3 = a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Philox4 out;
    out.v[0] = c0;
    out.v[1] = c1;
    out.v[2] = c2;
    out.v[3] = c3;
    return out;
}

__device__ __forceinline__ int wrapi(int a, int K) { return a < 0 ? a + K : (a >= K ? a - K : a); }

struct PassArgs {
    int16_t* spins;                 // all replicas, end to end
    const RepDev* reps;
    const int32_t* pass_rep;        // block -> replica
    const uint64_t* thr;            // per replica: 64 integer thresholds indexed by gb + M
    TrialEntry* list;
    uint32_t* list_count;
    hmc_trial_record* rec;          // indexed by site_off + site, or null
    unsigned long long* stats;
    const int64_t* sweep;           // Philox counter word 1 (low 32 bits)
    const float* Stab;              // compliance tables (lower-bound screen)
    const float* sigma;             // stress planes of `plane` floats (lower-bound screen)
    int64_t plane;
    int colour;
    int screen;
    int order;                      // logical block order (hmc_set_block_order)
};

// Point-zone energy 1/2 sigma.(S_old - S_new) sigma of the trial site: a lower bound of the
// zone energy change for every zone size.
__device__ __forceinline__ double point_zone_energy(const float* __restrict__ So, const float* __restrict__ Sn,
                                                    const float s[6])
{
    double d = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) {
            const int k = sym_index(i, j);
            const double w = (i == j ? 0.5 : 1.0) * (double)s[i] * (double)s[j];
            d += w * ((double)So[k] - (double)Sn[k]);
        }
    return d;
}

// 2-bit fields, for n = 0..26, of n % 3 (which = 0), (n / 3) % 3 (1) and n / 9 (2).
constexpr uint64_t slot_field_table(int which)
{
    uint64_t t = 0;
    for (int n = 0; n < 27; ++n) {
        const int v = which == 0 ? n % 3 : which == 1 ? (n / 3) % 3 : n / 9;
        t |= (uint64_t)v << (2 * n);
    }
    return t;
}

// Offset of neighbour slot k.  6: -x,+x,-y,+y,-z,+z.  26: (dz,dy,dx) lexicographic over
// {-1,0,1}^3 without the centre (n = k or k + 1 past the centre; the digits of n in base 3
// read from three constant bit tables, which a variable k turns into two shifts and masks).
template <int M>
__device__ __forceinline__ void slot_offset(int k, int& dx, int& dy, int& dz)
{
    if (M == 6) {
        dx = (k == 0) ? -1 : (k == 1 ? 1 : 0);
        dy = (k == 2) ? -1 : (k == 3 ? 1 : 0);
        dz = (k == 4) ? -1 : (k == 5 ? 1 : 0);
    } else {
        constexpr uint64_t TX = slot_field_table(0), TY = slot_field_table(1), TZ = slot_field_table(2);
        const int sh = 2 * (k + (k >= 13));
        dx = (int)((TX >> sh) & 3u) - 1;
        dy = (int)((TY >> sh) & 3u) - 1;
        dz = (int)((TZ >> sh) & 3u) - 1;
    }
}

// Active index t of a colour class, kept as (i, j, k): i counts the class's sites along x
// (K/2 of them), j along y (K/2 for 26 neighbours, K for 6), k along z.  One division pair
// places a thread's first site; its later sites, 256 indices apart, are reached by adding the
// per-block constants 256 / (K/2) and 256 % (K/2) with carries, so the per-site cost is a
// few adds instead of two integer divisions.
struct ActiveWalk {
    uint32_t i, j, k;
};

__device__ __forceinline__ ActiveWalk walk_start(uint32_t t, uint32_t Kh, uint32_t NJ)
{
    ActiveWalk w;
    const uint32_t row = t / Kh;
    w.i = t - row * Kh;
    w.k = row / NJ;
    w.j = row - w.k * NJ;
    return w;
}

__device__ __forceinline__ void walk_advance(ActiveWalk& w, uint32_t Kh, uint32_t NJ, uint32_t di, uint32_t dr)
{
    w.i += di;
    uint32_t rows = dr;
    if (w.i >= Kh) {
        w.i -= Kh;
        rows += 1;
    }
    w.j += rows;
    if (w.j >= NJ) {
        const uint32_t c = w.j / NJ;
        w.k += c;
        w.j -= c * NJ;
    }
}

template <int M>
__device__ __forceinline__ void walk_site(const ActiveWalk& w, int colour, int& x, int& y, int& z)
{
    if (M == 26) {
        x = 2 * (int)w.i + (colour & 1);
        y = 2 * (int)w.j + ((colour >> 1) & 1);
        z = 2 * (int)w.k + ((colour >> 2) & 1);
    } else {
        y = (int)w.j;
        z = (int)w.k;
        x = 2 * (int)w.i + ((y + z + colour) & 1);
    }
}

// Linear site index; every factor fits 24 bits for K <= 1024, so full-rate 24-bit multiplies.
__device__ __forceinline__ uint32_t site_of(int x, int y, int z, int K, int KK)
{
    return (uint32_t)x + __umul24((uint32_t)K, (uint32_t)y) + __umul24((uint32_t)KK, (uint32_t)z);
}

// Block-wide exclusive prefix sum of v (256 threads), with the block total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t& total)
{
    __shared__ uint32_t s_w[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t n = __shfl_up(inc, off);
        if (lane >= off) inc += n;
    }
    if (lane == 63) s_w[wid] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wid; ++w) before += s_w[w];
    total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
    return before + inc - v;
}

// Block-wide sums of two counts (256 threads), valid in thread 0.
__device__ __forceinline__ void block_sum2(uint32_t& a, uint32_t& b)
{
    __shared__ uint32_t s_a[4], s_b[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
    }
    if (lane == 0) {
        s_a[wid] = a;
        s_b[wid] = b;
    }
    __syncthreads();
    a = s_a[0] + s_a[1] + s_a[2] + s_a[3];
    b = s_b[0] + s_b[1] + s_b[2] + s_b[3];
}

// A chunk of kPassSites = 4 x 256 active sites belongs to one replica.  With SPT = 4 one
// block covers a chunk and each thread takes four sites, 256 apart; with SPT = 1 four blocks
// share a chunk, one site per thread (the same sites and draws, a quarter each).  Lattices
// with few chunks per pass (128^3 with 8 colours has 256) take SPT = 1 at zero load: four
// times the wavefronts to hide the chain of dependent reads of a site.  Phase 1 draws every trial and
// keeps only the real flips (q_new != q_old), which each wavefront compacts through LDS; phase
// 2 -- the 26 neighbour reads, the decision or the screen -- then takes the block's real flips
// as one list, 256 at a time, so that it runs once per 64 real flips of the block instead of
// once per site slot (inside grains most proposals are no-ops, and a single real flip would
// otherwise hold a whole wavefront): on large lattices a block of 1024 sites usually has fewer
// than 64, and three of its four wavefronts skip phase 2.  A colour pass has tens of
// thousands of blocks on large lattices, so the block appends its elastic trials with one
// atomic on the list counter and adds its statistics to one of the spread counter copies.
static_assert(kPassSites == 4 * 256, "a chunk is four sites per thread of a 256-thread block");
// SCREEN: the lower-bound screen's FP64 path is compiled in only where it is used, since it
// more than doubles the kernel's registers (126 against 48 VGPRs: 4 against 8 wavefronts per
// SIMD, which hide the chain of dependent reads of every site).
// NP2: every replica proposes a neighbour's spin and has a power-of-two edge, known at compile
// time (the common case), so the proposal and the wrap need no uniform branches.
template <int M, bool SCREEN, int SPT, bool NP2>
__global__ __launch_bounds__(256) void k_potts_pass(PassArgs a)
{
    static_assert(SPT == 1 || SPT == 4, "one or four sites per thread");
    constexpr int SUB = kPassSites / (256 * SPT);    // blocks per chunk
    __shared__ uint32_t s_item[4][SPT * 64][3];      // per wavefront: coords, q_old | q_new << 16, r1
    const int lb = logical_block((int)blockIdx.x, (int)gridDim.x, a.order);   // neighbouring rows share an L2
    const int chunk = lb / SUB, sub = lb % SUB;
    const int r = a.pass_rep[chunk];
    const RepDev R = a.reps[r];
    const uint32_t first =
        (uint32_t)(chunk - R.pass_first) * (uint32_t)kPassSites + (uint32_t)sub * 256u + threadIdx.x;
    const uint32_t n_active = (uint32_t)(R.n3 / (M == 26 ? 8 : 2));
    const bool elastic = R.elastic != 0;
    int16_t* spins = a.spins + R.site_off;
    const int K = R.K, KK = K * K, Km = K - 1;
    const bool pow2 = NP2 || (K & Km) == 0;
    const bool nbr_prop = NP2 || R.proposal == 0;
    const uint32_t sweep = (uint32_t)(*a.sweep);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const unsigned long long below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    uint32_t n_real = 0, n_other = 0, n_wave = 0;
    const uint32_t Kh = (uint32_t)R.Kh, NJ = (M == 26) ? Kh : (uint32_t)K;
    const uint32_t di = 256u % Kh, dr = 256u / Kh;
    ActiveWalk walk = walk_start(first, Kh, NJ);

    // ---- phase 1: draws, proposals; real flips to the wavefront's list ----
    // In three stages, so that all of a thread's spin reads are in flight together: the sites
    // and their draws (arithmetic only), then every own and proposed-neighbour spin read, then
    // the decisions and the list appends.
    uint32_t site[SPT], packed[SPT], nbr[SPT], r0[SPT], r1[SPT];
    bool ok[SPT];
#pragma unroll
    for (int it = 0; it < SPT; ++it) {
        if (it > 0) walk_advance(walk, Kh, NJ, di, dr);
        ok[it] = first + (uint32_t)it * 256u < n_active;
        int x, y, z;
        walk_site<M>(walk, a.colour, x, y, z);
        site[it] = site_of(x, y, z, K, KK);
        packed[it] = (uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20);
        const Philox4 rn = philox4x32_10(site[it], sweep, 0u, 0u, R.key0, R.key1);
        r0[it] = rn.v[0];
        r1[it] = rn.v[1];
        nbr[it] = site[it];
        if (nbr_prop) {
            const int k = (int)__umulhi(rn.v[0], (uint32_t)M);
            int dx, dy, dz;
            slot_offset<M>(k, dx, dy, dz);
            if (pow2)   // uniform branch: a power-of-two edge wraps by a mask
                nbr[it] = site_of((x + dx) & Km, (y + dy) & Km, (z + dz) & Km, K, KK);
            else
                nbr[it] = site_of(wrapi(x + dx, K), wrapi(y + dy, K), wrapi(z + dz, K), K, KK);
        }
    }
    int q_old[SPT], q_nb[SPT];
    const char* sb = reinterpret_cast<const char*>(spins);
#pragma unroll
    for (int it = 0; it < SPT; ++it) {
        q_old[it] = 0;
        q_nb[it] = 0;
        if (ok[it]) {
            q_old[it] = *reinterpret_cast<const int16_t*>(sb + 2u * site[it]);
            q_nb[it] = *reinterpret_cast<const int16_t*>(sb + 2u * nbr[it]);
        }
    }
#pragma unroll
    for (int it = 0; it < SPT; ++it) {
        bool real = false;
        uint32_t qq = 0;
        if (ok[it]) {
            int q_new = q_nb[it];
            if (!nbr_prop) {
                const uint32_t step = __umulhi(r0[it], (uint32_t)(R.Q - 1));
                q_new = (int)(((uint32_t)q_old[it] + 1u + step) % (uint32_t)R.Q);
            }
            real = (q_new != q_old[it]);
            qq = (uint32_t)q_old[it] | ((uint32_t)q_new << 16);
            if (!real && a.rec) {
                hmc_trial_record rc;
                rc.q_new = q_new;
                rc.gb = 0;
                rc.dPi = 0.0f;
                rc.r1 = r1[it];
                rc.flags = 0;
                rc.reserved = 0;
                a.rec[R.site_off + site[it]] = rc;
            }
        }
        const unsigned long long m = __ballot(real);
        if (real) {
            const uint32_t j = n_wave + (uint32_t)__popcll(m & below);
            s_item[wid][j][0] = packed[it];
            s_item[wid][j][1] = qq;
            s_item[wid][j][2] = r1[it];
        }
        n_wave += (uint32_t)__popcll(m);
        n_real += real ? 1u : 0u;
    }
    __shared__ uint32_t s_nw[4];
    if (lane == 0) s_nw[wid] = n_wave;
    __syncthreads();
    // the four wavefronts' lists, read as one list of the block's real flips
    const uint32_t c0 = s_nw[0], c1 = c0 + s_nw[1], c2 = c1 + s_nw[2], n_block = c2 + s_nw[3];

    // ---- phase 2: the block's real flips, 256 at a time (wavefronts past the end skip it) ----
    TrialEntry ent[SPT];
    bool solve[SPT];
    uint32_t n_solve = 0;
#pragma unroll
    for (int it = 0; it < SPT; ++it) {
        const uint32_t j = (uint32_t)(it * 256) + threadIdx.x;
        solve[it] = false;
        if (j < n_block) {
            const int wv = (j >= c0) + (j >= c1) + (j >= c2);
            const uint32_t jj = j - (wv == 0 ? 0u : wv == 1 ? c0 : wv == 2 ? c1 : c2);
            const uint32_t packed = s_item[wv][jj][0], qq = s_item[wv][jj][1], r1 = s_item[wv][jj][2];
            const int x = (int)(packed & 1023u), y = (int)((packed >> 10) & 1023u), z = (int)(packed >> 20);
            const int q_old = (int)(qq & 0xffffu), q_new = (int)(qq >> 16);
            const uint32_t site = site_of(x, y, z, K, KK);
            // byte offsets of the three x, y and z planes around the site (2 bytes per spin;
            // 2 K^3 <= 2^31 for K <= 1024): each neighbour is one add and a load off the
            // replica's spin base
            const uint32_t K2 = 2u * (uint32_t)K, KK2 = 2u * (uint32_t)KK;
            const uint32_t xs[3] = {2u * (uint32_t)wrapi(x - 1, K), 2u * (uint32_t)x, 2u * (uint32_t)wrapi(x + 1, K)};
            const uint32_t ys[3] = {(uint32_t)__umul24((uint32_t)wrapi(y - 1, K), K2),
                                    (uint32_t)__umul24((uint32_t)y, K2),
                                    (uint32_t)__umul24((uint32_t)wrapi(y + 1, K), K2)};
            const uint32_t zs[3] = {(uint32_t)__umul24((uint32_t)wrapi(z - 1, K), KK2),
                                    (uint32_t)__umul24((uint32_t)z, KK2),
                                    (uint32_t)__umul24((uint32_t)wrapi(z + 1, K), KK2)};
            const char* sb = reinterpret_cast<const char*>(spins);
            int gb = 0;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                int dx, dy, dz;
                slot_offset<M>(k, dx, dy, dz);
                const int qn = *reinterpret_cast<const int16_t*>(sb + (xs[dx + 1] + ys[dy + 1] + zs[dz + 1]));
                gb += (qn == q_old) - (qn == q_new);
            }
            bool accepted = false, screened = false;
            if (!elastic) {
                accepted = (uint64_t)r1 < a.thr[(int64_t)r * 64 + gb + M];
            } else if (SCREEN && r1 != 0u) {
                // reject without a solve when even the lowest possible zone energy loses:
                // dE >= J gb + lambda dPi_0 > max(0, E*(r1)) + margin
                float sp[6];
#pragma unroll
                for (int I = 0; I < 6; ++I) sp[I] = a.sigma[(int64_t)I * a.plane + R.site_off + site];
                const float* So = a.Stab + (R.grain_off + q_old) * kTab;
                const float* Sn = a.Stab + (R.grain_off + q_new) * kTab;
                const double lo = R.J * (double)gb + R.lambda * point_zone_energy(So, Sn, sp);
                const double estar = -R.kT * log((double)r1 * 2.3283064365386963e-10);
                double W = 0.0;   // stored-energy scale of the site for the margin
#pragma unroll
                for (int i = 0; i < 6; ++i)
#pragma unroll
                    for (int jj = i; jj < 6; ++jj)
                        W += (i == jj ? 0.5 : 1.0) * (double)sp[i] * (double)sp[jj] *
                             fabs((double)So[sym_index(i, jj)]);
                const double margin = 1e-4 * fabs(R.lambda) * W + 1e-9 * (1.0 + fabs(lo));
                screened = lo > fmax(0.0, estar) + margin;
            }
            if (a.rec) {
                hmc_trial_record rc;
                rc.q_new = q_new;
                rc.gb = gb;
                rc.dPi = 0.0f;
                rc.r1 = r1;
                rc.flags = 1 | (accepted ? 2 : 0) | (screened ? 8 : 0);
                rc.reserved = 0;
                a.rec[R.site_off + site] = rc;
            }
            // same-colour sites are never neighbours: nothing else in this pass reads `site`
            if (accepted) spins[site] = (int16_t)q_new;
            solve[it] = elastic && !screened;
            ent[it].site = site;
            ent[it].qr = (uint32_t)q_new | ((uint32_t)r << 16);
            ent[it].gb = gb;
            ent[it].r1 = r1;
            n_solve += solve[it] ? 1u : 0u;
            n_other += (elastic ? screened : accepted) ? 1u : 0u;
        }
    }
    // block-collective tail, reached by every thread (`elastic` is uniform over the block: a
    // block belongs to one replica; at zero load nothing enters the list)
    uint32_t off = 0;
    __shared__ uint32_t s_base;
    if (elastic) {
        uint32_t total = 0;
        off = block_exclusive_scan(n_solve, total);
        if (threadIdx.x == 0) s_base = total ? atomicAdd(a.list_count, total) : 0u;
    }
    block_sum2(n_real, n_other);   // (its barrier also publishes s_base)
    if (threadIdx.x == 0) {
        unsigned long long* st = a.stats + stat_copy(blockIdx.x);
        if (n_real) atomicAdd(&st[kStatReal], (unsigned long long)n_real);
        if (n_other) atomicAdd(&st[elastic ? kStatScreened : kStatAccepted], (unsigned long long)n_other);
    }
    if (elastic) {
        off += s_base;
#pragma unroll
        for (int it = 0; it < SPT; ++it)
            if (solve[it]) a.list[off++] = ent[it];
    }
}

// Deferred update of an elastic pass: every accepted entry writes its new state.
__global__ __launch_bounds__(256) void k_apply(int16_t* spins, const RepDev* reps, const TrialEntry* list,
                                               const uint8_t* acc, const uint32_t* count)
{
    const uint32_t n = *count;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x)
        if (acc[e]) {
            const TrialEntry t = list[e];
            spins[reps[t.qr >> 16].site_off + t.site] = (int16_t)(t.qr & 0xffffu);
        }
}

__global__ void k_set_i64(int64_t* p, int64_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_add_i64(int64_t* p, int64_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p += v;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_f32(float* p, float v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_convert_spins(const int32_t* in, int16_t* out, int64_t n, int32_t Q, uint32_t* err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = in[i];
        if (v < 0 || v >= Q) {
            atomicOr(err, 1u);
            out[i] = 0;
        } else {
            out[i] = (int16_t)v;
        }
    }
}

__global__ void k_check_finite(const float* p, int64_t n, uint32_t* flag, uint32_t bit)
{
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bad = bad || !isfinite(p[i]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, bit);
}

__global__ void k_export_spins(const int16_t* in, int32_t* out, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

static unsigned grid_for(int64_t n, int block, unsigned cap = 65535u * 8u)
{
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > (int64_t)cap) g = cap;
    return (unsigned)g;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_convert_spins(const int32_t* in, int16_t* out, int64_t n, int32_t Q, uint32_t* err, hipStream_t s)
{
    hipLaunchKernelGGL(k_convert_spins, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, in, out, n, Q, err);
    return hipGetLastError();
}

hipError_t launch_export_spins(const int16_t* in, int32_t* out, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_export_spins, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_check_finite(const float* p, int64_t n, uint32_t* flag, uint32_t bit, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, flag, bit);
    return hipGetLastError();
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_i64, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_potts_pass(hmc_ctx_s* c, int colour, hmc_trial_record* rec)
{
    PassArgs a;
    a.spins = c->d.spins;
    a.reps = c->d.reps;
    a.pass_rep = c->d.pass_rep;
    a.thr = c->d.thr;
    a.list = c->d.list;
    a.list_count = c->d.counters + kListCount + colour;
    a.rec = rec;
    a.stats = c->d.stats;
    a.sweep = c->d.sweep;
    a.Stab = c->d.Stab;
    a.sigma = c->d.sigma;
    a.plane = c->total_sites;
    a.colour = colour;
    a.order = c->block_order;
    a.screen = (c->p.zone_screen != 0 && c->d.sigma != nullptr) ? 1 : 0;
    // one site per thread while a pass has fewer chunks than 4 per compute unit and no trial
    // enters the zone-solve list: with the list in use, four times the blocks means four times
    // the same-address list appends (measured at 128^3 under load: 16.2 against 9.6 us)
    const bool one = c->pass_blocks < kPassSplitBelow && !(c->elastic_buffers && c->any_elastic());
    const dim3 grid((unsigned)(one ? 4 * c->pass_blocks : c->pass_blocks)), block(256);
    bool np2 = true;
    for (const RepDev& R : c->reps) np2 = np2 && R.proposal == 0 && (R.K & (R.K - 1)) == 0;
    const int tok = prof_begin(c, kProfPotts);
#define HMC_PASS(MM, SC, SPT)                                                                      \
    do {                                                                                           \
        if (np2) hipLaunchKernelGGL((k_potts_pass<MM, SC, SPT, true>), grid, block, 0, c->stream, a);  \
        else hipLaunchKernelGGL((k_potts_pass<MM, SC, SPT, false>), grid, block, 0, c->stream, a);     \
    } while (0)
    if (c->p.neighbors == 26) {
        if (one) {
            if (a.screen) HMC_PASS(26, true, 1);
            else HMC_PASS(26, false, 1);
        } else {
            if (a.screen) HMC_PASS(26, true, 4);
            else HMC_PASS(26, false, 4);
        }
    } else {
        if (one) {
            if (a.screen) HMC_PASS(6, true, 1);
            else HMC_PASS(6, false, 1);
        } else {
            if (a.screen) HMC_PASS(6, true, 4);
            else HMC_PASS(6, false, 4);
        }
    }
#undef HMC_PASS
    prof_end(c, tok);
    return hipGetLastError();
}

hipError_t launch_apply_pass(hmc_ctx_s* c, int colour)
{
    const unsigned g = grid_for(c->max_list, 256, 2048);
    const int tok = prof_begin(c, kProfApply);
    hipLaunchKernelGGL(k_apply, dim3(g), dim3(256), 0, c->stream, c->d.spins, c->d.reps, c->d.list, c->d.accept,
                       c->d.counters + kListCount + colour);
    prof_end(c, tok);
    return hipGetLastError();
}

}  // namespace hmc
