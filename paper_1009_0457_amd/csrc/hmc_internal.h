// hmc_internal.h -- shared declarations of the HIP library (host API <-> kernel launchers).
//
// Every kernel works on a table of replicas (independent lattices with their own size,
// load, temperature and Philox key) laid end to end in shared buffers.  A single-lattice
// context is a table of one; a batch fuses many replicas into each launch.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hmc.h"

namespace hmc {

// Per-grain tables on the device: the 21 distinct entries of a symmetric 6x6 Voigt matrix,
// upper triangle row by row, padded to 24 floats (96 bytes).
constexpr int kTab = 24;

__host__ __device__ constexpr int sym_index(int i, int j)
{
    return i * 6 - (i * (i - 1)) / 2 + (j - i);
}

// One entry of the compacted list of real trial flips of a colour pass.
struct TrialEntry {
    uint32_t site;     // site index within its replica
    uint32_t qr;       // q_new | replica << 16
    int32_t gb;
    uint32_t r1;
};

constexpr int kMaxReplicas = 4096;
constexpr int kSiteBlock = 256;        // nodes per block of node-parallel kernels
constexpr int kPassSites = 1024;       // active sites per chunk of a colour pass (one replica's)
constexpr int kPassSplitBelow = 1024;  // passes with fewer chunks run one site per thread
constexpr int kMaxChunkBlocks = 8192;  // blocks per replica of node-parallel reductions
constexpr int kTileX = 32, kTileY = 8;   // node tile of the explicit step in x, y
constexpr int kTileZMax = 32;            // deepest tile in z (node layers per block)

// Work-groups are dispatched to the 8 XCDs round-robin by their index, and each XCD has its
// own L2.  Launches whose neighbouring blocks share data (halo rows, neighbour planes) use
// this bijection of [0, G) as their logical block index, so that each XCD receives one
// contiguous eighth of the logical blocks and the shared rows stay in one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int G)
{
    const int x = b % kXcds, i = b / kXcds, q = G / kXcds, rm = G % kXcds;
    return x * q + (x < rm ? x : rm) + i;
}

// Logical block order of a launch: 0 the XCD-aware order above; 1 reversed; 2 a fixed shuffle
// (x -> x * 1000003 mod G, a bijection of [0, G) whenever the prime does not divide G; reversed
// when it does).  Results must not depend on it: orders 1 and 2 exist to show that no kernel
// relies on which work-group runs which part of the work, or when (hmc_set_block_order).
__device__ __forceinline__ int reorder_block(int x, int G, int order)
{
    if (order == 2 && G % 1000003 != 0) return (int)(((long long)x * 1000003LL) % (long long)G);
    if (order != 0) return G - 1 - x;
    return x;
}

__device__ __forceinline__ int logical_block(int b, int G, int order)
{
    return reorder_block(xcd_block(b, G), G, order);
}

// The same orders for grid-stride loops over a work list that may fill only part of the
// grid: order 0 keeps the dispatch index, so that the busy work-groups spread over all XCDs
// (under the XCD-aware order they would fill the first XCDs and leave the others idle).
__device__ __forceinline__ int stride_block(int b, int G, int order)
{
    return reorder_block(b, G, order);
}

// A named roctx range on the host thread for the scope's lifetime (sweeps, colour passes,
// refreshes, adjoint passes), so that a marker trace (rocprofv3 --marker-trace) shows the
// library's phases around its kernels.  Costs a call each way when no tool is attached.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

__host__ __device__ constexpr int tile_blocks_of(int K, int tz, int ty = kTileY)
{
    return ((K + kTileX - 1) / kTileX) * ((K + ty - 1) / ty) * ((K + tz - 1) / tz);
}

// Device description of one replica.
struct RepDev {
    int32_t K, Kh, Q, proposal;
    int32_t elastic;                 // elastic term on for this replica (lambda != 0, load != 0)
    int32_t tile_z;                  // node layers per block of the tiled explicit step
    int32_t tile_y;                  // node rows per block of the forward explicit step (8 or 16)
    int64_t n3;
    int64_t site_off;                // into spins / sigma / u / w planes (sites)
    int64_t grain_off;               // into Ctab / Stab (grains)
    int32_t pass_first, pass_blocks; // blocks of a colour pass (active sites / kPassSites, rounded up)
    int32_t node_first, node_blocks; // blocks of node-parallel kernels (<= kMaxChunkBlocks)
    int32_t tile_first, tile_blocks; // blocks of the tiled explicit step (32 x tile_y x tile_z nodes)
    double J, kT, lambda;
    float glob_alpha, glob_beta;
    double glob_alphaE;
    double Sigma[6];                 // applied average stress (GPa)
    uint32_t key0, key1;
};

// Slots of the per-replica device state block (doubles).
enum StateSlot {
    kE = 0,        // macroscopic strain E[6]
    kWE = 6,       // its heavy-ball velocity wE[6]
    kU = 12,       // stored energy of the last energy evaluation
    kStateDoubles = 16
};

// Stress sums of a sequence of explicit steps.  Each step adds its blocks' six sums, as
// 64-bit fixed-point integers (2^-26 GPa per voxel; integer adds commute, so the totals do not
// depend on the order the blocks finish in), into one of kSumCopies copies picked by block;
// the next step's blocks fold them into E themselves.  Three rotating buffers: the one being
// added to, the one being read, and the one being cleared for the step after.
constexpr int kSumCopies = 8;
constexpr int kSumSlots = kSumCopies * 8;      // per replica and buffer (8 int64 per copy)
constexpr double kSumScale = 67108864.0;       // 2^26
// (E, wE) of the step a sequence is at, per replica and parity: 16 doubles (E at 0, wE at 6).
constexpr int kSeqState = 16;

// Counters (uint32): list counts per colour, error flag.
enum CounterSlot { kListCount = 0, kErrFlag = 8, kLabelChanged = 9, kNonFinite = 10, kCounters = 16 };
// Bits of counters[kNonFinite], raised by kernels that meet a non-finite value and reported
// (then cleared) by the next call that synchronises the stream.
enum NonFiniteBit { kNfGlobal = 1, kNfZone = 2, kNfInjected = 4 };

// 64-bit statistics slots, kept in kStatCopies copies that blocks pick by index (fewer
// same-address atomics) and that the host sums.
enum StatSlot { kStatReal = 0, kStatSolves = 1, kStatAccepted = 2, kStatScreened = 3, kStats = 8 };
constexpr int kStatCopies = 64;
__host__ __device__ constexpr int stat_copy(unsigned block) { return (int)(block & (kStatCopies - 1)) * kStats; }

struct DeviceState {
    int16_t* spins = nullptr;        // sum of n3
    float* Ctab = nullptr;           // sum of Q, x kTab
    float* Stab = nullptr;
    float* sigma = nullptr;          // 6 planes of total sites
    float* u[2] = {nullptr, nullptr};  // 3 planes each (ping-pong)
    float* w = nullptr;              // 3 planes
    TrialEntry* list = nullptr;      // max_list
    uint8_t* accept = nullptr;       // max_list
    double* state = nullptr;         // n_rep x kStateDoubles
    double* partials = nullptr;      // total node blocks x 8
    unsigned long long* sums = nullptr;  // 3 x n_rep x kSumSlots (explicit-step stress sums)
    double* seq_state = nullptr;     // 2 x n_rep x kSeqState
    uint32_t* counters = nullptr;    // kCounters
    unsigned long long* stats = nullptr;  // kStats x kStatCopies
    uint64_t* thr = nullptr;         // n_rep x 64 integer Metropolis thresholds
    int32_t* tex_bin = nullptr;      // sum of Q
    unsigned long long* hist = nullptr;  // 64
    unsigned long long* bonds = nullptr; // 1
    RepDev* reps = nullptr;          // n_rep
    int32_t* pass_rep = nullptr;     // block -> replica for colour passes
    int32_t* node_rep = nullptr;     // block -> replica for node kernels
    int32_t* tile_rep = nullptr;     // block -> replica for the tiled explicit step
    int64_t* sweep = nullptr;        // device copy of the sweep index (Philox counter)
};

}  // namespace hmc

struct hmc_ctx_s {
    hmc_params p{};                 // common parameters (K of replica 0 for a single lattice)
    int32_t Q = 0;                  // total grains
    hipStream_t stream = nullptr;
    int device = 0;
    int n_rep = 1;
    bool is_batch = false;
    std::vector<hmc::RepDev> reps;  // host mirror of the replica table
    std::vector<int64_t> rep_euler_off;  // per replica, offset into `euler` (grains)
    int64_t total_sites = 0;
    int colours = 0;
    int64_t max_list = 0;
    int pass_blocks = 0;            // total blocks of a colour pass
    int node_blocks = 0;            // total blocks of node kernels
    int tile_blocks = 0;            // total blocks of the tiled explicit step
    bool step_streams = false;      // explicit step: own-node u and w read / written non-temporally
    bool elastic_buffers = false;
    bool have_orient = false, have_spins = false, have_load = false, have_stress = false;
    bool have_state = false;
    int cur_u = 0;
    int64_t sweep = 0;
    int64_t host_site_trials = 0;
    int64_t host_refresh_steps = 0;
    std::vector<double> euler;      // host copy of the orientations (texture bins)
    bool profiling = false;
    struct ProfPair {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<ProfPair> prof_pending;
    std::vector<hipEvent_t> prof_free;
    // captured sweeps: [0] without refresh, [1] with refresh (valid for the cur_u parity
    // recorded in graph_u)
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_u[2] = {-1, -1};
    bool use_graphs = false;
    int block_order = 0;            // hmc_set_block_order
    int adj_steps = 0, adj_every = 0;   // last hmc_elastic_forward
    // second stream (default priority) on which the adjoint's backward pass recomputes forward
    // segments while the context's stream runs adjoint steps; created on first use
    hipStream_t aux_stream = nullptr;
    hipEvent_t aux_ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hmc::DeviceState d;
    std::string err;

    bool any_elastic() const
    {
        for (const auto& r : reps)
            if (r.elastic) return true;
        return false;
    }
};

namespace hmc {

enum ProfClass { kProfPotts = 0, kProfZone, kProfApply, kProfRefreshStep, kProfRefreshOther, kProfClasses };
int prof_begin(hmc_ctx_s* c, int cls);   // returns a token (-1 when off)
// Synchronises the context's stream, reads and clears counters[kNonFinite]; HMC_ENUMERIC (with
// the context's message set) if any kernel raised it since the last report.
hmc_status report_nonfinite(hmc_ctx_s* c);
// Texture bin of each of Q grains (host, Bunge triples): floor(angle / bin_deg) clamped to
// nbins - 1, the angle between the (non-zero) lab axis and the grain's nearest crystal <100>.
void texture_bins(const double* euler, int64_t Q, const double axis[3], double bin_deg, int nbins, int32_t* bins);
// This thread's message for hmc_last_error(NULL) (calls without a context).
void set_thread_error(const char* msg);
void prof_end(hmc_ctx_s* c, int token);

// ---- launchers (each returns hipGetLastError of its launch) ----
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s);
hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t s);
hipError_t launch_convert_spins(const int32_t* in, int16_t* out, int64_t n, int32_t Q, uint32_t* err,
                                hipStream_t s);
hipError_t launch_export_spins(const int16_t* in, int32_t* out, int64_t n, hipStream_t s);
// Raises `bit` in *flag if any of the n floats at p is not finite.
hipError_t launch_check_finite(const float* p, int64_t n, uint32_t* flag, uint32_t bit, hipStream_t s);
hipError_t launch_potts_pass(hmc_ctx_s* c, int colour, hmc_trial_record* rec);
hipError_t launch_zone_pass(hmc_ctx_s* c, int colour, hmc_trial_record* rec);
hipError_t launch_apply_pass(hmc_ctx_s* c, int colour);
hipError_t launch_reuss(hmc_ctx_s* c);
hipError_t launch_global_steps(hmc_ctx_s* c, int n_steps);
// A sequence of explicit steps from the context's state (E, wE), enqueued on stream s:
// seq_begin, then seq_step for i = 0, 1, ... (each from uin to uout; E_record, if set,
// receives the step's E), then seq_end(n) with the number of steps taken, which leaves the
// context's state after them.  Profiling events are taken only on the context's stream.
hipError_t seq_begin(hmc_ctx_s* c, hipStream_t s);
hipError_t seq_step(hmc_ctx_s* c, hipStream_t s, int i, const float* uin, float* uout, double* E_record);
hipError_t seq_end(hmc_ctx_s* c, hipStream_t s, int n);
hipError_t launch_global_final(hmc_ctx_s* c, bool write_sigma);
// 2 x 2 x 2 material points per background cell (hmc_mp8.hip): n explicit steps, the final
// point stresses and stored energy.
hipError_t launch_mp8_steps(hmc_ctx_s* c, int n_steps);
// Grains of replica rep (hmc_grains.hip): per-site labels (the smallest site index of each
// face-connected cluster of equal spins) and their number; host-synchronous.
hipError_t launch_grain_labels(hmc_ctx_s* c, int rep, int32_t* labels, int64_t* n_grains, int* rounds);
hipError_t launch_mp8_final(hmc_ctx_s* c, bool write_sigma);
hipError_t launch_zero_wE(hmc_ctx_s* c);
hipError_t launch_unlike_bonds(hmc_ctx_s* c, int rep);
hipError_t launch_texture(hmc_ctx_s* c, int rep, int nbins);

}  // namespace hmc
