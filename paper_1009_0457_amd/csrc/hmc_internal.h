// hmc_internal.h -- shared declarations of the HIP library (host API <-> kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hmc.h"

namespace hmc {

// Per-grain tables on the device: the 21 distinct entries of a symmetric 6x6 Voigt matrix,
// upper triangle row by row, padded to 24 floats (96 bytes, three 32-byte sectors).
constexpr int kTab = 24;

__host__ __device__ constexpr int sym_index(int i, int j)
{
    // row-major upper triangle of a 6x6 matrix, i <= j
    return i * 6 - (i * (i - 1)) / 2 + (j - i);
}

// One entry of the compacted list of real trial flips of a colour pass.
struct TrialEntry {
    uint32_t site;
    int32_t q_new;
    int32_t gb;
    uint32_t r1;
};

// Slots of the small device state block (doubles).
enum StateSlot {
    kE = 0,        // macroscopic strain E[6]
    kWE = 6,       // its heavy-ball velocity wE[6]
    kSigma = 12,   // applied average stress (GPa)[6]
    kU = 18,       // stored energy of the last energy evaluation
    kStateDoubles = 32
};

// Counters (uint32): list counts per colour, then error flags.
enum CounterSlot {
    kListCount = 0,   // [8]
    kErrFlag = 8,
    kCounters = 16
};

// 64-bit statistics slots.
enum StatSlot { kStatReal = 0, kStatSolves = 1, kStatAccepted = 2, kStats = 8 };

constexpr int kMaxPartials = 8192;   // blocks of one reduction pass

struct DeviceState {
    int16_t* spins = nullptr;        // K^3
    float* Ctab = nullptr;           // Q x kTab
    float* Stab = nullptr;           // Q x kTab
    float* sigma = nullptr;          // 6 x K^3
    float* u[2] = {nullptr, nullptr};  // 3 x K^3 each (ping-pong)
    float* w = nullptr;              // 3 x K^3
    TrialEntry* list = nullptr;      // max_list
    uint8_t* accept = nullptr;       // max_list
    double* state = nullptr;         // kStateDoubles
    double* partials = nullptr;      // kMaxPartials x 8
    uint32_t* counters = nullptr;    // kCounters
    unsigned long long* stats = nullptr;  // kStats
    uint64_t* thr = nullptr;         // 2*M+1 integer Metropolis thresholds
    int32_t* tex_bin = nullptr;      // Q
    unsigned long long* hist = nullptr;  // 64
    unsigned long long* bonds = nullptr; // 1
};

}  // namespace hmc

struct hmc_ctx_s {
    hmc_params p{};
    int32_t Q = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    int64_t n3 = 0;
    int colours = 0;
    int64_t max_list = 0;
    bool elastic_buffers = false;   // lambda_el != 0: stress/displacement buffers exist
    bool load_nonzero = false;
    bool have_orient = false, have_spins = false, have_load = false, have_stress = false;
    bool have_state = false;        // displacement/E state initialised
    int cur_u = 0;                  // which u buffer is current
    int64_t sweep = 0;
    int64_t host_site_trials = 0;
    int64_t host_refresh_steps = 0;
    double sigma_GPa[6] = {0, 0, 0, 0, 0, 0};
    std::vector<double> euler;      // host copy of the orientations (texture bins)
    // kernel timing (hmc_set_profiling): pending event pairs per class
    bool profiling = false;
    struct ProfPair {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<ProfPair> prof_pending;
    std::vector<hipEvent_t> prof_free;
    hmc::DeviceState d;
    std::string err;
};

namespace hmc {

// ---- kernel timing classes and hooks (no-ops unless profiling is on) ----
enum ProfClass { kProfPotts = 0, kProfZone, kProfApply, kProfRefreshStep, kProfRefreshOther, kProfClasses };
int prof_begin(hmc_ctx_s* c, int cls);   // returns a token (-1 when off)
void prof_end(hmc_ctx_s* c, int token);

// ---- launchers (each returns hipGetLastError of its launch) ----
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);
hipError_t launch_convert_spins(const int32_t* in, int16_t* out, int64_t n, int32_t Q, uint32_t* err,
                                hipStream_t s);
hipError_t launch_export_spins(const int16_t* in, int32_t* out, int64_t n, hipStream_t s);
hipError_t launch_potts_pass(hmc_ctx_s* c, int colour, uint32_t sweep, hmc_trial_record* rec);
hipError_t launch_zone_pass(hmc_ctx_s* c, int colour, hmc_trial_record* rec);
hipError_t launch_apply_pass(hmc_ctx_s* c, int colour);
hipError_t launch_reuss(hmc_ctx_s* c);
hipError_t launch_global_steps(hmc_ctx_s* c, int n_steps);
hipError_t launch_global_final(hmc_ctx_s* c, bool write_sigma);
hipError_t launch_unlike_bonds(hmc_ctx_s* c);
hipError_t launch_texture(hmc_ctx_s* c, int nbins);
hipError_t launch_zero_wE(hmc_ctx_s* c);

}  // namespace hmc
