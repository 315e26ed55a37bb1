// hmc_api.hip -- host side of the C ABI declared in include/hmc.h: parameter defaults and
// validation, the per-grain stiffness tables (Sec. 5), workspace carving, and the order in
// which the kernels of a sweep are enqueued.
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

struct Layout {
    size_t spins, Ctab, Stab, sigma, u0, u1, w, list, accept, state, partials, counters, stats, thr, tex, hist,
        bonds, total;
};

int colours_of(int neighbors) { return neighbors == 26 ? 8 : 2; }

hmc_status check_params(const hmc_params* p, int32_t Q, std::string* why)
{
    auto fail = [&](hmc_status s, const char* m) {
        if (why) *why = m;
        return s;
    };
    if (!p) return fail(HMC_EINVAL, "null parameters");
    if (p->neighbors != 6 && p->neighbors != 26) return fail(HMC_EINVAL, "neighbors must be 6 or 26");
    if (p->K < 2 || p->K > 1024 || (p->K & 1)) return fail(HMC_ESHAPE, "K must be even and in [2, 1024]");
    if (Q < 1 || Q > 32767) return fail(HMC_ESHAPE, "Q must be in [1, 32767]");
    if (p->proposal != 0 && p->proposal != 1) return fail(HMC_EINVAL, "proposal must be 0 or 1");
    if (p->proposal == 1 && Q < 2) return fail(HMC_EINVAL, "uniform proposal needs Q >= 2");
    if (p->zone_h < 0 || p->zone_h > 3) return fail(HMC_EINVAL, "zone_h must be in [0, 3]");
    if (p->zone_steps < 0 || p->refresh_steps < 0 || p->cold_steps < 0 || p->refresh_every < 1)
        return fail(HMC_EINVAL, "negative step counts or refresh_every < 1");
    const double vals[] = {p->J, p->kT, p->C11, p->C12, p->C44, p->lambda_el, p->zone_alpha, p->zone_beta,
                           p->glob_alpha, p->glob_beta, p->glob_alphaE};
    for (double v : vals)
        if (!std::isfinite(v)) return fail(HMC_ENUMERIC, "non-finite parameter");
    if (!(p->kT > 0)) return fail(HMC_EINVAL, "kT must be positive");
    if (!(p->C11 - p->C12 > 0) || !(p->C11 + 2 * p->C12 > 0) || !(p->C44 > 0))
        return fail(HMC_ENUMERIC, "cubic constants are not positive definite");
    if (p->lambda_el != 0.0 && p->K < 2 * p->zone_h + 2)
        return fail(HMC_ESHAPE, "K must be at least 2h+2 with the elastic term on");
    return HMC_OK;
}

Layout layout_of(const hmc_params* p, int32_t Q)
{
    Layout L{};
    const size_t n3 = (size_t)p->K * p->K * p->K;
    const int C = colours_of(p->neighbors);
    const bool el = p->lambda_el != 0.0;
    const size_t max_list = n3 / C;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.spins = take(n3 * sizeof(int16_t));
    L.Ctab = take((size_t)Q * kTab * sizeof(float));
    L.Stab = take((size_t)Q * kTab * sizeof(float));
    L.sigma = el ? take(6 * n3 * sizeof(float)) : 0;
    L.u0 = el ? take(3 * n3 * sizeof(float)) : 0;
    L.u1 = el ? take(3 * n3 * sizeof(float)) : 0;
    L.w = el ? take(3 * n3 * sizeof(float)) : 0;
    L.list = el ? take(max_list * sizeof(TrialEntry)) : 0;
    L.accept = el ? take(max_list) : 0;
    L.state = take(kStateDoubles * sizeof(double));
    L.partials = take((size_t)kMaxPartials * 8 * sizeof(double));
    L.counters = take(kCounters * sizeof(uint32_t));
    L.stats = take(kStats * sizeof(unsigned long long));
    L.thr = take(64 * sizeof(uint64_t));
    L.tex = take((size_t)Q * sizeof(int32_t));
    L.hist = take(64 * sizeof(unsigned long long));
    L.bonds = take(sizeof(unsigned long long));
    L.total = o;
    return L;
}

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

hmc_status device_fail(hmc_ctx c, hipError_t e, const char* where)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    c->err = buf;
    return HMC_EDEVICE;
}

#define HMC_TRY(ctx, expr, where)                              \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return device_fail(ctx, e_, where); \
    } while (0)

hmc_status state_fail(hmc_ctx c, hmc_status s, const char* m)
{
    c->err = m;
    return s;
}

bool elastic_on(const hmc_ctx c) { return c->elastic_buffers && c->load_nonzero; }

hmc_status refresh(hmc_ctx c, int n_steps, bool cold)
{
    if (cold) {
        HMC_TRY(c, launch_fill_f32(c->d.u[0], 0.f, 3 * c->n3, c->stream), "refresh: clear u");
        HMC_TRY(c, launch_fill_f32(c->d.w, 0.f, 3 * c->n3, c->stream), "refresh: clear w");
        c->cur_u = 0;
        HMC_TRY(c, launch_reuss(c), "refresh: uniform-stress start");
    } else {
        HMC_TRY(c, launch_fill_f32(c->d.w, 0.f, 3 * c->n3, c->stream), "refresh: clear w");
        HMC_TRY(c, launch_zero_wE(c), "refresh: clear wE");
    }
    HMC_TRY(c, launch_global_steps(c, n_steps), "refresh: explicit steps");
    HMC_TRY(c, launch_global_final(c, true), "refresh: stress field");
    c->host_refresh_steps += n_steps;
    c->have_state = true;
    c->have_stress = true;
    return HMC_OK;
}

hmc_status run_pass(hmc_ctx c, int colour, uint32_t sweep, hmc_trial_record* rec)
{
    HMC_TRY(c, launch_fill_u32(c->d.counters + kListCount + colour, 0u, 1, c->stream), "pass: reset list");
    HMC_TRY(c, launch_potts_pass(c, colour, sweep, rec), "pass: potts");
    if (elastic_on(c)) {
        HMC_TRY(c, launch_zone_pass(c, colour, rec), "pass: zone solves");
        HMC_TRY(c, launch_apply_pass(c, colour), "pass: apply");
    }
    c->host_site_trials += c->n3 / c->colours;
    return HMC_OK;
}

}  // namespace

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

}  // namespace hmc

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
    // Sec. 4: lambda = 1e9 (l0/K)^3 / (2 E0), E0 = gamma_s l0^2 / (K^2 gamma*), Table 1
    const double l0 = 1.0e-3, gamma_s = 0.45, gamma_mc = 2.4;
    const double E0 = gamma_s * l0 * l0 / ((double)K * K) / gamma_mc;
    p->lambda_el = 1.0e9 * std::pow(l0 / K, 3) / (2.0 * E0);
    const double lam = std::fmax(p->C11 + 2 * p->C12, std::fmax(p->C11 - p->C12, 2 * p->C44));
    const double L = 4.0 * lam, shear = 0.5 * (p->C11 - p->C12);
    auto polyak = [&](double mu, double* a, double* b) {
        const double sl = std::sqrt(L), sm = std::sqrt(mu);
        *a = 4.0 / ((sl + sm) * (sl + sm));
        *b = ((sl - sm) / (sl + sm)) * ((sl - sm) / (sl + sm));
    };
    polyak(shear / ((2.0 * zone_h + 1) * (2.0 * zone_h + 1)), &p->zone_alpha, &p->zone_beta);
    const double sK = 2.0 * std::sin(M_PI / K);
    polyak(shear * sK * sK, &p->glob_alpha, &p->glob_beta);
    p->glob_alphaE = p->glob_alpha;
    p->seed = 1;
    return HMC_OK;
}

size_t hmc_workspace_bytes(const hmc_params* p, int32_t Q)
{
    if (check_params(p, Q, nullptr) != HMC_OK) return 0;
    return layout_of(p, Q).total;
}

hmc_status hmc_create(const hmc_params* p, int32_t Q, void* ws, size_t ws_bytes, hipStream_t stream, hmc_ctx* out)
{
    if (!out) return HMC_EINVAL;
    *out = nullptr;
    hmc_status st = check_params(p, Q, nullptr);
    if (st != HMC_OK) return st;
    const Layout L = layout_of(p, Q);
    if (!ws || ((uintptr_t)ws % kAlign) != 0) return HMC_EINVAL;
    if (ws_bytes < L.total) return HMC_ESHAPE;
    hmc_ctx c = new (std::nothrow) hmc_ctx_s();
    if (!c) return HMC_EINVAL;
    c->p = *p;
    c->Q = Q;
    c->stream = stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return HMC_EDEVICE;
    }
    c->n3 = (int64_t)p->K * p->K * p->K;
    c->colours = colours_of(p->neighbors);
    c->max_list = c->n3 / c->colours;
    c->elastic_buffers = p->lambda_el != 0.0;
    char* b = (char*)ws;
    c->d.spins = (int16_t*)(b + L.spins);
    c->d.Ctab = (float*)(b + L.Ctab);
    c->d.Stab = (float*)(b + L.Stab);
    if (c->elastic_buffers) {
        c->d.sigma = (float*)(b + L.sigma);
        c->d.u[0] = (float*)(b + L.u0);
        c->d.u[1] = (float*)(b + L.u1);
        c->d.w = (float*)(b + L.w);
        c->d.list = (TrialEntry*)(b + L.list);
        c->d.accept = (uint8_t*)(b + L.accept);
    }
    c->d.state = (double*)(b + L.state);
    c->d.partials = (double*)(b + L.partials);
    c->d.counters = (uint32_t*)(b + L.counters);
    c->d.stats = (unsigned long long*)(b + L.stats);
    c->d.thr = (uint64_t*)(b + L.thr);
    c->d.tex_bin = (int32_t*)(b + L.tex);
    c->d.hist = (unsigned long long*)(b + L.hist);
    c->d.bonds = (unsigned long long*)(b + L.bonds);

    // integer Metropolis thresholds for dE = J*gb: accept iff r1 < thr[gb + M] where
    // thr = 2^32 when dE <= 0, else ceil(2^32 exp(-dE/kT)) (same predicate as r1 < 2^32 P)
    const int M = p->neighbors;
    std::vector<uint64_t> thr(64, 0);
    for (int g = -M; g <= M; ++g) {
        const double dE = p->J * g;
        uint64_t t;
        if (dE <= 0.0) t = 1ull << 32;
        else t = (uint64_t)std::ceil(std::ldexp(std::exp(-dE / p->kT), 32));
        thr[g + M] = t;
    }
    std::vector<double> state0(kStateDoubles, 0.0);
    std::vector<uint32_t> ctr0(kCounters, 0u);
    std::vector<unsigned long long> st0(kStats, 0ull);
    hipError_t e = hipMemcpyAsync(c->d.thr, thr.data(), 64 * sizeof(uint64_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d.state, state0.data(), kStateDoubles * sizeof(double), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d.counters, ctr0.data(), kCounters * sizeof(uint32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d.stats, st0.data(), kStats * sizeof(unsigned long long), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        delete c;
        return HMC_EDEVICE;
    }
    *out = c;
    return HMC_OK;
}

void hmc_destroy(hmc_ctx c)
{
    if (!c) return;
    for (auto& pp : c->prof_pending) {
        (void)hipEventDestroy(pp.a);
        (void)hipEventDestroy(pp.b);
    }
    for (auto e : c->prof_free) (void)hipEventDestroy(e);
    delete c;
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

const char* hmc_last_error(hmc_ctx c) { return c ? c->err.c_str() : "null context"; }

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

hmc_status hmc_set_orientations(hmc_ctx c, const double* euler)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!euler) return state_fail(c, HMC_EINVAL, "null orientations");
    std::vector<float> Ct((size_t)c->Q * kTab, 0.f), St((size_t)c->Q * kTab, 0.f);
    for (int64_t g = 0; g < c->Q; ++g) {
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
    HMC_TRY(c, hipMemcpyAsync(c->d.Ctab, Ct.data(), Ct.size() * sizeof(float), hipMemcpyHostToDevice, c->stream),
            "set_orientations");
    HMC_TRY(c, hipMemcpyAsync(c->d.Stab, St.data(), St.size() * sizeof(float), hipMemcpyHostToDevice, c->stream),
            "set_orientations");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "set_orientations");
    c->euler.assign(euler, euler + 3 * (size_t)c->Q);
    c->have_orient = true;
    c->have_stress = false;
    return HMC_OK;
}

hmc_status hmc_set_spins(hmc_ctx c, const int32_t* spins_dev)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!spins_dev) return state_fail(c, HMC_EINVAL, "null spins");
    uint32_t* err = c->d.counters + kErrFlag;
    HMC_TRY(c, launch_fill_u32(err, 0u, 1, c->stream), "set_spins");
    HMC_TRY(c, launch_convert_spins(spins_dev, c->d.spins, c->n3, c->Q, err, c->stream), "set_spins");
    uint32_t flag = 0;
    HMC_TRY(c, hipMemcpyAsync(&flag, err, sizeof flag, hipMemcpyDeviceToHost, c->stream), "set_spins");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "set_spins");
    if (flag) {
        c->have_spins = false;
        return state_fail(c, HMC_EINVAL, "spin value outside [0, Q)");
    }
    c->have_spins = true;
    return HMC_OK;
}

hmc_status hmc_get_spins(hmc_ctx c, int32_t* spins_dev)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!spins_dev) return state_fail(c, HMC_EINVAL, "null output");
    if (!c->have_spins) return state_fail(c, HMC_ESTATE, "no spins set");
    HMC_TRY(c, launch_export_spins(c->d.spins, spins_dev, c->n3, c->stream), "get_spins");
    return HMC_OK;
}

hmc_status hmc_set_load(hmc_ctx c, const double sigma_MPa[6])
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!sigma_MPa) return state_fail(c, HMC_EINVAL, "null load");
    bool nz = false;
    for (int I = 0; I < 6; ++I) {
        if (!std::isfinite(sigma_MPa[I])) return state_fail(c, HMC_ENUMERIC, "non-finite load");
        c->sigma_GPa[I] = sigma_MPa[I] * 1e-3;
        nz = nz || sigma_MPa[I] != 0.0;
    }
    c->load_nonzero = nz;
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
    for (int32_t a = 0; a < n_sweeps; ++a) {
        const int64_t s = c->sweep;
        if (el && (s % c->p.refresh_every) == 0 && c->p.refresh_steps > 0) {
            hmc_status st = refresh(c, c->p.refresh_steps, false);
            if (st != HMC_OK) return st;
        }
        for (int col = 0; col < c->colours; ++col) {
            hmc_status st = run_pass(c, col, (uint32_t)s, nullptr);
            if (st != HMC_OK) return st;
        }
        c->sweep = s + 1;
    }
    return HMC_OK;
}

hmc_status hmc_colour_pass(hmc_ctx c, int32_t colour, hmc_trial_record* rec)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (colour < 0 || colour >= c->colours) return state_fail(c, HMC_EINVAL, "colour out of range");
    if (!c->have_orient || !c->have_spins) return state_fail(c, HMC_ESTATE, "pass needs orientations and spins");
    if (elastic_on(c) && !c->have_stress) return state_fail(c, HMC_ESTATE, "elastic pass needs a stress field");
    return run_pass(c, colour, (uint32_t)c->sweep, rec);
}

hmc_status hmc_energy(hmc_ctx c, int64_t* unlike, double* U)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!unlike || !U) return state_fail(c, HMC_EINVAL, "null output");
    if (!c->have_spins) return state_fail(c, HMC_ESTATE, "no spins set");
    HMC_TRY(c, hipMemsetAsync(c->d.bonds, 0, sizeof(unsigned long long), c->stream), "energy");
    HMC_TRY(c, launch_unlike_bonds(c), "energy");
    unsigned long long slots = 0;
    HMC_TRY(c, hipMemcpyAsync(&slots, c->d.bonds, sizeof slots, hipMemcpyDeviceToHost, c->stream), "energy");
    double u = 0.0;
    if (c->elastic_buffers && c->have_state && c->have_orient) {
        HMC_TRY(c, launch_global_final(c, false), "energy");
        HMC_TRY(c, hipMemcpyAsync(&u, c->d.state + kU, sizeof u, hipMemcpyDeviceToHost, c->stream), "energy");
    }
    HMC_TRY(c, hipStreamSynchronize(c->stream), "energy");
    *unlike = (int64_t)(slots / 2);
    *U = u;
    return HMC_OK;
}

hmc_status hmc_texture_histogram(hmc_ctx c, const double axis[3], double bin_deg, int32_t nbins, int64_t* counts)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!axis || !counts) return state_fail(c, HMC_EINVAL, "null argument");
    if (nbins < 1 || nbins > 64 || !(bin_deg > 0) || !std::isfinite(bin_deg))
        return state_fail(c, HMC_EINVAL, "need 1 <= nbins <= 64 and bin_deg > 0");
    if (!c->have_spins || !c->have_orient) return state_fail(c, HMC_ESTATE, "no spins/orientations");
    const double nrm = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    if (!(nrm > 0) || !std::isfinite(nrm)) return state_fail(c, HMC_EINVAL, "axis must be finite and non-zero");
    // per-grain bin on the host: angle = acos(max_m |(A^T d)_m|) between the axis d and the
    // nearest crystal <100>
    std::vector<int32_t> bins((size_t)c->Q);
    for (int64_t g = 0; g < c->Q; ++g) {
        double A[3][3];
        bunge(&c->euler[3 * g], A);
        double best = 0.0;
        for (int m = 0; m < 3; ++m) {
            const double cm = (A[0][m] * axis[0] + A[1][m] * axis[1] + A[2][m] * axis[2]) / nrm;
            best = std::fmax(best, std::fabs(cm));
        }
        const double ang = std::acos(std::fmin(best, 1.0)) * (180.0 / M_PI);
        const int b = (int)std::floor(ang / bin_deg);
        bins[g] = b < nbins - 1 ? b : nbins - 1;
    }
    std::vector<unsigned long long> h(64, 0ull);
    HMC_TRY(c, hipMemcpyAsync(c->d.tex_bin, bins.data(), bins.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream),
            "texture");
    HMC_TRY(c, hipMemsetAsync(c->d.hist, 0, 64 * sizeof(unsigned long long), c->stream), "texture");
    HMC_TRY(c, launch_texture(c, nbins), "texture");
    HMC_TRY(c, hipMemcpyAsync(h.data(), c->d.hist, 64 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream),
            "texture");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "texture");
    for (int b = 0; b < nbins; ++b) counts[b] = (int64_t)h[b];
    return HMC_OK;
}

hmc_status hmc_get_stress(hmc_ctx c, float* out)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!out) return state_fail(c, HMC_EINVAL, "null output");
    if (!c->elastic_buffers || !c->have_stress) return state_fail(c, HMC_ESTATE, "no stress field");
    HMC_TRY(c, hipMemcpyAsync(out, c->d.sigma, 6 * c->n3 * sizeof(float), hipMemcpyDeviceToDevice, c->stream),
            "get_stress");
    return HMC_OK;
}

hmc_status hmc_set_stress(hmc_ctx c, const float* in)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!in) return state_fail(c, HMC_EINVAL, "null input");
    if (!c->elastic_buffers) return state_fail(c, HMC_ESTATE, "elastic term disabled (lambda_el == 0)");
    HMC_TRY(c, hipMemcpyAsync(c->d.sigma, in, 6 * c->n3 * sizeof(float), hipMemcpyDeviceToDevice, c->stream),
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
    HMC_TRY(c, hipMemcpyAsync(out, c->d.u[c->cur_u], 3 * c->n3 * sizeof(float), hipMemcpyDeviceToDevice, c->stream),
            "get_displacement");
    return HMC_OK;
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
    return HMC_OK;
}

hmc_status hmc_set_elastic_state(hmc_ctx c, const float* u_dev, const double E_host[6])
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (!u_dev || !E_host) return state_fail(c, HMC_EINVAL, "null argument");
    if (!c->elastic_buffers) return state_fail(c, HMC_ESTATE, "elastic term disabled (lambda_el == 0)");
    for (int I = 0; I < 6; ++I)
        if (!std::isfinite(E_host[I])) return state_fail(c, HMC_ENUMERIC, "non-finite strain");
    double st[12];
    for (int I = 0; I < 6; ++I) {
        st[I] = E_host[I];
        st[6 + I] = 0.0;
    }
    c->cur_u = 0;
    HMC_TRY(c, hipMemcpyAsync(c->d.u[0], u_dev, 3 * c->n3 * sizeof(float), hipMemcpyDeviceToDevice, c->stream),
            "set_elastic_state");
    HMC_TRY(c, hipMemcpyAsync(c->d.state + kE, st, sizeof st, hipMemcpyHostToDevice, c->stream), "set_elastic_state");
    HMC_TRY(c, launch_fill_f32(c->d.w, 0.f, 3 * c->n3, c->stream), "set_elastic_state");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "set_elastic_state");
    c->have_state = true;
    return HMC_OK;
}

hmc_status hmc_set_sweep_index(hmc_ctx c, int64_t s)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    if (s < 0) return state_fail(c, HMC_EINVAL, "negative sweep index");
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
    unsigned long long s[kStats];
    HMC_TRY(c, hipMemcpyAsync(s, c->d.stats, sizeof s, hipMemcpyDeviceToHost, c->stream), "get_stats");
    HMC_TRY(c, hipStreamSynchronize(c->stream), "get_stats");
    out->site_trials = c->host_site_trials;
    out->real_flips = (int64_t)s[kStatReal];
    out->zone_solves = (int64_t)s[kStatSolves];
    out->accepted = (int64_t)s[kStatAccepted];
    out->refresh_steps = c->host_refresh_steps;
    return HMC_OK;
}

hmc_status hmc_reset_stats(hmc_ctx c)
{
    if (!c) return HMC_EINVAL;
    c->err.clear();
    HMC_TRY(c, hipMemsetAsync(c->d.stats, 0, kStats * sizeof(unsigned long long), c->stream), "reset_stats");
    c->host_site_trials = 0;
    c->host_refresh_steps = 0;
    return HMC_OK;
}

}  // extern "C"
