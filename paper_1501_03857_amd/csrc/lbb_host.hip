// Host runtime of the lbboil C-ABI (include/lbboil.h): parameter validation,
// EOS set-up (T_c, Maxwell coexistence), device allocation, the built-in
// initial state, the step loop with captured HIP graphs, read-back,
// heat-flux bookkeeping and checkpoints.
#include "lbboil.h"

#include "lbb_device.hpp"
#include "lbb_adjoint.hpp"

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <functional>
#include <mutex>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

// Device-memory budget of the process (0: none) and the bytes the library
// holds against it.
std::atomic<int64_t> g_budget{0}, g_held{0};

// Reserve `bytes` under the budget (ENOMEM, with nothing reserved, if it would
// be exceeded); give back with release_bytes.
int reserve_bytes(int64_t bytes, const char *what)
{
    const int64_t cap = g_budget.load();
    const int64_t now = g_held.fetch_add(bytes) + bytes;
    if (cap > 0 && now > cap) {
        g_held.fetch_sub(bytes);
        return fail(LBB_ENOMEM, std::string(what) + ": " + std::to_string(bytes) + " device bytes would exceed the budget of " +
                                    std::to_string(cap) + " (" + std::to_string(now - bytes) + " held)");
    }
    return LBB_OK;
}
void release_bytes(int64_t bytes) { g_held.fetch_sub(bytes); }

#define LBB_HIP(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(LBB_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kGraphSteps = 32;  // steps per captured graph (even: buffers return)

// ---- Peng-Robinson EOS on the host (Eq. (21)) ---------------------------

struct Eos {
    double a, b, R, Tc, kappa, T;
    double alpha() const  // the temperature factor phi(T) of the attraction
    {
        const double s = 1.0 + kappa * (1.0 - std::sqrt(T / Tc));
        return s * s;
    }
    double p(double r) const { return r * R * T / (1.0 - b * r) - a * alpha() * r * r / (1.0 + 2.0 * b * r - b * b * r * r); }
    double dp(double r) const
    {
        const double q = 1.0 + 2.0 * b * r - b * b * r * r;
        return R * T / ((1.0 - b * r) * (1.0 - b * r)) - 2.0 * a * alpha() * r * (1.0 + b * r) / (q * q);
    }
    // Gibbs free energy per unit mass, up to a constant: G = F + p/rho with
    // F = int p/rho^2 drho.  The attraction term integrates through the
    // factorisation 1 + 2 b rho - b^2 rho^2 = (sqrt2 - 1 + b rho)(sqrt2 + 1 - b rho).
    // Along an isotherm dG = dp/rho (Gibbs-Duhem).
    double gibbs(double r) const
    {
        const double s2 = std::sqrt(2.0);
        const double F = R * T * std::log(r / (1.0 - b * r)) -
                         a * alpha() / (2.0 * s2 * b) * std::log((s2 - 1.0 + b * r) / (s2 + 1.0 - b * r));
        return F + p(r) / r;
    }
};

// Extremum of a function that is unimodal on [lo, hi] by golden-section
// search (sign = +1: maximum, -1: minimum).
template <typename Fn>
double golden_extremum(Fn fn, double lo, double hi, double sign)
{
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    double x1 = hi - g * (hi - lo), x2 = lo + g * (hi - lo);
    double f1 = sign * fn(x1), f2 = sign * fn(x2);
    for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
        if (f1 > f2) {
            hi = x2;
            x2 = x1;
            f2 = f1;
            x1 = hi - g * (hi - lo);
            f1 = sign * fn(x1);
        } else {
            lo = x1;
            x1 = x2;
            f1 = f2;
            x2 = lo + g * (hi - lo);
            f2 = sign * fn(x2);
        }
    }
    return 0.5 * (lo + hi);
}

// Root of fn on [lo, hi] (fn(lo), fn(hi) of opposite signs) by Newton steps
// with derivative dfn, falling back to halving the bracket whenever a step
// would leave it.
template <typename Fn, typename Dfn>
double newton_bracketed(Fn fn, Dfn dfn, double lo, double hi)
{
    const bool rising = fn(lo) < fn(hi);
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 400; ++it) {
        const double f = fn(x);
        if (f == 0.0) return x;
        if ((f > 0.0) == rising) hi = x; else lo = x;
        const double d = dfn(x);
        double xn = (d != 0.0 && std::isfinite(d)) ? x - f / d : lo - 1.0;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (std::fabs(xn - x) <= 4e-16 * std::fabs(x) || !(hi > lo)) return xn;
        x = xn;
    }
    return x;
}

// Coexisting densities by the equal-area (equal chemical potential) rule:
// p(rho_V) = p(rho_L) = p0 and G(rho_V) = G(rho_L).  The two spinodals, the
// local maximum and minimum of the van der Waals loop, lie on either side of
// the critical density rho_c = 0.0778/(Z_c b) with Z_c = 0.3074 of the
// Peng-Robinson EOS.  For a trial p0 between the loop's extremes, rho_V and
// rho_L are the outer roots of p = p0; dG/dp0 = 1/rho along each branch, so
// the difference D(p0) = G(rho_L) - G(rho_V) falls with slope
// 1/rho_L - 1/rho_V, and Newton's method on D (kept inside a sign-change
// bracket) gives the saturation pressure.
bool maxwell(const Eos &e, double &rv, double &rl)
{
    const double rmax = 1.0 / e.b;
    const double rc = 0.0778 / (0.3074 * e.b);
    auto P = [&](double r) { return e.p(r); };
    auto dP = [&](double r) { return e.dp(r); };
    const double s1 = golden_extremum(P, 0.0, rc, 1.0);          // vapour spinodal (maximum)
    const double s2 = golden_extremum(P, rc, rmax * (1.0 - 1e-9), -1.0);  // liquid spinodal (minimum)
    if (!(e.dp(0.5 * (s1 + s2)) < 0.0) || !(s1 < s2)) return false;  // no loop: T >= T_c
    double p_hi = e.p(s1);
    double p_lo = std::max(e.p(s2), 0.0);
    if (!(p_hi > p_lo)) return false;
    auto roots = [&](double p0, double &v, double &l) {
        auto g = [&](double r) { return e.p(r) - p0; };
        v = newton_bracketed(g, dP, 0.0, s1);
        // p grows without bound towards 1/b: a finite upper end of the bracket
        double top = s2 + 0.5 * (rmax - s2);
        while (g(top) < 0.0) top = top + 0.5 * (rmax - top);
        l = newton_bracketed(g, dP, s2, top);
    };
    double v = 0, l = 0;
    roots(p_hi, v, l);
    if (!(e.gibbs(l) - e.gibbs(v) < 0.0)) return false;
    double p0 = 0.5 * (p_lo + p_hi);
    for (int it = 0; it < 200; ++it) {
        roots(p0, v, l);
        const double D = e.gibbs(l) - e.gibbs(v);
        if (D > 0.0) p_lo = p0; else p_hi = p0;
        double pn = p0 - D / (1.0 / l - 1.0 / v);
        if (!(pn > p_lo && pn < p_hi)) pn = 0.5 * (p_lo + p_hi);
        const bool done = std::fabs(pn - p0) <= 1e-15 * p0;
        p0 = pn;
        if (done) break;
    }
    roots(p0, rv, rl);
    return rv > 0.0 && rl > rv;
}

// ---- SplitMix64 (Steele, Lea, Flood 2014), counter-based use -------------
uint64_t splitmix64_at(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

uint64_t fnv1a(const void *data, size_t n, uint64_t h = 1469598103934665603ULL)
{
    const unsigned char *p = static_cast<const unsigned char *>(data);
    for (size_t k = 0; k < n; ++k) {
        h ^= p[k];
        h *= 1099511628211ULL;
    }
    return h;
}

struct BlobHeader {
    uint64_t magic;
    uint32_t version, precision;
    int32_t nx, ny, mode, periodic_y;
    uint64_t param_hash;
    uint64_t payload_bytes;
    uint64_t checksum;
};
constexpr uint64_t kMagic = 0x6c62626f696c3031ULL;  // "lbboil01"

}  // namespace

struct lbb_domain {
    lbb_params p{};
    lbb::DevParams dp{};
    size_t esz = 8;
    size_t N = 0;
    hipStream_t stream = nullptr;
    void *f[2] = {nullptr, nullptr};
    void *T[2] = {nullptr, nullptr};
    void *rho = nullptr, *vx = nullptr, *vy = nullptr;
    double *mass_part = nullptr, *hf_part = nullptr, *Tb_dev = nullptr;
    lbb::Scalars *sc = nullptr;
    int nbxA = 0, nbyA = 0, nbxB = 0, nbyB = 0;
    int shA = 0, shB = 0;                // tile shapes (indices into kShapeA, kShapeB)
    int cf = 0, cT = 0;
    lbb::Inst *d_inst = nullptr;         // this lattice as a one-entry launch table
    int *d_blkA = nullptr, *d_blkB = nullptr;
    bool poisoned = false;
    hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    std::vector<double> Tb;
    int64_t dev_bytes = 0;
    void *adj_mem = nullptr;             // adjoint workspace, kept between calls
    size_t adj_bytes = 0;
    int64_t held = 0;                    // device bytes held against the budget
};

struct lbb_param_dims {
    int nx, ny;
};

static_assert(sizeof(lbb_params) == 216, "lbb_params layout changed: update the Python binding");

namespace {

int validate(const lbb_params *p)
{
    if (!p) return fail(LBB_EINVAL, "params is NULL");
    if (p->nx < 3) return fail(LBB_EINVAL, "nx must be >= 3");
    if (p->periodic_y ? p->ny < 3 : p->ny < 4) return fail(LBB_EINVAL, "ny must be >= 4 (>= 3 when periodic_y)");
    if (p->precision != LBB_FP64 && p->precision != LBB_FP32) return fail(LBB_EINVAL, "unknown precision");
    // the kernels address a field plane with 32-bit byte offsets
    const int64_t plane = (int64_t)p->nx * p->ny * (p->precision == LBB_FP64 ? 8 : 4);
    if (plane >= (int64_t)1 << 32) return fail(LBB_EINVAL, "nx*ny*sizeof(real) must stay below 2^32 bytes");
    if (p->thermal_mode < LBB_COUPLED || p->thermal_mode > LBB_THERMAL_ONLY) return fail(LBB_EINVAL, "unknown thermal_mode");
    const double v[] = {p->a, p->b, p->R, p->omega, p->Ts_over_Tc, p->G, p->sigma, p->s_rho, p->s_e, p->s_zeta,
                        p->s_j, p->s_q, p->nu_L, p->nu_V, p->rho_L, p->rho_V, p->cv, p->cv_chi, p->g,
                        p->Gw_bottom, p->Gw_top, p->noise_amp};
    for (double x : v)
        if (!std::isfinite(x)) return fail(LBB_EINVAL, "non-finite parameter");
    if (!(p->a > 0 && p->b > 0 && p->R > 0 && p->cv > 0 && p->Ts_over_Tc > 0)) return fail(LBB_EINVAL, "a, b, R, c_v, T_s must be > 0");
    if (!(p->G < 0)) return fail(LBB_EINVAL, "G must be < 0");
    if (!(p->s_e > 0 && p->s_e < 2 && p->s_zeta > 0 && p->s_zeta < 2)) return fail(LBB_EINVAL, "s_e, s_zeta must lie in (0, 2)");
    if (!(p->nu_L > 0 && p->nu_V > 0)) return fail(LBB_EINVAL, "viscosities must be > 0");
    if (p->rho_L < 0 || p->rho_V < 0) return fail(LBB_EINVAL, "rho_L, rho_V must be >= 0");
    if (p->noise_amp < 0) return fail(LBB_EINVAL, "noise_amp must be >= 0");
    if (p->liquid_rows < 0 || p->liquid_rows > p->ny) return fail(LBB_EINVAL, "liquid_rows out of range");
    if (p->ghost_layer != 0 && p->ghost_layer != 1) return fail(LBB_EINVAL, "ghost_layer must be 0 or 1");
    if (p->reserved != 0) return fail(LBB_EINVAL, "reserved must be 0");
    return LBB_OK;
}

// Device parameters of a validated parameter set (rho_L, rho_V resolved).
void make_dev_params(const lbb_params &p, double Tc, double kap, lbb::DevParams &q)
{
    q = lbb::DevParams{};
    const double Ts = p.Ts_over_Tc * Tc;
    q.nx = p.nx;
    q.ny = p.ny;
    q.periodic_y = p.periodic_y ? 1 : 0;
    q.mode = p.thermal_mode;
    q.ghost = p.ghost_layer && !p.periodic_y ? 1 : 0;
    q.a = p.a;
    q.b = p.b;
    q.R = p.R;
    q.Tc = Tc;
    q.kappa = kap;
    q.Ts = Ts;
    q.T_ref = p.precision == LBB_FP64 ? 0.0 : Ts;
    q.G = p.G;
    q.sigma = p.sigma;
    q.s_rho = p.s_rho;
    q.s_e = p.s_e;
    q.s_zeta = p.s_zeta;
    q.s_j = p.s_j;
    q.s_q = p.s_q;
    const double tauL = 3.0 * p.nu_L + 0.5, tauV = 3.0 * p.nu_V + 0.5;
    q.tau_V = tauV;
    q.tau_slope = (tauL - tauV) / (p.rho_L - p.rho_V);
    q.rho_V = p.rho_V;
    q.cv = p.cv;
    q.cv_chi = p.cv_chi;
    q.chi = p.cv_chi / p.cv;
    q.g = p.g;
    q.Gw_bottom = p.Gw_bottom;
    q.Gw_top = p.Gw_top;
    q.sig_e = p.sigma / (1.0 / p.s_e - 0.5);
    q.sig_z = p.sigma / (1.0 / p.s_zeta - 0.5);
    q.inv_Tc = 1.0 / Tc;
    q.two_over_G = 2.0 / p.G;
    q.R_cv = p.R / p.cv;
    q.a_cv = p.a / p.cv;
    q.inv_cv = 1.0 / p.cv;
    q.k1k = kap * (1.0 + kap);
    q.k2_Tc = kap * kap / Tc;
    q.k1k_rsTc = kap * (1.0 + kap) / std::sqrt(Tc);
    q.R_cv12 = p.R / (12.0 * p.cv);
    q.a_cv12 = p.a / (12.0 * p.cv);
}

uint64_t param_hash(const lbb_params &p)
{
    lbb_params q = p;
    q.Gw_bottom = 0.0;  // changeable at run time
    q.noise_amp = 0.0;
    q.seed = 0;
    q.liquid_rows = 0;
    return fnv1a(&q, sizeof q);
}

lbb::Inst make_inst(const lbb_domain *d)
{
    lbb::Inst I{};
    I.P = d->dp;
    I.f[0] = d->f[0];
    I.f[1] = d->f[1];
    I.T[0] = d->T[0];
    I.T[1] = d->T[1];
    I.rho = d->rho;
    I.vx = d->vx;
    I.vy = d->vy;
    I.mass_part = d->mass_part;
    I.hf_part = d->hf_part;
    I.sc = d->sc;
    I.nbxA = d->nbxA;
    I.nbyA = d->nbyA;
    I.nbxB = d->nbxB;
    I.nbyB = d->nbyB;
    I.blkA0 = 0;
    I.blkB0 = 0;
    return I;
}

// Upload the one-entry launch table (after any parameter change).
int push_inst(lbb_domain *d)
{
    const lbb::Inst I = make_inst(d);
    LBB_HIP(hipMemcpyAsync(d->d_inst, &I, sizeof I, hipMemcpyHostToDevice, d->stream));
    LBB_HIP(hipStreamSynchronize(d->stream));
    return LBB_OK;
}

// The optional events are recorded by the dispatch itself (start and end of
// the kernel), so their interval is the kernel's own duration.
template <typename K, typename... A>
void launch_kernel(K kern, int nblocks, int nthreads, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, A... args)
{
    if (ev0)
        hipExtLaunchKernelGGL(kern, dim3(nblocks), dim3(nthreads), 0, st, ev0, ev1, 0, args...);
    else
        hipLaunchKernelGGL(kern, dim3(nblocks), dim3(nthreads), 0, st, args...);
}

// LB and thermal launches in tile shape `sh` (an index into kShapeA or
// kShapeB).  The optional events are recorded by the dispatch itself (start
// and end of the kernel), so their interval is the kernel's own duration.
template <typename S>
void launch_lb(hipStream_t st, const lbb::Inst *insts, const int *blk, int nblocks, int cf, int cT, int sh,
               hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    using namespace lbb;
    switch (sh) {
    case 1: launch_kernel(k_lb<S, kShapeA[1].ty, kShapeA[1].nw>, nblocks, 64 * kShapeA[1].nw, st, ev0, ev1, insts, blk, cf, cT); break;
    case 2: launch_kernel(k_lb<S, kShapeA[2].ty, kShapeA[2].nw>, nblocks, 64 * kShapeA[2].nw, st, ev0, ev1, insts, blk, cf, cT); break;
    case 3: launch_kernel(k_lb<S, kShapeA[3].ty, kShapeA[3].nw>, nblocks, 64 * kShapeA[3].nw, st, ev0, ev1, insts, blk, cf, cT); break;
    default: launch_kernel(k_lb<S, kShapeA[0].ty, kShapeA[0].nw>, nblocks, 64 * kShapeA[0].nw, st, ev0, ev1, insts, blk, cf, cT); break;
    }
}

template <typename S>
void launch_thermal(hipStream_t st, const lbb::Inst *insts, const int *blk, int nblocks, int cf, int cT, int sh,
                    hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    using namespace lbb;
    switch (sh) {
    case 1: launch_kernel(k_thermal<S, kShapeB[1].ty, kShapeB[1].nw>, nblocks, 64 * kShapeB[1].nw, st, ev0, ev1, insts, blk, cf, cT); break;
    case 2: launch_kernel(k_thermal<S, kShapeB[2].ty, kShapeB[2].nw>, nblocks, 64 * kShapeB[2].nw, st, ev0, ev1, insts, blk, cf, cT); break;
    case 3: launch_kernel(k_thermal<S, kShapeB[3].ty, kShapeB[3].nw>, nblocks, 64 * kShapeB[3].nw, st, ev0, ev1, insts, blk, cf, cT); break;
    default: launch_kernel(k_thermal<S, kShapeB[0].ty, kShapeB[0].nw>, nblocks, 64 * kShapeB[0].nw, st, ev0, ev1, insts, blk, cf, cT); break;
    }
}

template <typename S>
void launch_lb(lbb_domain *d, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    launch_lb<S>(d->stream, d->d_inst, d->d_blkA, d->nbxA * d->nbyA + 1, d->cf, d->cT, d->shA, ev0, ev1);
}

template <typename S>
void launch_thermal(lbb_domain *d, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr)
{
    launch_thermal<S>(d->stream, d->d_inst, d->d_blkB, d->nbxB * d->nbyB + 1, d->cf, d->cT, d->shB, ev0, ev1);
}

// Grid of the domain's launches for its tile shapes.
void set_grid(lbb_domain *d)
{
    d->nbxA = (d->p.nx + lbb::TXA - 1) / lbb::TXA;
    d->nbyA = (d->p.ny + lbb::kShapeA[d->shA].ty - 1) / lbb::kShapeA[d->shA].ty;
    d->nbxB = (d->p.nx + lbb::TXB - 1) / lbb::TXB;
    d->nbyB = (d->p.ny + lbb::kShapeB[d->shB].ty - 1) / lbb::kShapeB[d->shB].ty;
}

// Largest block counts over all tile shapes (sizes of the partial-sum and
// block-table buffers).
int max_blocks_A(const lbb_param_dims &g)
{
    int m = 0;
    for (const auto &t : lbb::kShapeA) m = std::max(m, ((g.nx + lbb::TXA - 1) / lbb::TXA) * ((g.ny + t.ty - 1) / t.ty));
    return m;
}
int max_blocks_B(const lbb_param_dims &g)
{
    int m = 0;
    for (const auto &t : lbb::kShapeB) m = std::max(m, ((g.nx + lbb::TXB - 1) / lbb::TXB) * ((g.ny + t.ty - 1) / t.ty));
    return m;
}

void advance_buffers(lbb_domain *d)
{
    if (d->dp.mode != lbb::MODE_THERMAL_ONLY) d->cf ^= 1;
    if (d->dp.mode != lbb::MODE_ISOTHERMAL) d->cT ^= 1;
}

template <typename S>
void enqueue_step(lbb_domain *d)
{
    launch_lb<S>(d);
    launch_thermal<S>(d);
    advance_buffers(d);
}

void enqueue_step_any(lbb_domain *d)
{
    if (d->p.precision == LBB_FP64) enqueue_step<double>(d);
    else enqueue_step<float>(d);
}

void drop_graphs(lbb_domain *d)
{
    for (auto &row : d->graph)
        for (auto &g : row)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

int build_graph(lbb_domain *d, hipGraphExec_t *out)
{
    const int cf = d->cf, cT = d->cT;
    LBB_HIP(hipStreamBeginCapture(d->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < kGraphSteps; ++k) enqueue_step_any(d);
    hipGraph_t g = nullptr;
    LBB_HIP(hipStreamEndCapture(d->stream, &g));
    d->cf = cf;  // capture recorded the launches; the state did not move
    d->cT = cT;
    hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LBB_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return LBB_OK;
}

int enqueue_steps(lbb_domain *d, int64_t n)
{
    while (n >= kGraphSteps) {
        hipGraphExec_t &g = d->graph[d->cf][d->cT];
        if (!g) {
            int rc = build_graph(d, &g);
            if (rc) return rc;
        }
        LBB_HIP(hipGraphLaunch(g, d->stream));
        // the buffers return to the same parity after an even number of steps
        n -= kGraphSteps;
    }
    for (int64_t k = 0; k < n; ++k) enqueue_step_any(d);
    hipLaunchKernelGGL(lbb::k_flush_heat_flux, dim3(1), dim3(lbb::NT), 0, d->stream, d->d_inst);
    LBB_HIP(hipGetLastError());
    return LBB_OK;
}

int check_errors(lbb_domain *d)
{
    lbb::Scalars s;
    LBB_HIP(hipMemcpyAsync(&s, d->sc, sizeof s, hipMemcpyDeviceToHost, d->stream));
    LBB_HIP(hipStreamSynchronize(d->stream));
    if (s.err_step != ~0ULL) {
        d->poisoned = true;
        std::string what;
        if (s.err_code & lbb::ERR_RHO) what += " non-positive or non-finite density;";
        if (s.err_code & lbb::ERR_PSI) what += " negative or non-finite pseudopotential radicand;";
        if (s.err_code & lbb::ERR_T) what += " non-positive or non-finite temperature;";
        return fail(LBB_ENONFINITE, "state became invalid at step " + std::to_string(s.err_step) + ":" + what);
    }
    return LBB_OK;
}

// Recompute rho_ave and the heat-flux partials from the current state.
template <typename S>
int refresh_reductions(lbb_domain *d)
{
    using namespace lbb;
    const int nm = d->nbxA * d->nbyA;
    hipLaunchKernelGGL(k_mass<S>, dim3(nm), dim3(NT), 0, d->stream, d->dp, static_cast<const S *>(d->f[d->cf]), d->mass_part);
    hipLaunchKernelGGL(k_reduce_mass, dim3(1), dim3(NT), 0, d->stream, d->dp, d->mass_part, nm, d->sc);
    hipLaunchKernelGGL(k_heat_flux_state<S>, dim3(d->nbxB), dim3(64), 0, d->stream, d->dp,
                       static_cast<const S *>(d->f[d->cf]), static_cast<const S *>(d->T[d->cT]), d->hf_part,
                       (double *)nullptr);
    hipLaunchKernelGGL(k_flush_heat_flux, dim3(1), dim3(NT), 0, d->stream, d->d_inst);
    LBB_HIP(hipGetLastError());
    return LBB_OK;
}

// Upload FP64 fields and build f = f_eq(rho, u), T; resets the counters.
template <typename S>
int set_state(lbb_domain *d, const double *rho, const double *ux, const double *uy, const double *T)
{
    const size_t N = d->N, nb = N * sizeof(double);
    double *buf = nullptr;
    LBB_HIP(hipMalloc(&buf, 4 * nb));
    double *drho = buf, *dux = buf + N, *duy = buf + 2 * N, *dT = buf + 3 * N;
    int rc = LBB_OK;
    do {
        if (hipMemcpyAsync(drho, rho, nb, hipMemcpyHostToDevice, d->stream) != hipSuccess ||
            (ux && hipMemcpyAsync(dux, ux, nb, hipMemcpyHostToDevice, d->stream) != hipSuccess) ||
            (uy && hipMemcpyAsync(duy, uy, nb, hipMemcpyHostToDevice, d->stream) != hipSuccess) ||
            (T && hipMemcpyAsync(dT, T, nb, hipMemcpyHostToDevice, d->stream) != hipSuccess)) {
            rc = fail(LBB_EDEVICE, "upload of the initial fields failed");
            break;
        }
        lbb::Scalars s{};
        s.err_step = ~0ULL;
        if (hipMemcpyAsync(d->sc, &s, sizeof s, hipMemcpyHostToDevice, d->stream) != hipSuccess) {
            rc = fail(LBB_EDEVICE, "scalar reset failed");
            break;
        }
        hipLaunchKernelGGL(lbb::k_set_state<S>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, d->stream, d->dp,
                           drho, ux ? dux : nullptr, uy ? duy : nullptr, T ? dT : nullptr, d->Tb_dev,
                           static_cast<S *>(d->f[0]), static_cast<S *>(d->T[0]), static_cast<S *>(d->T[1]), d->sc);
        d->cf = d->cT = 0;
        rc = refresh_reductions<S>(d);
        if (rc) break;
        if (hipStreamSynchronize(d->stream) != hipSuccess) {
            rc = fail(LBB_EDEVICE, "set-up kernels failed");
            break;
        }
    } while (0);
    (void)hipFree(buf);
    if (rc) return rc;
    rc = check_errors(d);
    if (rc) return fail(LBB_EINVAL, "initial state invalid (rho <= 0, T <= 0 or b rho >= 1)");
    d->poisoned = false;
    return LBB_OK;
}

void release(lbb_domain *d)
{
    if (!d) return;
    release_bytes(d->held);
    drop_graphs(d);
    for (void *q : {d->f[0], d->f[1], d->T[0], d->T[1], d->rho, d->vx, d->vy})
        if (q) (void)hipFree(q);
    for (void *q : {(void *)d->mass_part, (void *)d->hf_part, (void *)d->Tb_dev, (void *)d->sc,
                    (void *)d->d_inst, (void *)d->d_blkA, (void *)d->d_blkB, d->adj_mem})
        if (q) (void)hipFree(q);
    if (d->stream) (void)hipStreamDestroy(d->stream);
    delete d;
}

template <typename S>
int read_impl(lbb_domain *d, double *rho, double *ux, double *uy, double *T, double *f)
{
    const size_t N = d->N, nb = N * sizeof(double);
    double *buf = nullptr;
    LBB_HIP(hipMalloc(&buf, 13 * nb));
    double *r = buf, *u = buf + N, *v = buf + 2 * N, *t = buf + 3 * N, *ff = buf + 4 * N;
    const int nbxR = (d->p.nx + lbb::TXR - 1) / lbb::TXR, nbyR = (d->p.ny + lbb::TYR - 1) / lbb::TYR;
    hipLaunchKernelGGL(lbb::k_read<S>, dim3(nbxR * nbyR), dim3(lbb::NT), 0, d->stream, d->dp,
                       static_cast<const S *>(d->f[d->cf]), static_cast<const S *>(d->T[d->cT]), r, u, v, t, ff,
                       d->sc, nbxR);
    int rc = LBB_OK;
    if (hipGetLastError() != hipSuccess) rc = fail(LBB_EDEVICE, "read-back kernel failed");
    const struct { double *dst, *src; size_t n; } cp[] = {{rho, r, N}, {ux, u, N}, {uy, v, N}, {T, t, N}, {f, ff, 9 * N}};
    for (auto &c : cp)
        if (!rc && c.dst && hipMemcpyAsync(c.dst, c.src, c.n * sizeof(double), hipMemcpyDeviceToHost, d->stream) != hipSuccess)
            rc = fail(LBB_EDEVICE, "read-back copy failed");
    if (!rc && hipStreamSynchronize(d->stream) != hipSuccess) rc = fail(LBB_EDEVICE, "read-back failed");
    (void)hipFree(buf);
    return rc;
}

}  // namespace

extern "C" {

const char *lbb_last_error(void) { return g_err.c_str(); }

void lbb_default_params(lbb_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->nx = 128;
    p->ny = 64;
    p->precision = LBB_FP64;
    p->periodic_y = 0;
    p->thermal_mode = LBB_COUPLED;
    p->liquid_rows = (int32_t)std::floor(0.6 * 64);
    p->a = 2.0 / 49.0;
    p->b = 2.0 / 21.0;
    p->R = 1.0;
    p->omega = 0.344;
    p->Ts_over_Tc = 0.86;
    p->G = -1.0;
    p->sigma = 1.2;
    p->s_rho = 1.0;
    p->s_e = 0.8;
    p->s_zeta = 0.8;
    p->s_j = 1.0;
    p->s_q = 1.1;
    p->nu_L = 0.1;
    p->nu_V = 0.5 / 3.0;
    p->rho_L = 0.0;
    p->rho_V = 0.0;
    p->cv = 6.0;
    p->cv_chi = 0.028;
    p->g = 3e-5;
    p->Gw_bottom = 0.0;
    p->Gw_top = 0.0;
    p->noise_amp = 1e-3;
    p->seed = 1;
}

int lbb_eos_constants(double a, double b, double R, double omega, double *Tc, double *kappa)
{
    if (!(finite_pos(a) && finite_pos(b) && finite_pos(R) && std::isfinite(omega)))
        return fail(LBB_EINVAL, "a, b, R must be finite and > 0");
    if (Tc) *Tc = (a / b) * (0.0778 / 0.45724) / R;
    if (kappa) *kappa = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
    return LBB_OK;
}

int lbb_coexistence(double a, double b, double R, double omega, double T, double *rho_V, double *rho_L)
{
    double Tc = 0, kap = 0;
    int rc = lbb_eos_constants(a, b, R, omega, &Tc, &kap);
    if (rc) return rc;
    if (!(finite_pos(T) && T < Tc)) return fail(LBB_EINVAL, "coexistence needs 0 < T < T_c");
    Eos e{a, b, R, Tc, kap, T};
    double rv = 0, rl = 0;
    if (!maxwell(e, rv, rl)) return fail(LBB_EINVAL, "no two-phase region at this temperature");
    if (rho_V) *rho_V = rv;
    if (rho_L) *rho_L = rl;
    return LBB_OK;
}

int lbb_eos_pressure(double a, double b, double R, double omega, double rho, double T, double *p)
{
    double Tc = 0, kap = 0;
    int rc = lbb_eos_constants(a, b, R, omega, &Tc, &kap);
    if (rc) return rc;
    if (!p) return fail(LBB_EINVAL, "p is NULL");
    if (!(finite_pos(rho) && finite_pos(T) && b * rho < 1.0)) return fail(LBB_EINVAL, "needs rho > 0, T > 0, b rho < 1");
    const Eos e{a, b, R, Tc, kap, T};
    *p = e.p(rho);
    return LBB_OK;
}

int lbb_init_domain(const lbb_params *pin, const double *T_bottom, const double *rho0, lbb_domain **out)
{
    if (!out) return fail(LBB_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(pin);
    if (rc) return rc;
    lbb_params p = *pin;
    double Tc = 0, kap = 0;
    lbb_eos_constants(p.a, p.b, p.R, p.omega, &Tc, &kap);
    const double Ts = p.Ts_over_Tc * Tc;
    if (p.rho_L == 0.0 && p.rho_V == 0.0) {
        rc = lbb_coexistence(p.a, p.b, p.R, p.omega, Ts, &p.rho_V, &p.rho_L);
        if (rc) return fail(LBB_EINVAL, "rho_L = rho_V = 0 needs T_s < T_c for the Maxwell densities");
    }
    if (p.rho_L == p.rho_V) return fail(LBB_EINVAL, "rho_L must differ from rho_V");
    const size_t N = (size_t)p.nx * p.ny;
    std::vector<double> rho_host;
    if (!rho0) {
        rho_host.resize(N);
        for (int j = 0; j < p.ny; ++j)
            for (int i = 0; i < p.nx; ++i) {
                const size_t c = (size_t)j * p.nx + i;
                const double u = (double)(splitmix64_at(p.seed, c) >> 11) * (1.0 / 9007199254740992.0);
                rho_host[c] = (j < p.liquid_rows ? p.rho_L : p.rho_V) + p.noise_amp * (2.0 * u - 1.0);
            }
        rho0 = rho_host.data();
    }
    for (size_t c = 0; c < N; ++c)
        if (!finite_pos(rho0[c]) || p.b * rho0[c] >= 1.0) return fail(LBB_EINVAL, "initial density must satisfy 0 < rho < 1/b");
    std::vector<double> Tb(p.nx, Ts);
    if (T_bottom)
        for (int i = 0; i < p.nx; ++i) {
            if (!finite_pos(T_bottom[i])) return fail(LBB_EINVAL, "T_bottom must be finite and > 0");
            Tb[i] = T_bottom[i];
        }

    // the device bytes this domain will hold, reserved under the budget first
    const size_t esz = p.precision == LBB_FP64 ? 8 : 4;
    const int64_t planned = (int64_t)(N * esz * (2 * 9 + 2 + 3)) + (int64_t)N * 8 + ((int64_t)1 << 20);
    rc = reserve_bytes(planned, "domain");
    if (rc) return rc;
    struct Unreserve {
        int64_t n;
        ~Unreserve() { release_bytes(n); }
    } unreserve{planned};

    int dev = 0;
    LBB_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    LBB_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(LBB_EDEVICE, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);

    lbb_domain *d = new (std::nothrow) lbb_domain();
    if (!d) return fail(LBB_ENOMEM, "host allocation failed");
    d->p = p;
    d->N = N;
    d->esz = p.precision == LBB_FP64 ? 8 : 4;
    d->Tb = Tb;
    make_dev_params(p, Tc, kap, d->dp);
    set_grid(d);
    const lbb_param_dims dims{p.nx, p.ny};
    const int mbA = max_blocks_A(dims), mbB = max_blocks_B(dims);

    auto alloc = [&](void **ptr, size_t bytes) -> bool {
        if (hipMalloc(ptr, bytes) != hipSuccess) return false;
        d->dev_bytes += (int64_t)bytes;
        return hipMemset(*ptr, 0, bytes) == hipSuccess;
    };
    const size_t es = d->esz;
    bool ok = hipStreamCreateWithFlags(&d->stream, hipStreamNonBlocking) == hipSuccess;
    ok = ok && alloc(&d->f[0], 9 * N * es) && alloc(&d->f[1], 9 * N * es);
    ok = ok && alloc(&d->T[0], N * es) && alloc(&d->T[1], N * es);
    ok = ok && alloc(&d->rho, N * es) && alloc(&d->vx, N * es) && alloc(&d->vy, N * es);
    // mass partials: one per lattice row and LB tile column (also holds the
    // per-block partials of the set-up mass kernel, fewer)
    ok = ok && alloc((void **)&d->mass_part, (size_t)std::max(mbA, d->nbxA * p.ny) * sizeof(double));
    ok = ok && alloc((void **)&d->hf_part, (size_t)d->nbxB * sizeof(double));
    ok = ok && alloc((void **)&d->Tb_dev, (size_t)p.nx * sizeof(double));
    ok = ok && alloc((void **)&d->sc, sizeof(lbb::Scalars));
    ok = ok && alloc((void **)&d->d_inst, sizeof(lbb::Inst));
    ok = ok && alloc((void **)&d->d_blkA, (size_t)(mbA + 1) * sizeof(int));
    ok = ok && alloc((void **)&d->d_blkB, (size_t)(mbB + 1) * sizeof(int));
    if (!ok) {
        (void)hipGetLastError();
        release(d);
        return fail(LBB_ENOMEM, "device allocation failed");
    }
    if (hipMemcpy(d->Tb_dev, Tb.data(), p.nx * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        push_inst(d) != LBB_OK) {
        release(d);
        return fail(LBB_EDEVICE, "upload of T_bottom or the launch table failed");
    }
    rc = p.precision == LBB_FP64 ? set_state<double>(d, rho0, nullptr, nullptr, nullptr)
                                 : set_state<float>(d, rho0, nullptr, nullptr, nullptr);
    if (rc) {
        std::string m = g_err;
        release(d);
        return fail(rc, m);
    }
    g_held.fetch_add(d->dev_bytes);
    d->held = d->dev_bytes;
    *out = d;
    return LBB_OK;
}

int lbb_set_fields(lbb_domain *d, const double *rho, const double *ux, const double *uy, const double *T)
{
    if (!d || !rho) return fail(LBB_EINVAL, "domain and rho are required");
    for (size_t c = 0; c < d->N; ++c) {
        if (!finite_pos(rho[c]) || d->p.b * rho[c] >= 1.0) return fail(LBB_EINVAL, "rho must satisfy 0 < rho < 1/b");
        if ((ux && !std::isfinite(ux[c])) || (uy && !std::isfinite(uy[c]))) return fail(LBB_EINVAL, "non-finite velocity");
        if (T && !finite_pos(T[c])) return fail(LBB_EINVAL, "T must be finite and > 0");
    }
    return d->p.precision == LBB_FP64 ? set_state<double>(d, rho, ux, uy, T) : set_state<float>(d, rho, ux, uy, T);
}

int lbb_step_async(lbb_domain *d, int64_t n)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    if (n < 0) return fail(LBB_EINVAL, "n must be >= 0");
    if (d->poisoned) return fail(LBB_ESTATE, "domain poisoned by an earlier invalid state; load a state first");
    return enqueue_steps(d, n);
}

int lbb_sync(lbb_domain *d)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    LBB_HIP(hipStreamSynchronize(d->stream));
    return check_errors(d);
}

int lbb_step(lbb_domain *d, int64_t n)
{
    int rc = lbb_step_async(d, n);
    if (rc) return rc;
    return lbb_sync(d);
}

void *lbb_stream(lbb_domain *d) { return d ? (void *)d->stream : nullptr; }

int lbb_time_kernels(lbb_domain *d, int64_t n, double *ms_lb, double *ms_thermal, double *ms_step)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    if (n < 1) return fail(LBB_EINVAL, "n must be >= 1");
    if (d->poisoned) return fail(LBB_ESTATE, "domain poisoned by an earlier invalid state; load a state first");
    // per step: kernel start/end events of both launches, plus the ends of the run
    std::vector<hipEvent_t> ev(4 * (size_t)n + 2, nullptr);
    for (auto &e : ev) LBB_HIP(hipEventCreate(&e));
    const bool fp64 = d->p.precision == LBB_FP64;
    LBB_HIP(hipEventRecord(ev[0], d->stream));
    for (int64_t k = 0; k < n; ++k) {
        hipEvent_t *e = &ev[4 * k + 1];
        if (fp64) launch_lb<double>(d, e[0], e[1]); else launch_lb<float>(d, e[0], e[1]);
        LBB_HIP(hipGetLastError());
        if (fp64) launch_thermal<double>(d, e[2], e[3]); else launch_thermal<float>(d, e[2], e[3]);
        LBB_HIP(hipGetLastError());
        advance_buffers(d);
    }
    LBB_HIP(hipEventRecord(ev[4 * n + 1], d->stream));
    hipLaunchKernelGGL(lbb::k_flush_heat_flux, dim3(1), dim3(lbb::NT), 0, d->stream, d->d_inst);
    LBB_HIP(hipGetLastError());
    LBB_HIP(hipStreamSynchronize(d->stream));
    double a = 0, b = 0;
    float ms = 0;
    for (int64_t k = 0; k < n; ++k) {
        LBB_HIP(hipEventElapsedTime(&ms, ev[4 * k + 1], ev[4 * k + 2]));
        a += ms;
        LBB_HIP(hipEventElapsedTime(&ms, ev[4 * k + 3], ev[4 * k + 4]));
        b += ms;
    }
    LBB_HIP(hipEventElapsedTime(&ms, ev[0], ev[4 * n + 1]));
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (ms_lb) *ms_lb = a / (double)n;
    if (ms_thermal) *ms_thermal = b / (double)n;
    if (ms_step) *ms_step = (double)ms / (double)n;
    return check_errors(d);
}

int lbb_read_fields_dev(lbb_domain *d, double *rho, double *ux, double *uy, double *T, double *f, void *stream)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    // the library stream does not synchronize with the null stream by
    // itself, so the ordering is made explicit for any stream, NULL included
    hipStream_t cs = static_cast<hipStream_t>(stream);
    hipEvent_t ev = nullptr;
    LBB_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    {
        // the caller's earlier work on these buffers comes first
        hipError_t e0 = hipEventRecord(ev, cs);
        if (e0 == hipSuccess) e0 = hipStreamWaitEvent(d->stream, ev, 0);
        if (e0 != hipSuccess) {
            (void)hipEventDestroy(ev);
            return fail(LBB_EDEVICE, std::string("read-back to device buffers: ") + hipGetErrorString(e0));
        }
    }
    const int nbxR = (d->p.nx + lbb::TXR - 1) / lbb::TXR, nbyR = (d->p.ny + lbb::TYR - 1) / lbb::TYR;
    if (d->p.precision == LBB_FP64)
        hipLaunchKernelGGL(lbb::k_read<double>, dim3(nbxR * nbyR), dim3(lbb::NT), 0, d->stream, d->dp,
                           static_cast<const double *>(d->f[d->cf]), static_cast<const double *>(d->T[d->cT]), rho,
                           ux, uy, T, f, d->sc, nbxR);
    else
        hipLaunchKernelGGL(lbb::k_read<float>, dim3(nbxR * nbyR), dim3(lbb::NT), 0, d->stream, d->dp,
                           static_cast<const float *>(d->f[d->cf]), static_cast<const float *>(d->T[d->cT]), rho,
                           ux, uy, T, f, d->sc, nbxR);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        // and the caller's later work on its stream waits for the read
        e = hipEventRecord(ev, d->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev, 0);
    }
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return fail(LBB_EDEVICE, std::string("read-back to device buffers: ") + hipGetErrorString(e));
    return LBB_OK;
}

int lbb_read_fields(const lbb_domain *dc, uint32_t mask, double *rho, double *ux, double *uy, double *T, double *f)
{
    if (!dc) return fail(LBB_EINVAL, "domain is NULL");
    // reading uses the domain's stream and staging buffers but leaves its state alone
    lbb_domain *d = const_cast<lbb_domain *>(dc);
    if (!(mask & LBB_FIELD_RHO)) rho = nullptr;
    if (!(mask & LBB_FIELD_UX)) ux = nullptr;
    if (!(mask & LBB_FIELD_UY)) uy = nullptr;
    if (!(mask & LBB_FIELD_T)) T = nullptr;
    if (!(mask & LBB_FIELD_F)) f = nullptr;
    return d->p.precision == LBB_FP64 ? read_impl<double>(d, rho, ux, uy, T, f) : read_impl<float>(d, rho, ux, uy, T, f);
}

int lbb_wall_heat_flux(const lbb_domain *dc, double *q_now, double *q_mean, double *q_local, int64_t *n_samples)
{
    if (!dc) return fail(LBB_EINVAL, "domain is NULL");
    // the read-back uses the domain's stream but leaves its state alone
    lbb_domain *d = const_cast<lbb_domain *>(dc);
    lbb::Scalars s;
    LBB_HIP(hipMemcpyAsync(&s, d->sc, sizeof s, hipMemcpyDeviceToHost, d->stream));
    if (q_local) {
        double *ql = nullptr;
        LBB_HIP(hipMalloc(&ql, d->p.nx * sizeof(double)));
        if (d->p.precision == LBB_FP64)
            hipLaunchKernelGGL(lbb::k_heat_flux_state<double>, dim3(d->nbxB), dim3(64), 0, d->stream, d->dp,
                               static_cast<const double *>(d->f[d->cf]), static_cast<const double *>(d->T[d->cT]),
                               (double *)nullptr, ql);
        else
            hipLaunchKernelGGL(lbb::k_heat_flux_state<float>, dim3(d->nbxB), dim3(64), 0, d->stream, d->dp,
                               static_cast<const float *>(d->f[d->cf]), static_cast<const float *>(d->T[d->cT]),
                               (double *)nullptr, ql);
        hipError_t e = hipMemcpyAsync(q_local, ql, d->p.nx * sizeof(double), hipMemcpyDeviceToHost, d->stream);
        hipError_t e2 = hipStreamSynchronize(d->stream);
        (void)hipFree(ql);
        if (e != hipSuccess || e2 != hipSuccess) return fail(LBB_EDEVICE, "heat-flux read-back failed");
    }
    LBB_HIP(hipStreamSynchronize(d->stream));
    if (q_now) *q_now = s.q_now;
    if (q_mean) *q_mean = s.n_samples ? s.q_sum / (double)s.n_samples : NAN;
    if (n_samples) *n_samples = s.n_samples;
    return LBB_OK;
}

int lbb_reset_average(lbb_domain *d)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    lbb::Scalars s;
    LBB_HIP(hipMemcpyAsync(&s, d->sc, sizeof s, hipMemcpyDeviceToHost, d->stream));
    LBB_HIP(hipStreamSynchronize(d->stream));
    s.q_sum = 0.0;
    s.n_samples = 0;
    LBB_HIP(hipMemcpyAsync(d->sc, &s, sizeof s, hipMemcpyHostToDevice, d->stream));
    LBB_HIP(hipStreamSynchronize(d->stream));
    return LBB_OK;
}

int lbb_set_heater(lbb_domain *d, const double *T_bottom)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    std::vector<double> Tb(d->p.nx, d->dp.Ts);
    if (T_bottom)
        for (int i = 0; i < d->p.nx; ++i) {
            if (!finite_pos(T_bottom[i])) return fail(LBB_EINVAL, "T_bottom must be finite and > 0");
            Tb[i] = T_bottom[i];
        }
    d->Tb = Tb;
    LBB_HIP(hipMemcpyAsync(d->Tb_dev, Tb.data(), d->p.nx * sizeof(double), hipMemcpyHostToDevice, d->stream));
    const unsigned nb = (unsigned)((d->p.nx + 255) / 256);
    if (d->p.precision == LBB_FP64)
        hipLaunchKernelGGL(lbb::k_set_heater<double>, dim3(nb), dim3(256), 0, d->stream, d->dp, d->Tb_dev,
                           static_cast<double *>(d->T[0]), static_cast<double *>(d->T[1]));
    else
        hipLaunchKernelGGL(lbb::k_set_heater<float>, dim3(nb), dim3(256), 0, d->stream, d->dp, d->Tb_dev,
                           static_cast<float *>(d->T[0]), static_cast<float *>(d->T[1]));
    LBB_HIP(hipGetLastError());
    LBB_HIP(hipStreamSynchronize(d->stream));
    return LBB_OK;
}

int lbb_set_wettability(lbb_domain *d, double Gw_bottom)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    if (!std::isfinite(Gw_bottom)) return fail(LBB_EINVAL, "G_w must be finite");
    d->p.Gw_bottom = Gw_bottom;
    d->dp.Gw_bottom = Gw_bottom;
    return push_inst(d);  // captured graphs read the table, so they stay valid
}

int lbb_save_state(lbb_domain *d, void *buf, size_t *len)
{
    if (!d || !len) return fail(LBB_EINVAL, "domain and len are required");
    const size_t es = d->esz, N = d->N;
    const size_t payload = 10 * N * es + d->p.nx * sizeof(double) + sizeof(double) + sizeof(lbb::Scalars) +
                           d->nbxB * sizeof(double);
    const size_t need = sizeof(BlobHeader) + payload;
    if (!buf) {
        *len = need;
        return LBB_OK;
    }
    if (*len < need) return fail(LBB_EINVAL, "buffer too small");
    if (d->p.precision == LBB_FP64)
        hipLaunchKernelGGL(lbb::k_complete_walls<double>, dim3((d->p.nx + 255) / 256), dim3(256), 0, d->stream, d->dp,
                           static_cast<double *>(d->f[d->cf]));
    else
        hipLaunchKernelGGL(lbb::k_complete_walls<float>, dim3((d->p.nx + 255) / 256), dim3(256), 0, d->stream, d->dp,
                           static_cast<float *>(d->f[d->cf]));
    unsigned char *o = static_cast<unsigned char *>(buf) + sizeof(BlobHeader);
    unsigned char *p = o;
    LBB_HIP(hipMemcpyAsync(p, d->f[d->cf], 9 * N * es, hipMemcpyDeviceToHost, d->stream));
    p += 9 * N * es;
    LBB_HIP(hipMemcpyAsync(p, d->T[d->cT], N * es, hipMemcpyDeviceToHost, d->stream));
    p += N * es;
    std::memcpy(p, d->Tb.data(), d->p.nx * sizeof(double));
    p += d->p.nx * sizeof(double);
    std::memcpy(p, &d->p.Gw_bottom, sizeof(double));
    p += sizeof(double);
    LBB_HIP(hipMemcpyAsync(p, d->sc, sizeof(lbb::Scalars), hipMemcpyDeviceToHost, d->stream));
    p += sizeof(lbb::Scalars);
    LBB_HIP(hipMemcpyAsync(p, d->hf_part, d->nbxB * sizeof(double), hipMemcpyDeviceToHost, d->stream));
    LBB_HIP(hipStreamSynchronize(d->stream));
    BlobHeader h{};
    h.magic = kMagic;
    h.version = 1;
    h.precision = (uint32_t)d->p.precision;
    h.nx = d->p.nx;
    h.ny = d->p.ny;
    h.mode = d->p.thermal_mode;
    h.periodic_y = d->p.periodic_y;
    h.param_hash = param_hash(d->p);
    h.payload_bytes = payload;
    h.checksum = fnv1a(o, payload);
    std::memcpy(buf, &h, sizeof h);
    *len = need;
    return LBB_OK;
}

int lbb_load_state(lbb_domain *d, const void *buf, size_t len)
{
    if (!d || !buf) return fail(LBB_EINVAL, "domain and buf are required");
    if (len < sizeof(BlobHeader)) return fail(LBB_EINVAL, "blob too short");
    BlobHeader h;
    std::memcpy(&h, buf, sizeof h);
    const size_t es = d->esz, N = d->N;
    const size_t payload = 10 * N * es + d->p.nx * sizeof(double) + sizeof(double) + sizeof(lbb::Scalars) +
                           d->nbxB * sizeof(double);
    if (h.magic != kMagic || h.version != 1) return fail(LBB_EINVAL, "not an lbboil state blob");
    if (h.nx != d->p.nx || h.ny != d->p.ny || h.precision != (uint32_t)d->p.precision ||
        h.mode != d->p.thermal_mode || h.periodic_y != d->p.periodic_y || h.param_hash != param_hash(d->p))
        return fail(LBB_EINVAL, "blob belongs to a domain with other shape or parameters");
    if (h.payload_bytes != payload || len < sizeof h + payload) return fail(LBB_EINVAL, "blob size mismatch");
    const unsigned char *o = static_cast<const unsigned char *>(buf) + sizeof h;
    if (fnv1a(o, payload) != h.checksum) return fail(LBB_EINVAL, "blob checksum mismatch (corrupted)");
    const unsigned char *p = o;
    LBB_HIP(hipMemcpyAsync(d->f[0], p, 9 * N * es, hipMemcpyHostToDevice, d->stream));
    p += 9 * N * es;
    LBB_HIP(hipMemcpyAsync(d->T[0], p, N * es, hipMemcpyHostToDevice, d->stream));
    LBB_HIP(hipMemcpyAsync(d->T[1], p, N * es, hipMemcpyHostToDevice, d->stream));
    p += N * es;
    std::vector<double> Tb(d->p.nx);
    std::memcpy(Tb.data(), p, d->p.nx * sizeof(double));
    p += d->p.nx * sizeof(double);
    double Gw;
    std::memcpy(&Gw, p, sizeof Gw);
    p += sizeof(double);
    lbb::Scalars s;
    std::memcpy(&s, p, sizeof s);
    p += sizeof s;
    s.err_step = ~0ULL;
    s.err_code = 0;
    LBB_HIP(hipMemcpyAsync(d->sc, &s, sizeof s, hipMemcpyHostToDevice, d->stream));
    LBB_HIP(hipMemcpyAsync(d->hf_part, p, d->nbxB * sizeof(double), hipMemcpyHostToDevice, d->stream));
    LBB_HIP(hipStreamSynchronize(d->stream));
    d->Tb = Tb;
    LBB_HIP(hipMemcpy(d->Tb_dev, Tb.data(), d->p.nx * sizeof(double), hipMemcpyHostToDevice));
    d->cf = d->cT = 0;
    if (Gw != d->dp.Gw_bottom) {
        d->p.Gw_bottom = d->dp.Gw_bottom = Gw;
        int rc = push_inst(d);
        if (rc) return rc;
    }
    d->poisoned = false;
    return LBB_OK;
}

int lbb_info(lbb_domain *d, int64_t *t, int32_t *nx, int32_t *ny, int64_t *device_bytes)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    if (t) {
        lbb::Scalars s;
        LBB_HIP(hipMemcpyAsync(&s, d->sc, sizeof s, hipMemcpyDeviceToHost, d->stream));
        LBB_HIP(hipStreamSynchronize(d->stream));
        *t = s.tA;
    }
    if (nx) *nx = d->p.nx;
    if (ny) *ny = d->p.ny;
    if (device_bytes) *device_bytes = d->dev_bytes;
    return LBB_OK;
}

// ---- batched lattices --------------------------------------------------

struct lbb_batch {
    std::vector<lbb_domain *> doms;
    hipStream_t stream = nullptr;
    lbb::Inst *d_insts = nullptr;
    int *d_blkA = nullptr, *d_blkB = nullptr;
    int totA = 0, totB = 0;
    int cf = 0, cT = 0;
    int precision = 0, mode = 0;
    int shA = 0, shB = 0;                // tile shapes of the batch's launches
    hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    void *adj_mem = nullptr;             // adjoint workspace, kept between calls
    size_t adj_bytes = 0;
    int64_t held = 0;                    // device bytes held against the budget
};

static void batch_release(lbb_batch *b)
{
    if (!b) return;
    release_bytes(b->held);
    for (auto &row : b->graph)
        for (auto &g : row)
            if (g) (void)hipGraphExecDestroy(g);
    for (void *q : {(void *)b->d_insts, (void *)b->d_blkA, (void *)b->d_blkB, b->adj_mem})
        if (q) (void)hipFree(q);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    for (lbb_domain *d : b->doms) release(d);
    delete b;
}

static void batch_drop_graphs(lbb_batch *b)
{
    for (auto &row : b->graph)
        for (auto &g : row)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

// Block -> member tables of the batch's launches for its tile shapes (the
// buffers are sized for the largest block counts).
static int batch_tables(lbb_batch *b)
{
    std::vector<int> ta, tb;
    b->totA = b->totB = 0;
    for (size_t i = 0; i < b->doms.size(); ++i) {
        lbb_domain *d = b->doms[i];
        ta.insert(ta.end(), d->nbxA * d->nbyA + 1, (int)i);
        tb.insert(tb.end(), d->nbxB * d->nbyB + 1, (int)i);
        b->totA += d->nbxA * d->nbyA + 1;
        b->totB += d->nbxB * d->nbyB + 1;
    }
    LBB_HIP(hipMemcpy(b->d_blkA, ta.data(), ta.size() * sizeof(int), hipMemcpyHostToDevice));
    LBB_HIP(hipMemcpy(b->d_blkB, tb.data(), tb.size() * sizeof(int), hipMemcpyHostToDevice));
    return LBB_OK;
}

// Upload the launch table (all members, with their block offsets); members
// take the batch's tile shapes.
static int batch_push(lbb_batch *b)
{
    bool regrid = false;
    for (lbb_domain *d : b->doms)
        if (d->shA != b->shA || d->shB != b->shB) {
            d->shA = b->shA;
            d->shB = b->shB;
            set_grid(d);
            drop_graphs(d);
            int rc = push_inst(d);
            if (rc) return rc;
            regrid = true;
        }
    if (regrid) {
        int rc = batch_tables(b);
        if (rc) return rc;
        batch_drop_graphs(b);
    }
    std::vector<lbb::Inst> insts;
    int a0 = 0, b0 = 0;
    for (lbb_domain *d : b->doms) {
        lbb::Inst I = make_inst(d);
        I.blkA0 = a0;
        I.blkB0 = b0;
        a0 += d->nbxA * d->nbyA + 1;
        b0 += d->nbxB * d->nbyB + 1;
        insts.push_back(I);
    }
    LBB_HIP(hipMemcpyAsync(b->d_insts, insts.data(), insts.size() * sizeof(lbb::Inst), hipMemcpyHostToDevice,
                           b->stream));
    LBB_HIP(hipStreamSynchronize(b->stream));
    return LBB_OK;
}

static void batch_enqueue_step(lbb_batch *b)
{
    if (b->precision == LBB_FP64) {
        launch_lb<double>(b->stream, b->d_insts, b->d_blkA, b->totA, b->cf, b->cT, b->shA);
        launch_thermal<double>(b->stream, b->d_insts, b->d_blkB, b->totB, b->cf, b->cT, b->shB);
    } else {
        launch_lb<float>(b->stream, b->d_insts, b->d_blkA, b->totA, b->cf, b->cT, b->shA);
        launch_thermal<float>(b->stream, b->d_insts, b->d_blkB, b->totB, b->cf, b->cT, b->shB);
    }
    if (b->mode != LBB_THERMAL_ONLY) b->cf ^= 1;
    if (b->mode != LBB_ISOTHERMAL) b->cT ^= 1;
}

extern "C" int lbb_batch_init(const lbb_params *ps, int n, const double *const *T_bottoms,
                              const double *const *rho0s, lbb_batch **out)
{
    if (!out) return fail(LBB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ps || n < 1) return fail(LBB_EINVAL, "a batch needs n >= 1 parameter sets");
    for (int i = 1; i < n; ++i)
        if (ps[i].precision != ps[0].precision || ps[i].thermal_mode != ps[0].thermal_mode)
            return fail(LBB_EINVAL, "batch members must share precision and thermal_mode");
    lbb_batch *b = new (std::nothrow) lbb_batch();
    if (!b) return fail(LBB_ENOMEM, "host allocation failed");
    b->precision = ps[0].precision;
    b->mode = ps[0].thermal_mode;
    for (int i = 0; i < n; ++i) {
        lbb_domain *d = nullptr;
        int rc = lbb_init_domain(&ps[i], T_bottoms ? T_bottoms[i] : nullptr, rho0s ? rho0s[i] : nullptr, &d);
        if (rc) {
            std::string m = "batch member " + std::to_string(i) + ": " + g_err;
            batch_release(b);
            return fail(rc, m);
        }
        b->doms.push_back(d);
    }
    size_t capA = 0, capB = 0;
    for (lbb_domain *d : b->doms) {
        const lbb_param_dims dims{d->p.nx, d->p.ny};
        capA += max_blocks_A(dims) + 1;
        capB += max_blocks_B(dims) + 1;
    }
    bool ok = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc(&b->d_insts, n * sizeof(lbb::Inst)) == hipSuccess &&
              hipMalloc(&b->d_blkA, capA * sizeof(int)) == hipSuccess &&
              hipMalloc(&b->d_blkB, capB * sizeof(int)) == hipSuccess && batch_tables(b) == LBB_OK;
    if (!ok || batch_push(b) != LBB_OK) {
        (void)hipGetLastError();
        batch_release(b);
        return fail(LBB_ENOMEM, "batch launch tables could not be allocated");
    }
    *out = b;
    return LBB_OK;
}

// The batch steps its members together; they must share the buffer phase.
static int batch_phase(lbb_batch *b)
{
    b->cf = b->doms[0]->cf;
    b->cT = b->doms[0]->cT;
    for (lbb_domain *d : b->doms) {
        if (d->cf != b->cf || d->cT != b->cT)
            return fail(LBB_EINVAL, "batch members were stepped individually and are out of phase");
        if (d->poisoned) return fail(LBB_ESTATE, "a batch member is poisoned by an earlier invalid state");
    }
    return LBB_OK;
}

extern "C" int lbb_batch_step_async(lbb_batch *b, int64_t n)
{
    if (!b) return fail(LBB_EINVAL, "batch is NULL");
    if (n < 0) return fail(LBB_EINVAL, "n must be >= 0");
    int rc = batch_phase(b);
    if (rc) return rc;
    rc = batch_push(b);  // members' parameters may have changed through their handles
    if (rc) return rc;
    while (n >= kGraphSteps) {
        hipGraphExec_t &g = b->graph[b->cf][b->cT];
        if (!g) {
            const int cf = b->cf, cT = b->cT;
            LBB_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            for (int k = 0; k < kGraphSteps; ++k) batch_enqueue_step(b);
            hipGraph_t gr = nullptr;
            LBB_HIP(hipStreamEndCapture(b->stream, &gr));
            b->cf = cf;
            b->cT = cT;
            hipError_t e = hipGraphInstantiate(&g, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (e != hipSuccess) return fail(LBB_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        LBB_HIP(hipGraphLaunch(g, b->stream));
        n -= kGraphSteps;
    }
    for (int64_t k = 0; k < n; ++k) batch_enqueue_step(b);
    hipLaunchKernelGGL(lbb::k_flush_heat_flux, dim3((unsigned)b->doms.size()), dim3(lbb::NT), 0, b->stream, b->d_insts);
    LBB_HIP(hipGetLastError());
    for (lbb_domain *d : b->doms) {
        d->cf = b->cf;
        d->cT = b->cT;
    }
    return LBB_OK;
}

extern "C" int lbb_batch_sync(lbb_batch *b)
{
    if (!b) return fail(LBB_EINVAL, "batch is NULL");
    LBB_HIP(hipStreamSynchronize(b->stream));
    for (size_t i = 0; i < b->doms.size(); ++i) {
        int rc = check_errors(b->doms[i]);
        if (rc) return fail(rc, "batch member " + std::to_string(i) + ": " + g_err);
    }
    return LBB_OK;
}

extern "C" int lbb_batch_step(lbb_batch *b, int64_t n)
{
    int rc = lbb_batch_step_async(b, n);
    if (rc) return rc;
    return lbb_batch_sync(b);
}

extern "C" void *lbb_batch_stream(lbb_batch *b) { return b ? (void *)b->stream : nullptr; }

extern "C" int lbb_batch_heat_flux(lbb_batch *b, double *q_now, double *q_mean, int64_t *n_samples)
{
    if (!b) return fail(LBB_EINVAL, "batch is NULL");
    for (size_t i = 0; i < b->doms.size(); ++i) {
        double qn = 0, qm = 0;
        int64_t ns = 0;
        int rc = lbb_wall_heat_flux(b->doms[i], &qn, &qm, nullptr, &ns);
        if (rc) return rc;
        if (q_now) q_now[i] = qn;
        if (q_mean) q_mean[i] = qm;
        if (n_samples) n_samples[i] = ns;
    }
    return LBB_OK;
}

extern "C" lbb_domain *lbb_batch_domain(lbb_batch *b, int i)
{
    if (!b || i < 0 || i >= (int)b->doms.size()) return nullptr;
    return b->doms[i];
}

extern "C" int lbb_batch_size(lbb_batch *b) { return b ? (int)b->doms.size() : 0; }

extern "C" int lbb_batch_destroy(lbb_batch *b)
{
    if (!b) return fail(LBB_EINVAL, "batch is NULL");
    (void)hipStreamSynchronize(b->stream);
    batch_release(b);
    return LBB_OK;
}

}  // extern "C"

// ---- tile shapes and autotuning -------------------------------------------

namespace {

// Device copy of a lattice's current state, counters and heat-flux partials.
struct SavedState {
    void *f = nullptr, *T = nullptr;
    lbb::Scalars *sc = nullptr;
    double *hf = nullptr;
    ~SavedState()
    {
        for (void *q : {f, T, (void *)sc, (void *)hf})
            if (q) (void)hipFree(q);
    }
};

int save_state_dev(lbb_domain *d, int cf, int cT, SavedState &s, hipStream_t st)
{
    const size_t n = d->N, es = d->esz;
    LBB_HIP(hipMalloc(&s.f, 9 * n * es));
    LBB_HIP(hipMalloc(&s.T, n * es));
    LBB_HIP(hipMalloc((void **)&s.sc, sizeof(lbb::Scalars)));
    LBB_HIP(hipMalloc((void **)&s.hf, d->nbxB * sizeof(double)));
    LBB_HIP(hipMemcpyAsync(s.f, d->f[cf], 9 * n * es, hipMemcpyDeviceToDevice, st));
    LBB_HIP(hipMemcpyAsync(s.T, d->T[cT], n * es, hipMemcpyDeviceToDevice, st));
    LBB_HIP(hipMemcpyAsync(s.sc, d->sc, sizeof(lbb::Scalars), hipMemcpyDeviceToDevice, st));
    LBB_HIP(hipMemcpyAsync(s.hf, d->hf_part, d->nbxB * sizeof(double), hipMemcpyDeviceToDevice, st));
    return LBB_OK;
}

int restore_state_dev(lbb_domain *d, const SavedState &s, hipStream_t st)
{
    const size_t n = d->N, es = d->esz;
    LBB_HIP(hipMemcpyAsync(d->f[0], s.f, 9 * n * es, hipMemcpyDeviceToDevice, st));
    LBB_HIP(hipMemcpyAsync(d->T[0], s.T, n * es, hipMemcpyDeviceToDevice, st));
    LBB_HIP(hipMemcpyAsync(d->T[1], s.T, n * es, hipMemcpyDeviceToDevice, st));
    LBB_HIP(hipMemcpyAsync(d->sc, s.sc, sizeof(lbb::Scalars), hipMemcpyDeviceToDevice, st));
    LBB_HIP(hipMemcpyAsync(d->hf_part, s.hf, d->nbxB * sizeof(double), hipMemcpyDeviceToDevice, st));
    d->cf = d->cT = 0;
    d->poisoned = false;
    return LBB_OK;
}

int domain_set_tiles(lbb_domain *d, int a, int b)
{
    d->shA = a;
    d->shB = b;
    set_grid(d);
    drop_graphs(d);
    return push_inst(d);
}

bool valid_shapes(int a, int b) { return a >= 0 && a < lbb::NSHAPE_A && b >= 0 && b < lbb::NSHAPE_B; }

// Mean kernel durations (ms) of n batch steps, each launch carrying events
// that its dispatch records; the batch advances n steps.
template <typename S>
int batch_time_kernels(lbb_batch *b, int64_t n, double *ms_lb, double *ms_thermal)
{
    std::vector<hipEvent_t> ev(4 * (size_t)n, nullptr);
    for (auto &e : ev) LBB_HIP(hipEventCreate(&e));
    for (int64_t k = 0; k < n; ++k) {
        hipEvent_t *e = &ev[4 * k];
        launch_lb<S>(b->stream, b->d_insts, b->d_blkA, b->totA, b->cf, b->cT, b->shA, e[0], e[1]);
        launch_thermal<S>(b->stream, b->d_insts, b->d_blkB, b->totB, b->cf, b->cT, b->shB, e[2], e[3]);
        LBB_HIP(hipGetLastError());
        if (b->mode != LBB_THERMAL_ONLY) b->cf ^= 1;
        if (b->mode != LBB_ISOTHERMAL) b->cT ^= 1;
    }
    hipLaunchKernelGGL(lbb::k_flush_heat_flux, dim3((unsigned)b->doms.size()), dim3(lbb::NT), 0, b->stream, b->d_insts);
    LBB_HIP(hipStreamSynchronize(b->stream));
    double a = 0, c = 0;
    float ms = 0;
    for (int64_t k = 0; k < n; ++k) {
        LBB_HIP(hipEventElapsedTime(&ms, ev[4 * k], ev[4 * k + 1]));
        a += ms;
        LBB_HIP(hipEventElapsedTime(&ms, ev[4 * k + 2], ev[4 * k + 3]));
        c += ms;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    for (lbb_domain *d : b->doms) {
        d->cf = b->cf;
        d->cT = b->cT;
    }
    *ms_lb = a / (double)n;
    *ms_thermal = c / (double)n;
    for (size_t i = 0; i < b->doms.size(); ++i) {
        int rc = check_errors(b->doms[i]);
        if (rc) return fail(rc, "batch member " + std::to_string(i) + ": " + g_err);
    }
    return LBB_OK;
}

// Time every LB shape (thermal shape fixed), then every thermal shape (LB
// shape at its best), on the lattice's own state; keep the fastest of each
// when it beats the shape in use by more than kTuneMargin (timing noise is a
// few percent).  `set` applies a shape pair, `time` advances n steps and
// returns the mean kernel durations.
constexpr double kTuneMargin = 0.04;

template <typename Set, typename Time>
int tune_shapes(int steps, Set set, Time time, int a0, int b0, int *best_a, int *best_b, double *ms_lb,
                double *ms_thermal)
{
    double tA[lbb::NSHAPE_A], tB[lbb::NSHAPE_B];
    for (int a = 0; a < lbb::NSHAPE_A; ++a) {
        double ta, tb;
        int rc = set(a, b0);
        if (!rc) rc = time(1, &ta, &tb);  // first launches of the variant
        if (!rc) rc = time(steps, &ta, &tb);
        if (rc) return rc;
        tA[a] = ta;
        if (ms_lb) ms_lb[a] = ta;
    }
    int ba = 0;
    for (int a = 1; a < lbb::NSHAPE_A; ++a)
        if (tA[a] < tA[ba]) ba = a;
    if (!(tA[ba] < tA[a0] * (1.0 - kTuneMargin))) ba = a0;
    for (int t = 0; t < lbb::NSHAPE_B; ++t) {
        double ta, tb;
        int rc = set(ba, t);
        if (!rc) rc = time(1, &ta, &tb);
        if (!rc) rc = time(steps, &ta, &tb);
        if (rc) return rc;
        tB[t] = tb;
        if (ms_thermal) ms_thermal[t] = tb;
    }
    int bb = 0;
    for (int t = 1; t < lbb::NSHAPE_B; ++t)
        if (tB[t] < tB[bb]) bb = t;
    if (!(tB[bb] < tB[b0] * (1.0 - kTuneMargin))) bb = b0;
    *best_a = ba;
    *best_b = bb;
    return LBB_OK;
}

}  // namespace

extern "C" {

int lbb_tile_shapes(int32_t *n_lb, int32_t *n_thermal, int32_t *lb, int32_t *thermal)
{
    if (n_lb) *n_lb = lbb::NSHAPE_A;
    if (n_thermal) *n_thermal = lbb::NSHAPE_B;
    for (int i = 0; i < lbb::NSHAPE_A && lb; ++i) {
        lb[3 * i] = lbb::TXA;
        lb[3 * i + 1] = lbb::kShapeA[i].ty;
        lb[3 * i + 2] = lbb::kShapeA[i].nw;
    }
    for (int i = 0; i < lbb::NSHAPE_B && thermal; ++i) {
        thermal[3 * i] = lbb::TXB;
        thermal[3 * i + 1] = lbb::kShapeB[i].ty;
        thermal[3 * i + 2] = lbb::kShapeB[i].nw;
    }
    return LBB_OK;
}

int lbb_get_tiles(lbb_domain *d, int32_t *shape_lb, int32_t *shape_thermal)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    if (shape_lb) *shape_lb = d->shA;
    if (shape_thermal) *shape_thermal = d->shB;
    return LBB_OK;
}

int lbb_set_tiles(lbb_domain *d, int32_t shape_lb, int32_t shape_thermal)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    if (!valid_shapes(shape_lb, shape_thermal)) return fail(LBB_EINVAL, "unknown tile shape");
    LBB_HIP(hipStreamSynchronize(d->stream));
    return domain_set_tiles(d, shape_lb, shape_thermal);
}

int lbb_autotune(lbb_domain *d, int32_t steps, int32_t *shape_lb, int32_t *shape_thermal, double *ms_lb,
                 double *ms_thermal)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    if (steps < 1) return fail(LBB_EINVAL, "steps must be >= 1");
    if (d->poisoned) return fail(LBB_ESTATE, "domain poisoned by an earlier invalid state; load a state first");
    SavedState sv;
    int rc = save_state_dev(d, d->cf, d->cT, sv, d->stream);
    if (rc) return rc;
    int ba = d->shA, bb = d->shB;
    rc = tune_shapes(
        steps, [&](int a, int b) { return domain_set_tiles(d, a, b); },
        [&](int64_t n, double *ta, double *tb) {
            double tt;
            return lbb_time_kernels(d, n, ta, tb, &tt);
        },
        d->shA, d->shB, &ba, &bb, ms_lb, ms_thermal);
    const std::string err = rc ? g_err : std::string();
    const int rc2 = domain_set_tiles(d, ba, bb);
    const int rc3 = restore_state_dev(d, sv, d->stream);
    LBB_HIP(hipStreamSynchronize(d->stream));
    if (rc) return fail(rc, err);
    if (rc2) return rc2;
    if (rc3) return rc3;
    if (shape_lb) *shape_lb = ba;
    if (shape_thermal) *shape_thermal = bb;
    return LBB_OK;
}

int lbb_batch_set_tiles(lbb_batch *b, int32_t shape_lb, int32_t shape_thermal)
{
    if (!b) return fail(LBB_EINVAL, "batch is NULL");
    if (!valid_shapes(shape_lb, shape_thermal)) return fail(LBB_EINVAL, "unknown tile shape");
    LBB_HIP(hipStreamSynchronize(b->stream));
    b->shA = shape_lb;
    b->shB = shape_thermal;
    return batch_push(b);
}

int lbb_batch_autotune(lbb_batch *b, int32_t steps, int32_t *shape_lb, int32_t *shape_thermal, double *ms_lb,
                       double *ms_thermal)
{
    if (!b) return fail(LBB_EINVAL, "batch is NULL");
    if (steps < 1) return fail(LBB_EINVAL, "steps must be >= 1");
    int rc = batch_phase(b);
    if (rc) return rc;
    rc = batch_push(b);
    if (rc) return rc;
    std::vector<SavedState> sv(b->doms.size());
    for (size_t i = 0; i < b->doms.size() && !rc; ++i) rc = save_state_dev(b->doms[i], b->cf, b->cT, sv[i], b->stream);
    if (rc) return rc;
    int ba = b->shA, bb = b->shB;
    rc = tune_shapes(
        steps,
        [&](int a, int t) {
            b->shA = a;
            b->shB = t;
            return batch_push(b);
        },
        [&](int64_t n, double *ta, double *tb) {
            return b->precision == LBB_FP64 ? batch_time_kernels<double>(b, n, ta, tb)
                                            : batch_time_kernels<float>(b, n, ta, tb);
        },
        b->shA, b->shB, &ba, &bb, ms_lb, ms_thermal);
    const std::string err = rc ? g_err : std::string();
    b->shA = ba;
    b->shB = bb;
    int rc2 = batch_push(b);
    for (size_t i = 0; i < b->doms.size() && !rc2; ++i) rc2 = restore_state_dev(b->doms[i], sv[i], b->stream);
    b->cf = b->cT = 0;
    LBB_HIP(hipStreamSynchronize(b->stream));
    if (rc) return fail(rc, err);
    if (rc2) return rc2;
    if (shape_lb) *shape_lb = ba;
    if (shape_thermal) *shape_thermal = bb;
    return LBB_OK;
}

}  // extern "C"

// ---- adjoint --------------------------------------------------------------

namespace {

// Carves 256-byte aligned pieces out of one device allocation.
struct Carver {
    unsigned char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t n)
    {
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += (n * sizeof(T) + 255) & ~(size_t)255;
        return p;
    }
};

// The lattices of one adjoint run (a domain, or the members of a batch) and
// the forward launch tables that step them together on their own buffers.
struct AdjGroup {
    std::vector<lbb_domain *> doms;
    hipStream_t st = nullptr;
    const lbb::Inst *fwd_insts = nullptr;
    const int *blkA = nullptr, *blkB = nullptr;
    int totA = 0, totB = 0;
    std::vector<int> blkA0, blkB0;  // member offsets in the forward grids
    int *cf = nullptr, *cT = nullptr;
    int shA = 0, shB = 0;           // tile shapes of the forward launches
    void **mem = nullptr;           // cached workspace of the owner
    size_t *bytes = nullptr;
    int64_t *held = nullptr;        // the owner's bytes held against the budget
    // enqueue n forward steps of the owner on its stream (its graph path)
    std::function<int(int64_t)> advance;
};

// Per-lattice pieces of the workspace.
struct AdjMember {
    unsigned char *backup, *ck, *seg[2];
    lbb::Scalars *ck_sc;
    double *hf_backup, *lT[2], *gr[2];
    void *lf[2];  // population adjoints, storage precision
    lbb::AdjW w;
    int gx, nb, tgx, tnb;
    size_t n, state_bytes;
};

// Checkpoint interval when the caller leaves it open (K <= 0): every state
// kept (no recompute) when N + 2 stored states of all lattices take at most a
// quarter of the free device memory, else sqrt(N).
int64_t auto_K(const AdjGroup &g, int64_t N, size_t es)
{
    size_t per_state = 0;
    for (lbb_domain *d : g.doms) per_state += 10 * d->N * es;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    if ((double)(N + 2) * (double)per_state <= 0.25 * (double)free_b) return N;
    int64_t K = (int64_t)std::ceil(std::sqrt((double)N));
    return K < 1 ? 1 : K;
}

// Second stream and its two events for the recompute of the next segment,
// released on every return.
struct RecomputeStream {
    hipStream_t c = nullptr;
    hipEvent_t done = nullptr, free_buf = nullptr;
    hipError_t create()
    {
        hipError_t e = hipStreamCreateWithFlags(&c, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&free_buf, hipEventDisableTiming);
        return e;
    }
    ~RecomputeStream()
    {
        if (c) {
            (void)hipStreamSynchronize(c);
            (void)hipStreamDestroy(c);
        }
        if (done) (void)hipEventDestroy(done);
        if (free_buf) (void)hipEventDestroy(free_buf);
    }
};

// Reverse sweep with checkpoints every K steps.  With more than one segment
// the segment storage is doubled: while the reverse steps of segment s run on
// the group's stream from one buffer, a second stream recomputes segment
// s - 1 from its checkpoint into the other, so the recompute pass overlaps
// the reverse pass instead of adding to it.
template <typename S>
int adjoint_run(AdjGroup &g, int64_t N, int64_t K, double *J, double *dJ_dTb, double *dJ_dGw)
{
    using namespace lbb;
    const int nm = (int)g.doms.size();
    const size_t es = sizeof(S);
    const int64_t nck = (N + K - 1) / K;
    const int nbuf = nck > 1 ? 2 : 1;
    hipStream_t st = g.st;
    std::vector<AdjMember> m(nm);
    Inst *inst_seg = nullptr;  // [nbuf][K][nm]: step k of a segment reads stored state k, writes k+1
    AdjInst *d_ai = nullptr;
    int *d_amap = nullptr, *d_tmap = nullptr;
    int tot = 0, ttot = 0;
    for (int i = 0; i < nm; ++i) {
        const lbb_domain *d = g.doms[i];
        m[i].n = d->N;
        m[i].state_bytes = 10 * d->N * es;
        m[i].gx = (d->p.nx + AXB - 1) / AXB;
        m[i].nb = m[i].gx * ((d->p.ny + AYB - 1) / AYB);
        tot += m[i].nb;
    }
    // temperature-adjoint tiles: 16 rows high unless that gives fewer than
    // two tiles per compute unit, then 4 (16 waves either way; a 4-row tile
    // and its halo are 18 region rows, so most waves own one row and the
    // seven stencil phases are short)
    int tay = 16;
    {
        int t16 = 0;
        for (int i = 0; i < nm; ++i)
            t16 += ((g.doms[i]->p.nx + TAX - 1) / TAX) * ((g.doms[i]->p.ny + 15) / 16);
        if (t16 < 2 * 256) tay = 4;
        // 24-row tiles (LDS for one block per CU) cut the halo share where
        // there are at least four tiles per CU
        int t24 = 0;
        for (int i = 0; i < nm; ++i)
            t24 += ((g.doms[i]->p.nx + TAX - 1) / TAX) * ((g.doms[i]->p.ny + 23) / 24);
        if (t24 >= 4 * 256) tay = 24;
        // FP32 planes take half the LDS: 32-row tiles where there are at
        // least three per CU
        if (sizeof(S) == 4) {
            int t32 = 0;
            for (int i = 0; i < nm; ++i)
                t32 += ((g.doms[i]->p.nx + TAX - 1) / TAX) * ((g.doms[i]->p.ny + 31) / 32);
            if (t32 >= 3 * 256) tay = 32;
        }
    }
    for (int i = 0; i < nm; ++i) {
        const lbb_domain *d = g.doms[i];
        m[i].tgx = (d->p.nx + TAX - 1) / TAX;
        m[i].tnb = m[i].tgx * ((d->p.ny + tay - 1) / tay);
        ttot += m[i].tnb;
    }
    auto carve = [&](unsigned char *base) -> size_t {
        Carver cv{base};
        for (int i = 0; i < nm; ++i) {
            AdjMember &a = m[i];
            const size_t n = a.n;
            a.backup = cv.take<unsigned char>(a.state_bytes);
            a.ck = cv.take<unsigned char>((size_t)nck * a.state_bytes);
            for (int b = 0; b < 2; ++b)
                a.seg[b] = b < nbuf ? cv.take<unsigned char>((size_t)(K + 1) * a.state_bytes) : nullptr;
            a.ck_sc = cv.take<Scalars>((size_t)nck + 1);
            a.hf_backup = cv.take<double>(g.doms[i]->nbxB);
            for (int k = 0; k < 2; ++k) {
                a.lf[k] = cv.take<S>(9 * n);
                a.lT[k] = cv.take<double>(n);
                a.gr[k] = cv.take<double>(n);
            }
            AdjW &w = a.w;
            void **arr[] = {&w.rho, &w.jx, &w.jy, &w.psi, &w.T1, &w.sx, &w.sy, &w.Fx, &w.Fy, &w.vx,
                            &w.vy, &w.gDrx, &w.gDry, &w.gdiv, &w.grho, &w.gvx, &w.gvy, &w.gpsi, &w.gsx, &w.gsy};
            for (void **p : arr) *p = cv.take<S>(n);
            w.mpart = cv.take<double>(a.nb);
            w.fpart = cv.take<double>(2 * (size_t)a.nb);
            w.scal = cv.take<double>(4);
        }
        inst_seg = cv.take<Inst>((size_t)nbuf * K * nm);
        d_ai = cv.take<AdjInst>((size_t)nbuf * nm);
        d_amap = cv.take<int>(tot);
        d_tmap = cv.take<int>(ttot);
        return cv.off;
    };
    const size_t need = carve(nullptr);
    if (*g.bytes < need) {
        int rc = reserve_bytes((int64_t)need, "adjoint workspace");
        if (rc) return rc;
        if (*g.mem) {
            (void)hipStreamSynchronize(st);
            (void)hipFree(*g.mem);
            release_bytes((int64_t)*g.bytes);
            *g.held -= (int64_t)*g.bytes;
            *g.mem = nullptr;
            *g.bytes = 0;
        }
        if (hipMalloc(g.mem, need) != hipSuccess) {
            *g.mem = nullptr;
            release_bytes((int64_t)need);
            return fail(LBB_ENOMEM, "adjoint work memory could not be allocated");
        }
        *g.bytes = need;
        *g.held += (int64_t)need;
    }
    carve(static_cast<unsigned char *>(*g.mem));

    auto own_f = [&](int i) { return g.doms[i]->f[*g.cf]; };
    auto own_T = [&](int i) { return g.doms[i]->T[*g.cT]; };
    auto copy_state_out = [&](int i, unsigned char *dst) -> hipError_t {
        const size_t n = m[i].n;
        hipError_t e = hipMemcpyAsync(dst, own_f(i), 9 * n * es, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(dst + 9 * n * es, own_T(i), n * es, hipMemcpyDeviceToDevice, st);
        return e;
    };
    auto slot_step = [&](hipStream_t s, int b, int64_t k) {
        const Inst *tab = inst_seg + ((size_t)b * K + k) * nm;
        launch_lb<S>(s, tab, g.blkA, g.totA, 0, 0, g.shA);
        launch_thermal<S>(s, tab, g.blkB, g.totB, 0, 0, g.shB);
    };
    // buffer holding segment sg's states (the last segment uses buffer 0)
    auto buf_of = [&](int64_t sg) { return (int)((nck - 1 - sg) & 1); };
    RecomputeStream rs;
    if (nbuf > 1) LBB_HIP(rs.create());

    // keep each lattice's state, counters and heat-flux partials
    for (int i = 0; i < nm; ++i) {
        lbb_domain *d = g.doms[i];
        LBB_HIP(copy_state_out(i, m[i].backup));
        LBB_HIP(hipMemcpyAsync(&m[i].ck_sc[nck], d->sc, sizeof(Scalars), hipMemcpyDeviceToDevice, st));
        LBB_HIP(hipMemcpyAsync(m[i].hf_backup, d->hf_part, d->nbxB * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    // launch tables: stored-state steps and the adjoint grid
    std::vector<Inst> hinst((size_t)nbuf * K * nm);
    std::vector<AdjInst> hai((size_t)nbuf * nm);
    std::vector<int> hamap, htmap;
    hamap.reserve(tot);
    htmap.reserve(ttot);
    for (int i = 0; i < nm; ++i) {
        lbb_domain *d = g.doms[i];
        const size_t n = m[i].n;
        for (int b = 0; b < nbuf; ++b)
            for (int64_t k = 0; k < K; ++k) {
                Inst I = make_inst(d);
                S *x = reinterpret_cast<S *>(m[i].seg[b] + (size_t)k * m[i].state_bytes);
                S *y = reinterpret_cast<S *>(m[i].seg[b] + (size_t)(k + 1) * m[i].state_bytes);
                I.f[0] = x;
                I.f[1] = y;
                I.T[0] = x + 9 * n;
                I.T[1] = y + 9 * n;
                I.blkA0 = g.blkA0[i];
                I.blkB0 = g.blkB0[i];
                hinst[((size_t)b * K + k) * nm + i] = I;
            }
        AdjInst A{};
        A.P = d->dp;
        A.w = m[i].w;
        for (int k = 0; k < 2; ++k) {
            A.lf[k] = m[i].lf[k];
            A.lT[k] = m[i].lT[k];
            A.gr[k] = m[i].gr[k];
        }
        A.gx = m[i].gx;
        A.blk0 = (int)hamap.size();
        A.nb = m[i].nb;
        A.tgx = m[i].tgx;
        A.tblk0 = (int)htmap.size();
        for (int b = 0; b < nbuf; ++b) {
            A.seg = m[i].seg[b];
            hai[(size_t)b * nm + i] = A;
            hipLaunchKernelGGL(a_bcast_T<S>, dim3(256), dim3(256), 0, st, static_cast<const S *>(own_T(i)),
                               reinterpret_cast<S *>(m[i].seg[b]), n, (int)(K + 1));
        }
        hamap.insert(hamap.end(), m[i].nb, i);
        htmap.insert(htmap.end(), m[i].tnb, i);
    }
    LBB_HIP(hipMemcpyAsync(inst_seg, hinst.data(), hinst.size() * sizeof(Inst), hipMemcpyHostToDevice, st));
    LBB_HIP(hipMemcpyAsync(d_ai, hai.data(), hai.size() * sizeof(AdjInst), hipMemcpyHostToDevice, st));
    LBB_HIP(hipMemcpyAsync(d_amap, hamap.data(), tot * sizeof(int), hipMemcpyHostToDevice, st));
    LBB_HIP(hipMemcpyAsync(d_tmap, htmap.data(), ttot * sizeof(int), hipMemcpyHostToDevice, st));

    // forward with the averages restarted: J = q_sum / N afterwards.  States
    // of the last segment go straight into the slots (no recompute later).
    std::vector<Scalars> s0(nm);
    for (int i = 0; i < nm; ++i)
        LBB_HIP(hipMemcpyAsync(&s0[i], g.doms[i]->sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    LBB_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < nm; ++i) {
        s0[i].q_sum = 0.0;
        s0[i].n_samples = 0;
        LBB_HIP(hipMemcpyAsync(g.doms[i]->sc, &s0[i], sizeof(Scalars), hipMemcpyHostToDevice, st));
    }
    // Up to the last segment the owner steps through its own graphs, K steps
    // from one checkpoint to the next (tL is a multiple of K).
    const int64_t tL = (nck - 1) * K;
    for (int64_t t = 0; t < N;) {
        if (t % K == 0)
            for (int i = 0; i < nm; ++i) {
                LBB_HIP(copy_state_out(i, t < tL ? m[i].ck + (size_t)(t / K) * m[i].state_bytes : m[i].seg[0]));
                LBB_HIP(hipMemcpyAsync(&m[i].ck_sc[t / K], g.doms[i]->sc, sizeof(Scalars), hipMemcpyDeviceToDevice,
                                       st));
            }
        if (t < tL) {
            const int rc = g.advance(K);
            if (rc) return rc;
            t += K;
        } else {
            slot_step(st, 0, t - tL);
            LBB_HIP(hipGetLastError());
            ++t;
        }
    }
    hipLaunchKernelGGL(k_flush_heat_flux, dim3(nm), dim3(NT), 0, st, g.fwd_insts);
    LBB_HIP(hipStreamSynchronize(st));
    std::vector<Scalars> s1(nm);
    for (int i = 0; i < nm; ++i) {
        int rc = check_errors(g.doms[i]);
        if (rc) return nm > 1 ? fail(rc, "batch member " + std::to_string(i) + ": " + g_err) : rc;
        LBB_HIP(hipMemcpyAsync(&s1[i], g.doms[i]->sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    }
    LBB_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < nm; ++i) J[i] = s1[i].q_sum / (double)N;

    // reverse sweep: the adjoint of the final state starts from its heat-flux sample
    const double wq = 1.0 / (double)N;
    for (int i = 0; i < nm; ++i) {
        LBB_HIP(hipMemsetAsync(m[i].lf[0], 0, 9 * m[i].n * es, st));
        LBB_HIP(hipMemsetAsync(m[i].lT[0], 0, m[i].n * sizeof(double), st));
        LBB_HIP(hipMemsetAsync(m[i].gr[0], 0, m[i].n * sizeof(double), st));
        LBB_HIP(hipMemsetAsync(m[i].w.scal, 0, 4 * sizeof(double), st));
    }
    const dim3 grid(tot), blk(NTA);
    int cur = 0;
    hipLaunchKernelGGL(a_hf<S>, grid, blk, 0, st, d_ai, d_amap, (int)(N - tL), wq, cur);
    // recompute of segment sg from its checkpoint into its buffer, on the
    // second stream once the reverse steps that last read that buffer are done
    auto recompute = [&](int64_t sg) -> hipError_t {
        const int64_t t0 = sg * K, t1 = (t0 + K < N) ? t0 + K : N;
        const int b = buf_of(sg);
        hipError_t e = hipEventRecord(rs.free_buf, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(rs.c, rs.free_buf, 0);
        for (int i = 0; i < nm && e == hipSuccess; ++i) {
            e = hipMemcpyAsync(m[i].seg[b], m[i].ck + (size_t)sg * m[i].state_bytes, m[i].state_bytes,
                               hipMemcpyDeviceToDevice, rs.c);
            if (e == hipSuccess)
                e = hipMemcpyAsync(g.doms[i]->sc, &m[i].ck_sc[sg], sizeof(Scalars), hipMemcpyDeviceToDevice, rs.c);
        }
        if (e != hipSuccess) return e;
        for (int64_t t = t0; t + 1 < t1; ++t) slot_step(rs.c, b, t - t0);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(rs.done, rs.c);
        return e;
    };
    for (int64_t sg = nck - 1; sg >= 0; --sg) {
        const int64_t t0 = sg * K, t1 = (t0 + K < N) ? t0 + K : N;
        const AdjInst *ai = d_ai + (size_t)buf_of(sg) * nm;
        if (sg < nck - 1) LBB_HIP(hipStreamWaitEvent(st, rs.done, 0));  // segment sg recomputed
        if (sg > 0) LBB_HIP(recompute(sg - 1));
        hipLaunchKernelGGL(a_macro<S>, grid, blk, 0, st, ai, d_amap, (int)(t1 - 1 - t0));
        for (int64_t t = t1 - 1; t >= t0; --t) {
            const int k = (int)(t - t0);
            if (tay == 32) {
                if constexpr (sizeof(S) == 4)
                    hipLaunchKernelGGL((a_theradj<S, 32, 16>), dim3(ttot), dim3(64 * 16), 0, st, ai, d_tmap, cur);
            } else if (tay == 24) hipLaunchKernelGGL((a_theradj<S, 24, 16>), dim3(ttot), dim3(64 * 16), 0, st, ai, d_tmap, cur);
            else if (tay == 16) hipLaunchKernelGGL((a_theradj<S, 16, 16>), dim3(ttot), dim3(64 * 16), 0, st, ai, d_tmap, cur);
            else hipLaunchKernelGGL((a_theradj<S, 4, 16>), dim3(ttot), dim3(64 * 16), 0, st, ai, d_tmap, cur);
            hipLaunchKernelGGL(a_lb<S>, grid, blk, 0, st, ai, d_amap, k, cur);
            hipLaunchKernelGGL(a_final<S>, grid, blk, 0, st, ai, d_amap, k, cur, t >= 1 ? wq : 0.0,
                               t > t0 ? 1 : 0);
            cur ^= 1;
        }
        LBB_HIP(hipGetLastError());
    }
    // gradients: row 0 of the adjoint of T^0, and the accumulated G_w part
    std::vector<std::vector<double>> gT(nm);
    std::vector<double> gGw(nm, 0.0);
    for (int i = 0; i < nm; ++i) {
        gT[i].resize(g.doms[i]->p.nx);
        LBB_HIP(hipMemcpyAsync(gT[i].data(), m[i].lT[cur], gT[i].size() * sizeof(double), hipMemcpyDeviceToHost, st));
        LBB_HIP(hipMemcpyAsync(&gGw[i], m[i].w.scal + 2, sizeof(double), hipMemcpyDeviceToHost, st));
    }
    // restore every lattice's state
    for (int i = 0; i < nm; ++i) {
        lbb_domain *d = g.doms[i];
        const size_t n = m[i].n;
        LBB_HIP(hipMemcpyAsync(d->f[0], m[i].backup, 9 * n * es, hipMemcpyDeviceToDevice, st));
        LBB_HIP(hipMemcpyAsync(d->T[0], m[i].backup + 9 * n * es, n * es, hipMemcpyDeviceToDevice, st));
        LBB_HIP(hipMemcpyAsync(d->T[1], m[i].backup + 9 * n * es, n * es, hipMemcpyDeviceToDevice, st));
        LBB_HIP(hipMemcpyAsync(d->sc, &m[i].ck_sc[nck], sizeof(Scalars), hipMemcpyDeviceToDevice, st));
        LBB_HIP(hipMemcpyAsync(d->hf_part, m[i].hf_backup, d->nbxB * sizeof(double), hipMemcpyDeviceToDevice, st));
        d->cf = d->cT = 0;
    }
    *g.cf = *g.cT = 0;
    LBB_HIP(hipStreamSynchronize(st));
    size_t off = 0;
    for (int i = 0; i < nm; ++i) {
        for (double v : gT[i])
            if (!std::isfinite(v)) return fail(LBB_ENONFINITE, "adjoint produced a non-finite gradient");
        if (dJ_dTb) std::memcpy(dJ_dTb + off, gT[i].data(), gT[i].size() * sizeof(double));
        if (dJ_dGw) dJ_dGw[i] = gGw[i];
        off += gT[i].size();
    }
    return LBB_OK;
}

int adjoint_checks(const lbb_domain *d)
{
    if (d->p.periodic_y || d->p.thermal_mode != LBB_COUPLED)
        return fail(LBB_EUNSUPPORTED, "the adjoint covers the coupled model with walls");
    if (d->p.ghost_layer)
        return fail(LBB_EUNSUPPORTED, "the adjoint does not cover the ghost-layer wall variant");
    if (d->poisoned) return fail(LBB_ESTATE, "domain poisoned by an earlier invalid state; load a state first");
    return LBB_OK;
}

int adjoint_group(AdjGroup &g, int precision, int64_t N, int64_t K, double *J, double *dJ_dTb, double *dJ_dGw)
{
    if (K <= 0) K = auto_K(g, N, precision == LBB_FP64 ? 8 : 4);
    if (K > N) K = N;
    return precision == LBB_FP64 ? adjoint_run<double>(g, N, K, J, dJ_dTb, dJ_dGw)
                                 : adjoint_run<float>(g, N, K, J, dJ_dTb, dJ_dGw);
}

}  // namespace

extern "C" int lbb_adjoint(lbb_domain *d, int64_t N, int64_t K, const int32_t *heater_idx, int32_t n_heater,
                           double *J, double *dJ_dTb, double *dJ_dGw)
{
    if (!d || !J) return fail(LBB_EINVAL, "domain and J are required");
    if (N < 1) return fail(LBB_EINVAL, "N must be >= 1");
    if (!heater_idx && dJ_dTb && n_heater != d->p.nx) return fail(LBB_EINVAL, "without heater_idx, n_heater must be nx");
    if (heater_idx && n_heater < 0) return fail(LBB_EINVAL, "n_heater must be >= 0");
    if (heater_idx)
        for (int32_t k = 0; k < n_heater; ++k)
            if (heater_idx[k] < 0 || heater_idx[k] >= d->p.nx) return fail(LBB_EINVAL, "heater index outside [0, nx)");
    // the gradient over the whole bottom wall, then the heater nodes' entries
    std::vector<double> gTb(dJ_dTb ? (size_t)d->p.nx : 0);
    int rc = adjoint_checks(d);
    if (rc) return rc;
    AdjGroup g;
    g.doms = {d};
    g.st = d->stream;
    g.fwd_insts = d->d_inst;
    g.blkA = d->d_blkA;
    g.blkB = d->d_blkB;
    g.totA = d->nbxA * d->nbyA + 1;
    g.totB = d->nbxB * d->nbyB + 1;
    g.blkA0 = {0};
    g.blkB0 = {0};
    g.cf = &d->cf;
    g.cT = &d->cT;
    g.shA = d->shA;
    g.shB = d->shB;
    const size_t before = d->adj_bytes;
    g.mem = &d->adj_mem;
    g.bytes = &d->adj_bytes;
    g.held = &d->held;
    g.advance = [d](int64_t n) { return enqueue_steps(d, n); };
    rc = adjoint_group(g, d->p.precision, N, K, J, dJ_dTb ? gTb.data() : nullptr, dJ_dGw);
    d->dev_bytes += (int64_t)d->adj_bytes - (int64_t)before;
    if (rc == LBB_OK && dJ_dTb)
        for (int32_t k = 0; k < (heater_idx ? n_heater : d->p.nx); ++k) dJ_dTb[k] = gTb[heater_idx ? heater_idx[k] : k];
    return rc;
}

extern "C" int lbb_batch_adjoint(lbb_batch *b, int64_t N, int64_t K, double *J, double *dJ_dTb, double *dJ_dGw)
{
    if (!b || !J) return fail(LBB_EINVAL, "batch and J are required");
    if (N < 1) return fail(LBB_EINVAL, "N must be >= 1");
    int rc = batch_phase(b);
    if (rc) return rc;
    for (size_t i = 0; i < b->doms.size(); ++i) {
        rc = adjoint_checks(b->doms[i]);
        if (rc) return fail(rc, "batch member " + std::to_string(i) + ": " + g_err);
    }
    rc = batch_push(b);
    if (rc) return rc;
    AdjGroup g;
    g.doms = b->doms;
    g.st = b->stream;
    g.fwd_insts = b->d_insts;
    g.blkA = b->d_blkA;
    g.blkB = b->d_blkB;
    g.totA = b->totA;
    g.totB = b->totB;
    int a0 = 0, b0 = 0;
    for (lbb_domain *d : b->doms) {
        g.blkA0.push_back(a0);
        g.blkB0.push_back(b0);
        a0 += d->nbxA * d->nbyA + 1;
        b0 += d->nbxB * d->nbyB + 1;
    }
    g.cf = &b->cf;
    g.cT = &b->cT;
    g.shA = b->shA;
    g.shB = b->shB;
    g.mem = &b->adj_mem;
    g.bytes = &b->adj_bytes;
    g.held = &b->held;
    g.advance = [b](int64_t n) { return lbb_batch_step_async(b, n); };
    return adjoint_group(g, b->precision, N, K, J, dJ_dTb, dJ_dGw);
}

extern "C" int lbb_set_device_budget(int64_t bytes)
{
    if (bytes < 0) return fail(LBB_EINVAL, "the budget must be >= 0 (0: none)");
    g_budget.store(bytes);
    return LBB_OK;
}

extern "C" int64_t lbb_device_bytes_held(void) { return g_held.load(); }

extern "C" int lbb_batch_info(lbb_batch *b, int64_t *device_bytes)
{
    if (!b) return fail(LBB_EINVAL, "batch is NULL");
    if (device_bytes) {
        int64_t s = (int64_t)b->adj_bytes;
        for (lbb_domain *d : b->doms) s += d->dev_bytes;
        *device_bytes = s;
    }
    return LBB_OK;
}

extern "C" {

int lbb_destroy(lbb_domain *d)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    if (d->stream) (void)hipStreamSynchronize(d->stream);
    release(d);
    return LBB_OK;
}

}  // extern "C"

// ---- stepping without allocation -----------------------------------------
//
// The per-block partial sums, the one-entry launch table, the block maps and
// the scalars of lbb_step_noalloc live in this array.  Its host-side name
// is only a stand-in for the symbol: the device address of each GPU's copy
// comes from hipGetSymbolAddress (noalloc_scratch below), and only that
// address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[LBB_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

// Device address of `scratch` on device `dev`, resolved once per device
// with that device current.
int noalloc_scratch(int dev, unsigned char **out)
{
    static std::mutex mu;
    static unsigned char *addr[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) return fail(LBB_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LBB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        addr[dev] = static_cast<unsigned char *>(p);
    }
    *out = addr[dev];
    return LBB_OK;
}

// Byte offsets of the pieces of the scratch array for one lattice (default
// tile shapes), each 256-byte aligned; `total` is the bytes needed.
struct NoallocLayout {
    size_t inst, sc, blkA, blkB, mass, hf, total;
    int nbxA, nbyA, nbxB, nbyB;
};

NoallocLayout noalloc_layout(int nx, int ny)
{
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    NoallocLayout L{};
    L.nbxA = (nx + lbb::TXA - 1) / lbb::TXA;
    L.nbyA = (ny + lbb::kShapeA[0].ty - 1) / lbb::kShapeA[0].ty;
    L.nbxB = (nx + lbb::TXB - 1) / lbb::TXB;
    L.nbyB = (ny + lbb::kShapeB[0].ty - 1) / lbb::kShapeB[0].ty;
    const size_t nA = (size_t)L.nbxA * L.nbyA + 1, nB = (size_t)L.nbxB * L.nbyB + 1;
    const size_t nmass = std::max((size_t)L.nbxA * ny, (size_t)L.nbxA * L.nbyA);
    size_t o = 0;
    L.inst = o;
    o += up(sizeof(lbb::Inst));
    L.sc = o;
    o += up(sizeof(lbb::Scalars));
    L.blkA = o;
    o += up(nA * sizeof(int));
    L.blkB = o;
    o += up(nB * sizeof(int));
    L.mass = o;
    o += up(nmass * sizeof(double));
    L.hf = o;
    o += up((size_t)L.nbxB * sizeof(double));
    L.total = o;
    return L;
}

// Launch table, zeroed block maps (a single lattice: every block belongs to
// entry 0) and reset scalars, written by a kernel so that nothing is copied
// from host memory and no memset node is involved.
__global__ void k_noalloc_setup(lbb::Inst I, lbb::Inst *inst, int *blkA, int nA, int *blkB, int nB, lbb::Scalars *sc)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    if (tid == 0) {
        *inst = I;
        lbb::Scalars s{};
        s.err_step = ~0ULL;
        *sc = s;
    }
    for (int k = tid; k < nA; k += stride) blkA[k] = 0;
    for (int k = tid; k < nB; k += stride) blkB[k] = 0;
}

__global__ void k_noalloc_result(const lbb::Scalars *sc, lbb_noalloc_result *out)
{
    if (threadIdx.x != 0) return;
    lbb_noalloc_result r{};
    r.q_now = sc->q_now;
    r.n_samples = sc->n_samples;
    r.q_mean = sc->n_samples > 0 ? sc->q_sum / (double)sc->n_samples : __builtin_nan("");
    r.err_step = sc->err_step == ~0ULL ? -1 : (int64_t)sc->err_step;
    r.err_code = sc->err_code;
    *out = r;
}

// The work of lbb_step_noalloc after validation: the set-up reductions of
// the given state (as lbb_init_domain's), n steps of single launches, the
// final heat-flux bookkeeping and the result.
template <typename S>
void noalloc_enqueue(const lbb::Inst &I, unsigned char *base, const NoallocLayout &L, int &cf, int &cT, int64_t n,
                     lbb_noalloc_result *result, hipStream_t st)
{
    using namespace lbb;
    Inst *inst = reinterpret_cast<Inst *>(base + L.inst);
    Scalars *sc = reinterpret_cast<Scalars *>(base + L.sc);
    int *blkA = reinterpret_cast<int *>(base + L.blkA);
    int *blkB = reinterpret_cast<int *>(base + L.blkB);
    const int nA = L.nbxA * L.nbyA + 1, nB = L.nbxB * L.nbyB + 1;
    hipLaunchKernelGGL(k_noalloc_setup, dim3((std::max(nA, nB) + 255) / 256), dim3(256), 0, st, I, inst, blkA, nA,
                       blkB, nB, sc);
    const int nm = L.nbxA * L.nbyA;
    const S *f = static_cast<const S *>(I.f[cf]);
    hipLaunchKernelGGL(k_mass<S>, dim3(nm), dim3(NT), 0, st, I.P, f, I.mass_part);
    hipLaunchKernelGGL(k_reduce_mass, dim3(1), dim3(NT), 0, st, I.P, I.mass_part, nm, sc);
    hipLaunchKernelGGL(k_heat_flux_state<S>, dim3(L.nbxB), dim3(64), 0, st, I.P, f,
                       static_cast<const S *>(I.T[cT]), I.hf_part, (double *)nullptr);
    hipLaunchKernelGGL(k_flush_heat_flux, dim3(1), dim3(NT), 0, st, inst);
    for (int64_t k = 0; k < n; ++k) {
        launch_lb<S>(st, inst, blkA, nA, cf, cT, 0);
        launch_thermal<S>(st, inst, blkB, nB, cf, cT, 0);
        if (I.P.mode != MODE_THERMAL_ONLY) cf ^= 1;
        if (I.P.mode != MODE_ISOTHERMAL) cT ^= 1;
    }
    hipLaunchKernelGGL(k_flush_heat_flux, dim3(1), dim3(NT), 0, st, inst);
    hipLaunchKernelGGL(k_noalloc_result, dim3(1), dim3(64), 0, st, sc, result);
}

}  // namespace

extern "C" int lbb_step_noalloc(const lbb_params *pin, void *const f[2], void *const T[2], void *rho, void *vx,
                                void *vy, int32_t phase[2], int64_t n, lbb_noalloc_result *result, void *stream)
{
    int rc = validate(pin);
    if (rc) return rc;
    if (!f || !T || !f[0] || !f[1] || !T[0] || !T[1] || !rho || !vx || !vy || !phase || !result)
        return fail(LBB_EINVAL, "lbb_step_noalloc: every buffer, phase and result are required");
    if (n < 0) return fail(LBB_EINVAL, "lbb_step_noalloc: n must be >= 0");
    if ((phase[0] != 0 && phase[0] != 1) || (phase[1] != 0 && phase[1] != 1))
        return fail(LBB_EINVAL, "lbb_step_noalloc: phase entries must be 0 or 1");
    lbb_params p = *pin;
    double Tc = 0, kap = 0;
    lbb_eos_constants(p.a, p.b, p.R, p.omega, &Tc, &kap);
    if (p.rho_L == 0.0 && p.rho_V == 0.0) {
        rc = lbb_coexistence(p.a, p.b, p.R, p.omega, p.Ts_over_Tc * Tc, &p.rho_V, &p.rho_L);
        if (rc) return fail(LBB_EINVAL, "rho_L = rho_V = 0 needs T_s < T_c for the Maxwell densities");
    }
    if (p.rho_L == p.rho_V) return fail(LBB_EINVAL, "rho_L must differ from rho_V");
    const NoallocLayout L = noalloc_layout(p.nx, p.ny);
    if (L.total > LBB_NOALLOC_SCRATCH_BYTES)
        return fail(LBB_EINVAL, "lbb_step_noalloc: a " + std::to_string(p.nx) + "x" + std::to_string(p.ny) +
                                    " lattice needs " + std::to_string(L.total) + " scratch bytes, more than the " +
                                    std::to_string((size_t)LBB_NOALLOC_SCRATCH_BYTES) + " the library holds");
    int dev = 0;
    LBB_HIP(hipGetDevice(&dev));
    unsigned char *base = nullptr;
    rc = noalloc_scratch(dev, &base);
    if (rc) return rc;
    lbb::Inst I{};
    make_dev_params(p, Tc, kap, I.P);
    I.f[0] = f[0];
    I.f[1] = f[1];
    I.T[0] = T[0];
    I.T[1] = T[1];
    I.rho = rho;
    I.vx = vx;
    I.vy = vy;
    I.mass_part = reinterpret_cast<double *>(base + L.mass);
    I.hf_part = reinterpret_cast<double *>(base + L.hf);
    I.sc = reinterpret_cast<lbb::Scalars *>(base + L.sc);
    I.nbxA = L.nbxA;
    I.nbyA = L.nbyA;
    I.nbxB = L.nbxB;
    I.nbyB = L.nbyB;
    int cf = phase[0], cT = phase[1];
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (p.precision == LBB_FP64) noalloc_enqueue<double>(I, base, L, cf, cT, n, result, st);
    else noalloc_enqueue<float>(I, base, L, cf, cT, n, result, st);
    LBB_HIP(hipGetLastError());
    phase[0] = cf;
    phase[1] = cT;
    return LBB_OK;
}

// ---- three-dimensional lattices ------------------------------------------
#include "lbb3_host.hpp"
