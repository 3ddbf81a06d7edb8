// Host runtime of the three-dimensional path (D3Q19; include/lbboil.h,
// "Three-dimensional lattices").  Included at the end of lbb_host.hip: it
// uses that file's validation, device-parameter set-up, error reporting and
// device-memory budget.
#pragma once

#include "lbb3_device.hpp"

struct lbb3_domain {
    lbb_params p{};
    lbb::DevParams dp{};
    lbb3::Geom3 g{};
    size_t esz = 8;
    hipStream_t stream = nullptr;
    void *f[2] = {nullptr, nullptr};
    void *T[2] = {nullptr, nullptr};
    void *rho = nullptr, *v = nullptr, *coef = nullptr, *Ts = nullptr, *acc = nullptr;
    double *psi = nullptr, *mpart = nullptr, *hpart = nullptr, *Tb_dev = nullptr;
    lbb3::Scalars3 *sc = nullptr;
    int nb = 0;   // blocks of the per-node launches
    int ncu = 0;  // compute units of the device
    int cf = 0, cT = 0;
    bool poisoned = false;
    hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    std::vector<void *> allocs;
    int64_t held = 0;
};

namespace {

void release3(lbb3_domain *d)
{
    for (auto &row : d->graph)
        for (auto &g : row)
            if (g) (void)hipGraphExecDestroy(g);
    for (void *p : d->allocs) (void)hipFree(p);
    if (d->stream) (void)hipStreamDestroy(d->stream);
    release_bytes(d->held);
    delete d;
}

// The state reductions of the current state (rho_ave, heat-flux sample):
// psi and rho of the current state, then one reduction block.
template <typename S>
void enqueue_reductions3(lbb3_domain *d, int advance)
{
    using namespace lbb3;
    S *v = static_cast<S *>(d->v);
    hipLaunchKernelGGL(k3_psi<S>, dim3(d->nb), dim3(NT3), 0, d->stream, d->dp, d->g,
                       static_cast<const S *>(d->f[d->cf]), static_cast<const S *>(d->T[d->cT]),
                       static_cast<S *>(d->rho), d->psi, v, v + d->g.n, v + 2 * (size_t)d->g.n, d->mpart, d->hpart,
                       d->sc);
    hipLaunchKernelGGL(k3_reduce, dim3(1), dim3(NR3), 0, d->stream, d->g, d->mpart, d->hpart, d->nb, d->sc, advance);
}

// Column tiles and plane runs of the first RK4 stage.  The runs are sized
// for about `target` blocks: in FP32 (a 30 KB ring, four blocks a CU) short
// runs of about three planes, several rounds of blocks; in FP64 (a 60 KB
// ring, two blocks a CU) one round of long runs.  Timed on the 150 x 151 x
// 150 pool: FP32 337.6 us per step with runs of 3 planes against 338.6-340.2
// with runs of 2 to 9, FP64 626.2 us with runs of 17 against 632-638 with
// shorter ones.
lbb3::Tiles3 stage0_tiles(const lbb3::Geom3 &g, int target)
{
    using namespace lbb3;
    Tiles3 t{(g.nx + TXZ - 1) / TXZ, (g.ny + TYZ - 1) / TYZ, 1, g.nz};
    const int runs = std::max(1, std::min(g.nz, target / (t.ntx * t.nty)));
    t.zc = (g.nz + runs - 1) / runs;
    t.ntz = (g.nz + t.zc - 1) / t.zc;
    return t;
}

// One time step: reductions of state t, LB update, RK4 temperature step.
template <typename S>
void enqueue_step3(lbb3_domain *d)
{
    using namespace lbb3;
    enqueue_reductions3<S>(d, 1);
    const size_t n = d->g.n;
    S *v = static_cast<S *>(d->v);
    if (d->dp.mode != lbb::MODE_THERMAL_ONLY)
        hipLaunchKernelGGL(k3_lb<S>, dim3(d->nb), dim3(NT3), 0, d->stream, d->dp, d->g,
                           static_cast<const S *>(d->f[d->cf]), static_cast<S *>(d->f[d->cf ^ 1]), d->psi, v,
                           v + n, v + 2 * n, d->sc);
    if (d->dp.mode != lbb::MODE_ISOTHERMAL) {
        const S *T0 = static_cast<const S *>(d->T[d->cT]);
        S *T1 = static_cast<S *>(d->T[d->cT ^ 1]);
        S *Ts0 = static_cast<S *>(d->Ts), *Ts1 = Ts0 + n;
        S *acc = static_cast<S *>(d->acc), *coef = static_cast<S *>(d->coef);
        const S *rho = static_cast<const S *>(d->rho);
        const Tiles3 tl = stage0_tiles(d->g, (sizeof(S) == 4 ? 16 : 2) * d->ncu);
        hipLaunchKernelGGL(k3_stage0<S>, dim3(tl.ntx * tl.nty * tl.ntz), dim3(NSZ), 0, d->stream, d->dp, d->g, tl, T0,
                           Ts0, acc, coef, rho, v, v + n, v + 2 * n);
        hipLaunchKernelGGL((k3_stage<S, 1>), dim3(d->nb), dim3(NT3), 0, d->stream, d->dp, d->g, T0, Ts0, Ts1, acc,
                           coef, d->sc);
        hipLaunchKernelGGL((k3_stage<S, 2>), dim3(d->nb), dim3(NT3), 0, d->stream, d->dp, d->g, T0, Ts1, Ts0, acc,
                           coef, d->sc);
        hipLaunchKernelGGL((k3_stage<S, 3>), dim3(d->nb), dim3(NT3), 0, d->stream, d->dp, d->g, T0, Ts0, T1, acc,
                           coef, d->sc);
    }
    if (d->dp.mode != lbb::MODE_THERMAL_ONLY) d->cf ^= 1;
    if (d->dp.mode != lbb::MODE_ISOTHERMAL) d->cT ^= 1;
}

void enqueue_step3_any(lbb3_domain *d)
{
    if (d->p.precision == LBB_FP64) enqueue_step3<double>(d);
    else enqueue_step3<float>(d);
}

void enqueue_reductions3_any(lbb3_domain *d, int advance)
{
    if (d->p.precision == LBB_FP64) enqueue_reductions3<double>(d, advance);
    else enqueue_reductions3<float>(d, advance);
}

int build_graph3(lbb3_domain *d, hipGraphExec_t *out)
{
    const int cf = d->cf, cT = d->cT;
    LBB_HIP(hipStreamBeginCapture(d->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < kGraphSteps; ++k) enqueue_step3_any(d);
    hipGraph_t g = nullptr;
    LBB_HIP(hipStreamEndCapture(d->stream, &g));
    d->cf = cf;
    d->cT = cT;
    const hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LBB_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    return LBB_OK;
}

int enqueue_steps3(lbb3_domain *d, int64_t n)
{
    while (n >= kGraphSteps) {
        hipGraphExec_t &g = d->graph[d->cf][d->cT];
        if (!g) {
            const int rc = build_graph3(d, &g);
            if (rc) return rc;
        }
        LBB_HIP(hipGraphLaunch(g, d->stream));
        n -= kGraphSteps;  // an even count: the buffers return to their parity
    }
    for (int64_t k = 0; k < n; ++k) enqueue_step3_any(d);
    enqueue_reductions3_any(d, 0);  // rho_ave and the heat-flux sample of the final state
    LBB_HIP(hipGetLastError());
    return LBB_OK;
}

int check_errors3(lbb3_domain *d)
{
    lbb3::Scalars3 s;
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

// f = f_eq(rho, u), T with the Dirichlet rows; counters reset
template <typename S>
int set_state3(lbb3_domain *d, const double *rho, const double *u, const double *T)
{
    const size_t n = d->g.n;
    double *buf = nullptr;
    LBB_HIP(hipMalloc(&buf, 5 * n * sizeof(double)));
    int rc = LBB_OK;
    do {
        if (hipMemcpyAsync(buf, rho, n * sizeof(double), hipMemcpyHostToDevice, d->stream) != hipSuccess ||
            (u && hipMemcpyAsync(buf + n, u, 3 * n * sizeof(double), hipMemcpyHostToDevice, d->stream) != hipSuccess) ||
            (T && hipMemcpyAsync(buf + 4 * n, T, n * sizeof(double), hipMemcpyHostToDevice, d->stream) != hipSuccess)) {
            rc = fail(LBB_EDEVICE, "upload of the initial fields failed");
            break;
        }
        lbb3::Scalars3 s{};
        s.err_step = ~0ULL;
        if (hipMemcpyAsync(d->sc, &s, sizeof s, hipMemcpyHostToDevice, d->stream) != hipSuccess) {
            rc = fail(LBB_EDEVICE, "scalar reset failed");
            break;
        }
        hipLaunchKernelGGL(lbb3::k3_set_state<S>, dim3(d->nb), dim3(lbb3::NT3), 0, d->stream, d->dp, d->g, buf,
                           u ? buf + n : nullptr, T ? buf + 4 * n : nullptr, d->Tb_dev, static_cast<S *>(d->f[0]),
                           static_cast<S *>(d->T[0]), static_cast<S *>(d->T[1]), d->sc);
        d->cf = d->cT = 0;
        enqueue_reductions3<S>(d, 0);
        if (hipStreamSynchronize(d->stream) != hipSuccess) {
            rc = fail(LBB_EDEVICE, "set-up kernels failed");
            break;
        }
    } while (0);
    (void)hipFree(buf);
    if (rc) return rc;
    return check_errors3(d);
}

}  // namespace

extern "C" {

int lbb3_init_domain(const lbb_params *pin, int32_t nz, const double *T_bottom, const double *rho0,
                     lbb3_domain **out)
{
    if (!out) return fail(LBB_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(pin);
    if (rc) return rc;
    if (pin->ghost_layer) return fail(LBB_EUNSUPPORTED, "the ghost-layer wall is two-dimensional only");
    if (nz < 3) return fail(LBB_EINVAL, "nz must be >= 3");
    lbb_params p = *pin;
    const int64_t n64 = (int64_t)p.nx * p.ny * nz;
    const size_t esz = p.precision == LBB_FP64 ? 8 : 4;
    // nodes are indexed with 32-bit integers and planes with 32-bit offsets
    if (n64 * (int64_t)esz >= ((int64_t)1 << 32) || n64 * 8 >= ((int64_t)1 << 32) || 19 * n64 >= ((int64_t)1 << 32))
        return fail(LBB_EINVAL, "nx*ny*nz too large: 19 nx ny nz and nx ny nz * 8 bytes must stay below 2^32");
    double Tc = 0, kap = 0;
    lbb_eos_constants(p.a, p.b, p.R, p.omega, &Tc, &kap);
    const double Ts = p.Ts_over_Tc * Tc;
    if (p.rho_L == 0.0 && p.rho_V == 0.0) {
        rc = lbb_coexistence(p.a, p.b, p.R, p.omega, Ts, &p.rho_V, &p.rho_L);
        if (rc) return fail(LBB_EINVAL, "rho_L = rho_V = 0 needs T_s < T_c for the Maxwell densities");
    }
    if (p.rho_L == p.rho_V) return fail(LBB_EINVAL, "rho_L must differ from rho_V");
    const size_t n = (size_t)n64;
    std::vector<double> rho_host;
    if (!rho0) {
        rho_host.resize(n);
        for (size_t c = 0; c < n; ++c) {
            const int y = (int)((c / (size_t)p.nx) % (size_t)p.ny);
            const double u = (double)(splitmix64_at(p.seed, c) >> 11) * (1.0 / 9007199254740992.0);
            rho_host[c] = (y < p.liquid_rows ? p.rho_L : p.rho_V) + p.noise_amp * (2.0 * u - 1.0);
        }
        rho0 = rho_host.data();
    }
    for (size_t c = 0; c < n; ++c)
        if (!finite_pos(rho0[c]) || p.b * rho0[c] >= 1.0) return fail(LBB_EINVAL, "initial density must satisfy 0 < rho < 1/b");
    std::vector<double> Tb((size_t)p.nx * nz, Ts);
    if (T_bottom)
        for (size_t k = 0; k < Tb.size(); ++k) {
            if (!finite_pos(T_bottom[k])) return fail(LBB_EINVAL, "T_bottom must be finite and > 0");
            Tb[k] = T_bottom[k];
        }
    const int nb = (int)((n + lbb3::NT3 - 1) / lbb3::NT3);
    const int64_t planned = (int64_t)(n * esz * (2 * 19 + 2 + 4 + 5 + 3)) + (int64_t)n * 8 +
                            (int64_t)2 * nb * 8 + (int64_t)Tb.size() * 8 + 4096;
    rc = reserve_bytes(planned, "3-D domain");
    if (rc) return rc;
    int dev = 0;
    LBB_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    LBB_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        release_bytes(planned);
        return fail(LBB_EDEVICE, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
    }
    lbb3_domain *d = new (std::nothrow) lbb3_domain();
    if (!d) {
        release_bytes(planned);
        return fail(LBB_ENOMEM, "host allocation failed");
    }
    d->held = planned;
    d->p = p;
    d->esz = esz;
    make_dev_params(p, Tc, kap, d->dp);
    d->g = lbb3::Geom3{p.nx, p.ny, nz, (unsigned)n};
    d->nb = nb;
    d->ncu = std::max(1, prop.multiProcessorCount);
    bool ok = hipStreamCreateWithFlags(&d->stream, hipStreamNonBlocking) == hipSuccess;
    auto alloc = [&](void **ptr, size_t bytes) -> bool {
        if (!ok || hipMalloc(ptr, bytes) != hipSuccess) return false;
        d->allocs.push_back(*ptr);
        return hipMemset(*ptr, 0, bytes) == hipSuccess;
    };
    ok = ok && alloc(&d->f[0], 19 * n * esz) && alloc(&d->f[1], 19 * n * esz);
    ok = ok && alloc(&d->T[0], n * esz) && alloc(&d->T[1], n * esz);
    ok = ok && alloc(&d->rho, n * esz) && alloc(&d->v, 3 * n * esz) && alloc(&d->coef, 5 * n * esz);
    ok = ok && alloc(&d->Ts, 2 * n * esz) && alloc(&d->acc, n * esz);
    ok = ok && alloc((void **)&d->psi, n * sizeof(double));
    ok = ok && alloc((void **)&d->mpart, (size_t)nb * sizeof(double)) && alloc((void **)&d->hpart, (size_t)nb * sizeof(double));
    ok = ok && alloc((void **)&d->Tb_dev, Tb.size() * sizeof(double));
    ok = ok && alloc((void **)&d->sc, sizeof(lbb3::Scalars3));
    if (!ok) {
        (void)hipGetLastError();
        release3(d);
        return fail(LBB_ENOMEM, "device allocation failed");
    }
    if (hipMemcpy(d->Tb_dev, Tb.data(), Tb.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        release3(d);
        return fail(LBB_EDEVICE, "upload of T_bottom failed");
    }
    rc = p.precision == LBB_FP64 ? set_state3<double>(d, rho0, nullptr, nullptr)
                                 : set_state3<float>(d, rho0, nullptr, nullptr);
    if (rc) {
        const std::string m = g_err;
        release3(d);
        return fail(rc, m);
    }
    *out = d;
    return LBB_OK;
}

int lbb3_set_fields(lbb3_domain *d, const double *rho, const double *u, const double *T)
{
    if (!d || !rho) return fail(LBB_EINVAL, "domain and rho are required");
    for (size_t c = 0; c < d->g.n; ++c)
        if (!finite_pos(rho[c]) || d->p.b * rho[c] >= 1.0) return fail(LBB_EINVAL, "density must satisfy 0 < rho < 1/b");
    for (int k = 0; k < 2; ++k)
        for (auto &g : d->graph[k])
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    const int rc = d->p.precision == LBB_FP64 ? set_state3<double>(d, rho, u, T) : set_state3<float>(d, rho, u, T);
    d->poisoned = rc != LBB_OK;
    return rc;
}

int lbb3_step_async(lbb3_domain *d, int64_t n)
{
    if (!d || n < 0) return fail(LBB_EINVAL, "domain is NULL or n < 0");
    if (d->poisoned) return fail(LBB_ESTATE, "domain holds an invalid state (reload or set the fields)");
    return enqueue_steps3(d, n);
}

int lbb3_sync(lbb3_domain *d)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    return check_errors3(d);
}

int lbb3_step(lbb3_domain *d, int64_t n)
{
    const int rc = lbb3_step_async(d, n);
    return rc ? rc : lbb3_sync(d);
}

void *lbb3_stream(lbb3_domain *d) { return d ? (void *)d->stream : nullptr; }

int lbb3_read_fields(lbb3_domain *d, double *rho, double *u, double *T, double *f)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    const size_t n = d->g.n;
    double *buf = nullptr;
    LBB_HIP(hipMalloc(&buf, 24 * n * sizeof(double)));
    double *drho = buf, *du = buf + n, *dT = buf + 4 * n, *df = buf + 5 * n;
    if (d->p.precision == LBB_FP64)
        hipLaunchKernelGGL(lbb3::k3_read<double>, dim3(d->nb), dim3(lbb3::NT3), 0, d->stream, d->dp, d->g,
                           static_cast<const double *>(d->f[d->cf]), static_cast<const double *>(d->T[d->cT]),
                           d->psi, d->sc, drho, du, dT, df, (double *)nullptr);
    else
        hipLaunchKernelGGL(lbb3::k3_read<float>, dim3(d->nb), dim3(lbb3::NT3), 0, d->stream, d->dp, d->g,
                           static_cast<const float *>(d->f[d->cf]), static_cast<const float *>(d->T[d->cT]),
                           d->psi, d->sc, drho, du, dT, df, (double *)nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, drho, n * sizeof(double), hipMemcpyDeviceToHost, d->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u, du, 3 * n * sizeof(double), hipMemcpyDeviceToHost, d->stream);
    if (e == hipSuccess && T) e = hipMemcpyAsync(T, dT, n * sizeof(double), hipMemcpyDeviceToHost, d->stream);
    if (e == hipSuccess && f) e = hipMemcpyAsync(f, df, 19 * n * sizeof(double), hipMemcpyDeviceToHost, d->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(LBB_EDEVICE, std::string("read-back: ") + hipGetErrorString(e));
    return LBB_OK;
}

int lbb3_wall_heat_flux(lbb3_domain *d, double *q_now, double *q_mean, double *q_local, int64_t *n_samples)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    lbb3::Scalars3 s;
    LBB_HIP(hipMemcpyAsync(&s, d->sc, sizeof s, hipMemcpyDeviceToHost, d->stream));
    if (q_local) {
        const size_t m = (size_t)d->g.nx * d->g.nz;
        double *buf = nullptr;
        LBB_HIP(hipMalloc(&buf, m * sizeof(double)));
        hipError_t e = hipMemsetAsync(buf, 0, m * sizeof(double), d->stream);
        if (e == hipSuccess) {
            if (d->p.precision == LBB_FP64)
                hipLaunchKernelGGL(lbb3::k3_read<double>, dim3(d->nb), dim3(lbb3::NT3), 0, d->stream, d->dp, d->g,
                                   static_cast<const double *>(d->f[d->cf]), static_cast<const double *>(d->T[d->cT]),
                                   d->psi, d->sc, nullptr, nullptr, nullptr, nullptr, buf);
            else
                hipLaunchKernelGGL(lbb3::k3_read<float>, dim3(d->nb), dim3(lbb3::NT3), 0, d->stream, d->dp, d->g,
                                   static_cast<const float *>(d->f[d->cf]), static_cast<const float *>(d->T[d->cT]),
                                   d->psi, d->sc, nullptr, nullptr, nullptr, nullptr, buf);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(q_local, buf, m * sizeof(double), hipMemcpyDeviceToHost, d->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
        (void)hipFree(buf);
        if (e != hipSuccess) return fail(LBB_EDEVICE, std::string("heat flux read-back: ") + hipGetErrorString(e));
    }
    LBB_HIP(hipStreamSynchronize(d->stream));
    if (q_now) *q_now = s.q_now;
    if (q_mean) *q_mean = s.n_samples > 0 ? s.q_sum / (double)s.n_samples : std::nan("");
    if (n_samples) *n_samples = s.n_samples;
    return LBB_OK;
}

int lbb3_reset_average(lbb3_domain *d)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    lbb3::Scalars3 s;
    LBB_HIP(hipMemcpyAsync(&s, d->sc, sizeof s, hipMemcpyDeviceToHost, d->stream));
    LBB_HIP(hipStreamSynchronize(d->stream));
    s.q_sum = 0.0;
    s.n_samples = 0;
    LBB_HIP(hipMemcpyAsync(d->sc, &s, sizeof s, hipMemcpyHostToDevice, d->stream));
    LBB_HIP(hipStreamSynchronize(d->stream));
    return LBB_OK;
}

int lbb3_set_heater(lbb3_domain *d, const double *T_bottom)
{
    if (!d || !T_bottom) return fail(LBB_EINVAL, "domain and T_bottom are required");
    const size_t m = (size_t)d->g.nx * d->g.nz;
    for (size_t k = 0; k < m; ++k)
        if (!finite_pos(T_bottom[k])) return fail(LBB_EINVAL, "T_bottom must be finite and > 0");
    LBB_HIP(hipMemcpyAsync(d->Tb_dev, T_bottom, m * sizeof(double), hipMemcpyHostToDevice, d->stream));
    const int nbk = (int)((m + lbb3::NT3 - 1) / lbb3::NT3);
    if (d->p.precision == LBB_FP64)
        hipLaunchKernelGGL(lbb3::k3_set_heater<double>, dim3(nbk), dim3(lbb3::NT3), 0, d->stream, d->dp, d->g,
                           d->Tb_dev, static_cast<double *>(d->T[0]), static_cast<double *>(d->T[1]));
    else
        hipLaunchKernelGGL(lbb3::k3_set_heater<float>, dim3(nbk), dim3(lbb3::NT3), 0, d->stream, d->dp, d->g,
                           d->Tb_dev, static_cast<float *>(d->T[0]), static_cast<float *>(d->T[1]));
    LBB_HIP(hipGetLastError());
    // the heat flux of the current state changes with T_b
    enqueue_reductions3_any(d, 0);
    LBB_HIP(hipStreamSynchronize(d->stream));
    return LBB_OK;
}

int lbb3_info(lbb3_domain *d, int64_t *t, int64_t *device_bytes)
{
    if (!d) return fail(LBB_EINVAL, "domain is NULL");
    lbb3::Scalars3 s;
    LBB_HIP(hipMemcpyAsync(&s, d->sc, sizeof s, hipMemcpyDeviceToHost, d->stream));
    LBB_HIP(hipStreamSynchronize(d->stream));
    if (t) *t = s.t;
    if (device_bytes) *device_bytes = d->held;
    return LBB_OK;
}

int lbb3_destroy(lbb3_domain *d)
{
    if (!d) return LBB_OK;
    (void)hipStreamSynchronize(d->stream);
    release3(d);
    return LBB_OK;
}

}  // extern "C"
