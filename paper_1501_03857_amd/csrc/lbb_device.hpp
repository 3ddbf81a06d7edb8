// Device code of the lbboil library: the two kernels of one time step of the
// hybrid thermal pseudopotential LB boiling model (arXiv:1501.03857, Sec. 2)
// plus the small kernels used at set-up and read-back.  gfx950, wave64.
//
// Data layout in HBM (structure of arrays, x fastest, row pitch nx):
//   f[2][9][ny][nx]  post-streaming distributions, double-buffered.  Wall-row
//                    populations that would arrive from outside the lattice
//                    are never written; every reader completes them with the
//                    Zou-He rule from the populations of the same node.
//   T[2][ny][nx]     temperature stored as T - T_ref (T_ref = 0 in FP64,
//                    T_s in FP32 for precision), double-buffered; the wall
//                    rows hold the Dirichlet values in both buffers.
//   rho, vx, vy      density and the velocity the temperature equation sees,
//                    written by the LB kernel for the thermal kernel.
//   partials         per-block FP64 partial sums of mass and heat flux.
//
// One step t -> t+1 is two launches:
//   k_lb      : per tile (62 x 12 by default, halo 1): rho and psi (FP64 EOS, Eq. (21)) of
//               the tile and its halo into LDS; per interior node the forces
//               (Eqs. (7), (9), (22)), velocity (Eq. (6)), MRT collision with
//               the improved forcing (Eqs. (2), (4), (5), (8)) and push
//               streaming (Eq. (3)) into the other buffer; FP64 mass partials
//               of the streamed state (exact identity, so the next step's
//               rho_ave needs no extra pass).  One extra block, first in the
//               grid, reduces the heat-flux partials of the previous thermal launch.
//   k_thermal: per tile (56 x 24 by default, halo 4): RK4 (Eqs. (19)-(20)) of Eq. (18) in
//               LDS with the region shrinking by one node per stage; FP64
//               heat-flux partials of the new state on the bottom tile row.
//               One extra block, first in the grid, reduces the mass
//               partials of k_lb into rho_ave for the next step.
// All reductions run in a fixed order, so results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbb {

constexpr int NT = 256;   // threads per block of the small kernels (4 waves)
constexpr int TXR = 64;   // read-back tile
constexpr int TYR = 8;
constexpr int TXA = 62;   // LB tile width: tile + halo of one is one wave wide
constexpr int HB = 4;     // thermal halo (RK4 has four stencil stages)
constexpr int TXB = 64 - 2 * HB;  // thermal tile width: tile + halo is one wave wide

// Tile shapes the launches can take (height, waves per block); the host picks
// one of each per lattice or batch, by default or by timing them on the
// lattice (autotune).  Index 0 is the default.  With one lattice row per
// wave the LB kernel needs 72 VGPRs (7 waves per SIMD), against 118 with
// three rows per wave, and the extra waves in flight hide the load latency
// of phase 1 behind the arithmetic of other waves.
struct TileShape {
    int ty, nw;
};
constexpr int NSHAPE_A = 4, NSHAPE_B = 4;
constexpr TileShape kShapeA[NSHAPE_A] = {{4, 4}, {8, 8}, {12, 4}, {4, 2}};
constexpr TileShape kShapeB[NSHAPE_B] = {{24, 16}, {40, 16}, {16, 16}, {8, 8}};

// 1/x from the hardware reciprocal estimate (relative error near 2^-23)
// refined by two Newton-Raphson steps, r <- r + r (1 - x r), each of which
// squares the error: within a few ulp for finite nonzero normal x.  Cheaper
// than the correctly rounded division sequence; the FP64 tolerances allow it.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// 1/sqrt(x) from the hardware estimate refined by two Newton-Raphson steps,
// y <- y + y (1/2 - x y^2 / 2): within a few ulp for normal x > 0.
__device__ __forceinline__ double rsq_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
    e = fma(-h * y, y, 0.5);
    return fma(y, e, y);
}

// sqrt(x) from the hardware reciprocal square root y ~ 1/sqrt(x):
// Goldschmidt's coupled iteration on g ~ sqrt(x), h ~ 1/(2 sqrt(x))
// (r = 1/2 - g h; g <- g + g r; h <- h + h r), twice, then one Newton
// correction g <- g + h (x - g^2).  Within a few ulp for normal x > 0;
// 0 for x = 0, NaN below.
__device__ __forceinline__ double sqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    g = fma(d, h, g);
    return x > 0.0 ? g : (x == 0.0 ? 0.0 : __builtin_nan(""));
}

// sqrt(x) as sqrt_nr for normal x > 0 only (no zero or negative handling):
// for arguments that are positive by construction or checked around it.
__device__ __forceinline__ double sqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}

// Type of the RK4 stage arithmetic: FP64 storage keeps FP64; FP32 storage
// runs the stages in FP32 on T - T_s (rounding ~4e-10 absolute) with the EOS
// coefficients formed in FP64.
template <typename S> struct ThermalCfg;
// sqrt of the stage arithmetic: the refined estimate (a few ulp) in FP64,
// the hardware instruction (1 ulp) in FP32
__device__ __forceinline__ double stage_sqrt(double x) { return sqrt_nr(x); }
__device__ __forceinline__ float stage_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// DPP move of a double (two 32-bit moves) with control `ctl`; lanes the
// pattern gives no source, or whose row `rmask` leaves out, read 0.
template <int CTL, int RMASK>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTL, RMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTL, RMASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum of one double per lane over the wave, valid in lane 63, in a fixed
// order: an inclusive scan inside each row of 16 lanes (shifts by 1, 2, 4,
// 8), then the total of row 0 added into row 1 and of row 2 into row 3, then
// the total of rows 0-1 into rows 2-3.  Every lane must be active.
__device__ __forceinline__ double wave_sum_to_last(double v)
{
    v += dpp_d<0x111 /* row_shr:1 */, 0xf>(v);
    v += dpp_d<0x112 /* row_shr:2 */, 0xf>(v);
    v += dpp_d<0x114 /* row_shr:4 */, 0xf>(v);
    v += dpp_d<0x118 /* row_shr:8 */, 0xf>(v);
    v += dpp_d<0x142 /* row_bcast:15 */, 0xa>(v);
    v += dpp_d<0x143 /* row_bcast:31 */, 0xc>(v);
    return v;
}

// The value a lane's left (lane - 1) or right (lane + 1) neighbour holds,
// through the wave-wide row shift of DPP (0 in the first and last lane).
// Every lane of the wave must be active.
__device__ __forceinline__ float lane_from_left(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138 /* wave_shr:1 */, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_from_right(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130 /* wave_shl:1 */, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_from_left(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_from_right(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

template <> struct ThermalCfg<float> {
    using C = float;
};
template <> struct ThermalCfg<double> {
    using C = double;
};

enum : int { MODE_COUPLED = 0, MODE_ISOTHERMAL = 1, MODE_THERMAL_ONLY = 2 };
enum : int { ERR_RHO = 1, ERR_PSI = 2, ERR_T = 4 };

struct DevParams {
    int nx, ny;
    int periodic_y, mode;
    int ghost, pad_;             // ghost: F_m on the wall rows through a ghost layer
    double a, b, R, Tc, kappa;
    double Ts, T_ref;            // saturation temperature, storage offset of T
    double G, sigma;
    double s_rho, s_e, s_zeta, s_j, s_q;
    double tau_V, tau_slope;     // tau_nu(rho) = tau_V + (rho - rho_V) tau_slope
    double rho_V;
    double cv, chi, cv_chi;
    double g, Gw_bottom, Gw_top;
    double sig_e, sig_z;         // sigma/(tau_e - 1/2), sigma/(tau_zeta - 1/2)
    double inv_Tc, two_over_G;
    // uniform factors of the thermal step, formed on the host (the GPU has no
    // scalar FP64 unit, so each wave would otherwise divide in its vector ALU)
    double R_cv, a_cv, inv_cv;    // R / c_v, a / c_v, 1 / c_v
    double k1k, k2_Tc;            // kappa (1 + kappa), kappa^2 / T_c
    double k1k_rsTc;              // kappa (1 + kappa) / sqrt(T_c)
    double R_cv12, a_cv12;        // R / (12 c_v), a / (12 c_v)
};

// Device-resident scalars of one domain.  tA is the state index seen by the
// LB launch, tB the one seen by the thermal launch; each is written only by
// the other launch's reduction block, so no launch reads a counter it writes.
struct Scalars {
    double rho_ave;
    double q_now;
    double q_sum;
    long long n_samples;
    long long last_counted;      // state index of the last heat-flux sample
    long long tA;
    long long tB;
    unsigned long long err_step; // first failing step, ~0 if none
    unsigned int err_code;
    unsigned int pad;
};

// One lattice of a launch: its parameters, buffers and place in the grid.
// The LB and thermal launches cover any number of lattices of any sizes; a
// block finds its lattice through a block -> lattice table.
struct Inst {
    DevParams P;
    void *f[2], *T[2];
    void *rho, *vx, *vy;
    double *mass_part, *hf_part;
    Scalars *sc;
    int nbxA, nbyA, nbxB, nbyB;
    int blkA0, blkB0;  // first block of this lattice in the LB / thermal grids
};

// Tile of a lattice's q-th block (0 <= q < nb).  Workgroups are dispatched
// to the 8 XCDs round-robin, so blocks q, q+8, q+16, ... share an XCD and its
// L2; they get one contiguous run of tiles (row-major), so halo rows and the
// cache lines straddling tile edges are fetched once per XCD instead of once
// per tile.  With nb = 8m + r the XCD class x = q mod 8 owns m (+1 if x < r)
// tiles starting at x m + min(x, r).
__device__ __forceinline__ int xcd_tile(int q, int nb)
{
    const int x = q & 7, k = q >> 3, m = nb >> 3, r = nb & 7;
    return x * m + (x < r ? x : r) + k;
}

__device__ __forceinline__ int wrapi(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

// Plane-wise global memory access.  A field plane's base address is uniform
// (scalar registers) and the lane adds a 32-bit byte offset, so each access
// is one global load or store with no per-lane 64-bit address arithmetic.
// The host keeps every plane below 4 GiB (nx ny sizeof(S) < 2^32), and the
// cast to the global address space is free: lattice arrays are device
// allocations.
template <typename T>
using gmem = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ T ld_at(const T *plane, unsigned byte_off)
{
    return *(const gmem<T> *)((const gmem<char> *)plane + byte_off);
}

template <typename T>
__device__ __forceinline__ void st_at(T *plane, unsigned byte_off, T v)
{
    *(gmem<T> *)((gmem<char> *)plane + byte_off) = v;
}

// Zou-He completion of a wall node with zero wall velocity (Sec. 3.1): the
// three populations arriving from outside follow from the known ones.
__device__ __forceinline__ void zou_he(double f[9], int bottom)
{
    const double d13 = f[1] - f[3];
    if (bottom) {
        f[2] = f[4];
        f[5] = f[7] - 0.5 * d13;
        f[6] = f[8] + 0.5 * d13;
    } else {
        f[4] = f[2];
        f[7] = f[5] + 0.5 * d13;
        f[8] = f[6] - 0.5 * d13;
    }
}

// Load the 9 populations of node c, completing wall nodes when the state
// came from streaming (every mode but THERMAL_ONLY, where f is frozen).
template <typename Ptr>
__device__ __forceinline__ void load_node(const DevParams &P, Ptr f, size_t N, size_t c, int gy, double fl[9])
{
#pragma unroll
    for (int a = 0; a < 9; ++a) fl[a] = (double)f[(size_t)a * N + c];
    if (!P.periodic_y && P.mode != MODE_THERMAL_ONLY) {
        if (gy == 0) zou_he(fl, 1);
        else if (gy == P.ny - 1) zou_he(fl, 0);
    }
}

// Widen the 9 stored populations of a node to FP64 and complete a wall node.
template <typename S>
__device__ __forceinline__ void complete_node(const DevParams &P, const S fs[9], int gy, double fl[9])
{
#pragma unroll
    for (int a = 0; a < 9; ++a) fl[a] = (double)fs[a];
    if (!P.periodic_y && P.mode != MODE_THERMAL_ONLY) {
        if (gy == 0) zou_he(fl, 1);
        else if (gy == P.ny - 1) zou_he(fl, 0);
    }
}

// psi = sqrt(2 (p_EOS - rho/3) / G) with the Peng-Robinson p_EOS (Eq. (21)),
// always in FP64.  Returns a negative value on a negative radicand.
// The two fractions of p_EOS share one reciprocal:
//   p = [rho R T D2 - a phi rho^2 D1] / (D1 D2), D1 = 1 - b rho,
//   D2 = 1 + 2 b rho - b^2 rho^2.
__device__ __forceinline__ double pseudopotential(const DevParams &P, double rho, double T)
{
    // T > 0 on every node (the temperature step flags any other value), so
    // the root of T/T_c needs no zero or sign handling
    const double s = 1.0 + P.kappa * (1.0 - sqrt_pos(T * P.inv_Tc));
    const double phi = s * s;
    const double D1 = 1.0 - P.b * rho;
    const double D2 = 1.0 + 2.0 * P.b * rho - P.b * P.b * rho * rho;
    const double p = (rho * P.R * T * D2 - P.a * phi * rho * rho * D1) * rcp_nr(D1 * D2);
    const double r = P.two_over_G * (p - rho * (1.0 / 3.0));
    return r > 0.0 ? sqrt_pos(r) : (r == 0.0 ? 0.0 : -1.0);
}

__device__ __forceinline__ void flag_error(Scalars *sc, long long t, unsigned code)
{
    atomicMin(&sc->err_step, (unsigned long long)t);
    atomicOr(&sc->err_code, code);
}

// Wave64 + block sum of one double per thread (NTH threads), result valid in
// thread 0.  Fixed tree, so the result is reproducible.
template <int NTH = NT>
__device__ __forceinline__ double block_sum(double v, double *red /* [NTH/64] */)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NTH / 64; ++k) s += red[k];
    return s;
}

// Fixed-order sum of n doubles by one block; result valid in thread 0.
template <int NTH = NT>
__device__ __forceinline__ double block_sum_array(const double *__restrict__ a, int n, double *red)
{
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += NTH) s += a[k];
    return block_sum<NTH>(s, red);
}

// Fixed-order sum of n doubles by the first 256 threads of a block of at
// least 256 threads (the others add nothing), the same for any block size;
// result valid in thread 0.  All threads of the block must call it.
// s + a[k0] + a[k0 + stride] + ... (k < n), added in that order; the loads are
// issued 16 at a time so a long sum waits for memory once per 16 terms.
__device__ __forceinline__ double ordered_sum(const double *__restrict__ a_, int k0, int n, int stride, double s)
{
    const gmem<double> *__restrict__ a = (const gmem<double> *)a_;
    int k = k0;
    for (; k + 15 * stride < n; k += 16 * stride) {
        double v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = a[k + j * stride];
#pragma unroll
        for (int j = 0; j < 16; ++j) s += v[j];
    }
    for (; k < n; k += stride) s += a[k];
    return s;
}

__device__ __forceinline__ double fixed_sum(const double *__restrict__ a, int n, double *red /* [>= 4] */)
{
    double s = 0.0;
    if (threadIdx.x < NT) s = ordered_sum(a, threadIdx.x, n, NT, 0.0);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0 && w < NT / 64) red[w] = s;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k) t += red[k];
    return t;
}

// Heat-flux bookkeeping: q of state t from the partial sums over x; counted
// once per state index (t > last_counted), never for the initial state.
__device__ __forceinline__ void reduce_heat_flux(const double *__restrict__ hf_part, int n_hf, int nx,
                                                 Scalars *sc, long long t)
{
    if (threadIdx.x == 0) {
        const double s = ordered_sum(hf_part, 0, n_hf, 1, 0.0);
        const double q = s / (double)nx;
        sc->q_now = q;
        if (t > sc->last_counted) {
            sc->q_sum += q;
            sc->n_samples += 1;
            sc->last_counted = t;
        }
    }
}

// ---------------------------------------------------------------------------
// Velocity-independent pieces shared by the LB step and the read-back.
// Total force on an interior node (Eq. (7) + Eq. (22) + Eq. (9)) and
// Q = |F_m|^2 / psi^2 (Eq. (8)), from the LDS psi tile with a halo of one.
// Wall rows carry no force (F = 0, Q = 0): the paper does not apply F_m
// there (Sec. 3.2), and any body force on a Zou-He node would become a mass
// flux through the wall.  The fluid-solid force acts on the rows next to the
// walls, with the wall rows as the solid of Eq. (22).  In the ghost-layer
// variant (P.ghost) the wall rows do get F_m and Q, with the neighbours
// beyond the wall read from a ghost fluid layer that mirrors the first fluid
// row about the wall row (so F_m has no normal part there); buoyancy still
// skips them.
template <int W>
__device__ __forceinline__ void node_force(const DevParams &P, const double *psi_s, int lx, int ly, int gy,
                                           double rho, double rho_ave, double &Fx, double &Fy, double &Q)
{
    Fx = Fy = Q = 0.0;
    const bool bot = !P.periodic_y && gy == 0, top = !P.periodic_y && gy == P.ny - 1;
    if ((bot || top) && !P.ghost) return;
    const int c = (ly + 1) * W + (lx + 1);
    const double pc = psi_s[c];
    const double pE = psi_s[c + 1], pW = psi_s[c - 1];
    // the LDS row beyond a wall holds no lattice node; the ghost layer
    // replaces it by the mirror image of the row on the other side
    const int cn = top ? c - W : c + W, cs = bot ? c + W : c - W;
    const double pN = psi_s[cn], pS = psi_s[cs];
    const double pNE = psi_s[cn + 1], pNW = psi_s[cn - 1], pSW = psi_s[cs - 1], pSE = psi_s[cs + 1];
    // sum_a w_a psi(x + e_a) e_a with w = 1/3 (axes), 1/12 (diagonals)
    const double sx = (pE - pW) * (1.0 / 3.0) + (pNE - pNW - pSW + pSE) * (1.0 / 12.0);
    const double sy = (pN - pS) * (1.0 / 3.0) + (pNE + pNW - pSW - pSE) * (1.0 / 12.0);
    Fx = -P.G * pc * sx;
    Fy = -P.G * pc * sy;
    Q = P.G * P.G * (sx * sx + sy * sy);
    if (bot || top) return;
    // fluid-solid force on the rows next to the walls (wall rows are the solid)
    if (!P.periodic_y) {
        if (gy == 1) Fy += P.Gw_bottom * pc * pc * (1.0 / 6.0);
        if (gy == P.ny - 2) Fy -= P.Gw_top * pc * pc * (1.0 / 6.0);
    }
    // buoyancy, Eq. (9)
    Fy -= (rho - rho_ave) * P.g;
}

// MRT collision of one node (Eqs. (2), (4), (5), (8)) in moment space with
// the D2Q9 basis (rho, e, zeta, jx, qx, jy, qy, pxx, pxy); returns f*.
// s_nu = 1/tau_nu(rho) comes from the caller, which forms it with 1/rho from
// one reciprocal.
__device__ __forceinline__ void collide(const DevParams &P, double f[9], double rho, double vx, double vy,
                                        double Fx, double Fy, double Q, double s_nu)
{
    // moments m = M f, from sums and differences shared between the rows of M
    const double d13 = f[1] - f[3], d24 = f[2] - f[4];
    const double d57 = f[5] - f[7], d68 = f[6] - f[8];
    const double s13 = f[1] + f[3], s24 = f[2] + f[4];
    const double s57 = f[5] + f[7], s68 = f[6] + f[8];
    const double s14 = s13 + s24, s58 = s57 + s68;
    const double m_e = -(4) * f[0] - s14 + (2) * s58;
    const double m_z = (4) * f[0] - (2) * s14 + s58;
    const double dx58 = d57 - d68, dy58 = d57 + d68;  // sum over the diagonals of e_x f, e_y f
    const double jx = d13 + dx58;
    const double qx = -(2) * d13 + dx58;
    const double jy = d24 + dy58;
    const double qy = -(2) * d24 + dy58;
    const double pxx = s13 - s24;
    const double pxy = s57 - s68;

    const double v2 = vx * vx + vy * vy;
    const double vF = vx * Fx + vy * Fy;
    const double s_e = (P.s_e), s_z = (P.s_zeta), s_j = (P.s_j), s_q = (P.s_q);

    // m* = m - L (m - m_eq) + (I - L/2) S
    const double e_s = m_e - s_e * (m_e - rho * ((-2) + (3) * v2)) + ((1) - (0.5) * s_e) * ((6) * vF + (P.sig_e) * Q);
    const double z_s = m_z - s_z * (m_z - rho * ((1) - (3) * v2)) + ((1) - (0.5) * s_z) * (-(6) * vF - (P.sig_z) * Q);
    const double jx_s = jx - s_j * (jx - rho * vx) + ((1) - (0.5) * s_j) * Fx;
    const double qx_s = qx - s_q * (qx + rho * vx) - ((1) - (0.5) * s_q) * Fx;
    const double jy_s = jy - s_j * (jy - rho * vy) + ((1) - (0.5) * s_j) * Fy;
    const double qy_s = qy - s_q * (qy + rho * vy) - ((1) - (0.5) * s_q) * Fy;
    const double pxx_s = pxx - s_nu * (pxx - rho * (vx * vx - vy * vy)) + ((1) - (0.5) * s_nu) * (2) * (vx * Fx - vy * Fy);
    const double pxy_s = pxy - s_nu * (pxy - rho * vx * vy) + ((1) - (0.5) * s_nu) * (vx * Fy + vy * Fx);
    // rho* = rho (s_rho drops out: m_eq,rho = rho and S_rho = 0)

    // f* = M^{-1} m* with M^{-1} = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
    // rho/9 rounded once: 1/9 as its nearest double plus the remainder.
    // rho * fl(1/9) alone is biased (fl(1/9) < 1/9), and the nine outputs
    // sum to 9 r9, so every node would lose a fixed 5.6e-17 rho of mass per
    // step; this product gives the correctly rounded quotient instead.
    const double r9 = fma(rho, 1.0 / 9.0, rho * 0x1.c71c71c71c71cp-58);
    const double e36 = e_s * (1.0 / 36.0), z36 = z_s * (1.0 / 36.0);
    const double jx6 = jx_s * (1.0 / 6.0), jy6 = jy_s * (1.0 / 6.0);
    const double qx12 = qx_s * (1.0 / 12.0), qy12 = qy_s * (1.0 / 12.0);
    const double pxx4 = pxx_s * (0.25), pxy4 = pxy_s * (0.25);
    const double axis = r9 - e36 - (2) * z36;
    const double diag = r9 + (2) * e36 + z36;
    // shared sums of the columns of M^T: axis and diagonal pairs differ only
    // in the signs of these
    const double ax = jx6 - (2) * qx12, ay = jy6 - (2) * qy12;
    const double cx = jx6 + qx12, cy = jy6 + qy12;
    const double ap = axis + pxx4, am = axis - pxx4;
    const double dp = diag + pxy4, dm = diag - pxy4;
    const double cp = cx + cy, cm = cx - cy;
    f[0] = r9 - (4) * e36 + (4) * z36;
    f[1] = ap + ax;
    f[2] = am + ay;
    f[3] = ap - ax;
    f[4] = am - ay;
    f[5] = dp + cp;
    f[6] = dm - cm;
    f[7] = dp - cp;
    f[8] = dm + cm;
}

__constant__ const int kEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ const int kEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Phase 1 shared by the LB step and the read-back: rho and psi of the tile
// and a halo of one into LDS.  Nodes beyond a wall get psi = 0 (never read).
template <typename S, int TX, int TY>
__device__ __forceinline__ void tile_psi(const DevParams &P, const S *__restrict__ fin, const S *__restrict__ Tin,
                                         int x0, int y0, double *psi_s, Scalars *sc, long long t)
{
    constexpr int W = TX + 2, H = TY + 2;
    const size_t N = (size_t)P.nx * P.ny;
    for (int k = threadIdx.x; k < W * H; k += NT) {
        const int lx = k % W - 1, ly = k / W - 1;
        const int gx = wrapi(x0 + lx, P.nx);
        int gy = y0 + ly;
        if (P.periodic_y) gy = wrapi(gy, P.ny);
        else if (gy < 0 || gy >= P.ny) {
            psi_s[k] = 0.0;
            continue;
        }
        const size_t c = (size_t)gy * P.nx + gx;
        double fl[9];
        load_node(P, fin, N, c, gy, fl);
        double rho = 0.0;
        {
            double r = fl[0];
#pragma unroll
            for (int a = 1; a < 9; ++a) r += fl[a];
            rho = r;
        }
        const double T = P.T_ref + (double)Tin[c];
        const double psi = pseudopotential(P, rho, T);
        if (!(rho > 0.0) || !(rho < 1e300)) flag_error(sc, t, ERR_RHO);
        if (!(psi >= 0.0) || !(psi < 1e300)) flag_error(sc, t, ERR_PSI);
        psi_s[k] = psi;
    }
}

// ---------------------------------------------------------------------------
// LB step: forces, collision and push streaming; mass partials.
// Layout: the tile (TXA x TYA) with its halo of one node is 64 columns wide,
// lane = column, and each of the NWA waves owns every NWA-th row.  Phase 1
// issues every population and temperature load of the wave's rows and halo
// row, then forms rho and psi (FP64 EOS) on the tile and halo, keeping each
// node's populations in registers; phase 2 collides the interior nodes and
// pushes.  The parameters are read in place through the lattice table
// (copied, they would not fit the scalar registers beside the plane bases).
template <typename S, int TYA, int NWA>
__global__ __launch_bounds__(64 * NWA, TYA == NWA ? 7 : 1) void k_lb(const Inst *__restrict__ insts, const int *__restrict__ blk2inst,
                                                 int cf, int cT)
{
    const Inst &I = insts[blk2inst[blockIdx.x]];
    const DevParams &P = I.P;
    const bool frozen = P.mode == MODE_THERMAL_ONLY;
    const S *__restrict__ fin = static_cast<const S *>(I.f[cf]);
    S *__restrict__ fout = static_cast<S *>(I.f[cf ^ 1]);
    const S *__restrict__ Tin = static_cast<const S *>(I.T[cT]);
    S *__restrict__ rho_o = static_cast<S *>(I.rho);
    S *__restrict__ vx_o = static_cast<S *>(I.vx);
    S *__restrict__ vy_o = static_cast<S *>(I.vy);
    Scalars *__restrict__ sc = I.sc;
    const int nbx = I.nbxA, nby = I.nbyA;
    const int blk = (int)blockIdx.x - I.blkA0;
    static_assert(TYA % NWA == 0, "LB rows must split evenly over the waves");
    constexpr int IPW_A = TYA / NWA;             // interior rows per wave
    constexpr int H = TYA + 2;                   // region rows (halo rows 0 and H-1)
    __shared__ double psi_s[H * 64];
    const long long t = sc->tA;
    // block 0 of the lattice reduces the previous thermal launch's partials; it
    // needs nothing from this launch, so it runs first, beside the tiles
    if (blk == 0) {
        reduce_heat_flux(I.hf_part, I.nbxB, P.nx, sc, t);
        if (threadIdx.x == 0) sc->tB = t;  // the thermal launch of this step
        return;
    }
    const int tile = xcd_tile(blk - 1, nbx * nby);
    const int bx = tile % nbx, by = tile / nbx;
    const int x0 = bx * TXA, y0 = by * TYA;
    const size_t N = (size_t)P.nx * P.ny;
    const bool walls = !P.periodic_y;
    // the wave index is uniform over the wave: keep row logic on the scalar unit
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gx = wrapi(x0 + lane - 1, P.nx);
    const unsigned gxu = (unsigned)gx;

    // lattice row of region row r (wrapped when periodic); false beyond a wall
    auto row_of = [&](int r, int &gy) -> bool {
        gy = y0 + r - 1;
        if (P.periodic_y) {
            gy = wrapi(gy, P.ny);
            return true;
        }
        return gy >= 0 && gy < P.ny;
    };
    // rho and psi of node (r, lane) into LDS; returns rho
    // Row kind, uniform over the wave (one lattice row per wave): 1 bottom
    // wall, 2 top wall, 0 any other row (or no walls, or f frozen).  Wall
    // rows complete their populations by the Zou-He rule; the code of each
    // kind is generated separately, so other rows carry none of it.
    auto kind_of = [&](int gy) -> int {
        if (!walls || frozen) return 0;
        return gy == 0 ? 1 : (gy == P.ny - 1 ? 2 : 0);
    };
    auto psi_node = [&](int r, int gy, const S fs[9], S Tn) -> double {
        double fl[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) fl[a] = (double)fs[a];
        // rho = sum of the completed populations; on a wall row the three
        // unknowns sum to the three opposite knowns (Zou-He, zero velocity)
        double rr;
        const int kind = kind_of(gy);
        if (kind == 1) rr = fl[0] + fl[1] + fl[3] + 2.0 * (fl[4] + fl[7] + fl[8]);
        else if (kind == 2) rr = fl[0] + fl[1] + fl[3] + 2.0 * (fl[2] + fl[5] + fl[6]);
        else {
            rr = fl[0];
#pragma unroll
            for (int a = 1; a < 9; ++a) rr += fl[a];
        }
        if (!frozen) {
            const double T = P.T_ref + (double)Tn;
            const double psi = pseudopotential(P, rr, T);
            if (!(rr > 0.0) || !(rr < 1e300)) flag_error(sc, t, ERR_RHO);
            if (!(psi >= 0.0) || !(psi < 1e300)) flag_error(sc, t, ERR_PSI);
            psi_s[r * 64 + lane] = psi;
        }
        return rr;
    };

    // phase 1: the wave's interior rows (populations kept in registers) and,
    // for waves 0 and 1, the halo rows 0 and H-1 (psi only).  Every global
    // load of the phase is issued before the first arithmetic, so their
    // latencies overlap.
    S fs[IPW_A][9], Tv[IPW_A];
    double rho[IPW_A];
    int gys[IPW_A];
    bool live[IPW_A], inl[IPW_A];
#pragma unroll
    for (int m = 0; m < IPW_A; ++m) {
        const int r = 1 + wv + NWA * m;
        int gy;
        inl[m] = row_of(r, gy);
        // a ragged last tile row beyond ny is not collided here, but with
        // periodic y it wraps onto a real row whose psi its neighbour needs
        live[m] = inl[m] && y0 + r - 1 < P.ny;
        gys[m] = gy;
        if (!inl[m]) continue;
        const unsigned o = ((unsigned)gy * (unsigned)P.nx + gxu) * (unsigned)sizeof(S);
#pragma unroll
        for (int a = 0; a < 9; ++a) fs[m][a] = ld_at(fin + (size_t)a * N, o);
        Tv[m] = frozen ? S(0) : ld_at(Tin, o);
    }
    const int rh_ = wv == 0 ? 0 : H - 1;
    int gyh = 0;
    const bool halo = wv < 2 && row_of(rh_, gyh);
    S hs[9], Th = S(0);
    if (halo) {
        const unsigned o = ((unsigned)gyh * (unsigned)P.nx + gxu) * (unsigned)sizeof(S);
#pragma unroll
        for (int a = 0; a < 9; ++a) hs[a] = ld_at(fin + (size_t)a * N, o);
        Th = frozen ? S(0) : ld_at(Tin, o);
    }
#pragma unroll
    for (int m = 0; m < IPW_A; ++m) {
        rho[m] = 1.0;
        if (inl[m]) rho[m] = psi_node(1 + wv + NWA * m, gys[m], fs[m], Tv[m]);
    }
    if (halo) (void)psi_node(rh_, gyh, hs, Th);
    __syncthreads();
    const double rho_ave = sc->rho_ave;

    double mrow[IPW_A];
#pragma unroll
    for (int m = 0; m < IPW_A; ++m) {
        const int r = 1 + wv + NWA * m;
        const int gy = gys[m];
        mrow[m] = 0.0;
        if (!live[m] || lane < 1 || lane > TXA || x0 + lane - 1 >= P.nx) continue;
        constexpr unsigned sz = (unsigned)sizeof(S);
        const unsigned rowc = (unsigned)gy * (unsigned)P.nx, oc = (rowc + gxu) * sz;
        double f[9];
        complete_node(P, fs[m], gy, f);
        const double rh = rho[m];
        const double jx = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
        const double jy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
        const bool wall_row = walls && (gy == 0 || gy == P.ny - 1);
        if (frozen) {
            // THERMAL_ONLY: f is frozen, the temperature sees sum e f / rho
            st_at(rho_o, oc, S(rh));
            st_at(vx_o, oc, wall_row ? S(0) : S(jx / rh));
            st_at(vy_o, oc, wall_row ? S(0) : S(jy / rh));
            double mm = 0.0;
#pragma unroll
            for (int a = 0; a < 9; ++a) mm += f[a];
            mrow[m] = mm;
            continue;
        }
        double Fx, Fy, Q;
        node_force<64>(P, psi_s, lane - 1, r - 1, gy, rh, rho_ave, Fx, Fy, Q);
        const double inv_rho = rcp_nr(rh);
        const double vx = (jx + 0.5 * Fx) * inv_rho;
        const double vy = (jy + 0.5 * Fy) * inv_rho;
        st_at(rho_o, oc, S(rh));
        st_at(vx_o, oc, wall_row ? S(0) : S(vx));
        st_at(vy_o, oc, wall_row ? S(0) : S(vy));
        collide(P, f, rh, vx, vy, Fx, Fy, Q, rcp_nr(P.tau_V + (rh - P.rho_V) * P.tau_slope));
        // The mass partial sums the post-collision populations before they
        // are rounded to the storage precision: in FP32 storage it then
        // differs from the stored mass by the rounding of the populations
        // (relative ~1e-7 per node, ~1e-10 over a lattice), far below what
        // rho_ave moves the buoyancy by.
        // push streaming, Eq. (3); populations leaving through a wall are
        // dropped.  Mass of the streamed state: each population counts once,
        // except those that leave through a wall (0) and those that arrive on
        // a wall row, whose Zou-He partners are reconstructed with the same
        // sum (2).
        const int xe = gx + 1 == P.nx ? 0 : gx + 1;
        const int xw = gx == 0 ? P.nx - 1 : gx - 1;
        int yn = gy + 1, ys = gy - 1;
        if (P.periodic_y) {
            if (yn == P.ny) yn = 0;
            if (ys < 0) ys = P.ny - 1;
        }
        const bool has_n = yn < P.ny, has_s = ys >= 0;
        const unsigned rown = (unsigned)yn * (unsigned)P.nx, rows = (unsigned)ys * (unsigned)P.nx;
        const unsigned xeu = (unsigned)xe, xwu = (unsigned)xw;
        st_at(fout + 0 * N, oc, S(f[0]));
        st_at(fout + 1 * N, (rowc + xeu) * sz, S(f[1]));
        st_at(fout + 3 * N, (rowc + xwu) * sz, S(f[3]));
        if (has_n) {
            st_at(fout + 2 * N, (rown + gxu) * sz, S(f[2]));
            st_at(fout + 5 * N, (rown + xeu) * sz, S(f[5]));
            st_at(fout + 6 * N, (rown + xwu) * sz, S(f[6]));
        }
        if (has_s) {
            st_at(fout + 4 * N, (rows + gxu) * sz, S(f[4]));
            st_at(fout + 7 * N, (rows + xwu) * sz, S(f[7]));
            st_at(fout + 8 * N, (rows + xeu) * sz, S(f[8]));
        }
        const double up = f[2] + f[5] + f[6];
        const double dn = f[4] + f[7] + f[8];
        double mm = f[0] + f[1] + f[3];
        const double wu = !walls ? 1.0 : (gy == P.ny - 1 ? 0.0 : (gy == P.ny - 2 ? 2.0 : 1.0));
        const double wd = !walls ? 1.0 : (gy == 0 ? 0.0 : (gy == 1 ? 2.0 : 1.0));
        mm += wu * up + wd * dn;
        mrow[m] = mm;
    }
    // mass partials per lattice row and 62-column chunk, summed over the wave
    // in a fixed order (the same for every tile height)
#pragma unroll
    for (int m = 0; m < IPW_A; ++m) {
        const double v = wave_sum_to_last(mrow[m]);
        if (live[m] && lane == 63) I.mass_part[(size_t)gys[m] * nbx + bx] = v;
    }
}

// ---------------------------------------------------------------------------
// Thermal step: RK4 of Eq. (18) with rho, v frozen; heat-flux partials.
//   K = -(ax d_x T + ay d_y T) + chi lap T + c1 T + c2 sqrt(T)
// with ax = vx - chi d_x rho / rho, ay likewise, and the pressure-work term
// -w T (dp/dT)_rho, w = div v / (rho c_v), written through
// (dp/dT)_rho = A - B phi'(T), A = rho R/(1 - b rho),
// B = a rho^2/(1 + 2 b rho - b^2 rho^2) and
// T phi'(T) = kappa^2 T/T_c - kappa (1 + kappa) sqrt(T/T_c):
//   c1 = w (-A + B kappa^2/T_c),  c2 = -w B kappa (1 + kappa)/sqrt(T_c),
// both formed once per node in FP64 (rho is frozen over the step) and
// rounded once to the stage type; each stage then needs one square root.
// Layout: the tile (TXB x TY) with its halo of HB nodes is 64 columns wide,
// so lane = column and each of the NWB waves owns every NWB-th row of the
// region; stage k is evaluated on the region shrunk by k+1 nodes.  The
// coefficients of K stay in registers (a wave evaluates K only at its own
// rows), the stage inputs alternate between two LDS planes (one barrier per
// stage) and the RK4 sums stay in registers.  The parameters are copied into
// registers once: read through the lattice table they would be fetched again
// after every barrier.
template <typename S, int TY, int NWB>
__global__ __launch_bounds__(64 * NWB) void k_thermal(const Inst *__restrict__ insts,
                                                      const int *__restrict__ blk2inst, int cf, int cT)
{
    const Inst &I = insts[blk2inst[blockIdx.x]];
    const DevParams P = I.P;
    const S *__restrict__ Tin = static_cast<const S *>(I.T[cT]);
    S *__restrict__ Tout = static_cast<S *>(I.T[cT ^ 1]);
    const S *__restrict__ rho_i = static_cast<const S *>(I.rho);
    const S *__restrict__ vx_i = static_cast<const S *>(I.vx);
    const S *__restrict__ vy_i = static_cast<const S *>(I.vy);
    const S *__restrict__ fnew = static_cast<const S *>(I.f[P.mode == MODE_THERMAL_ONLY ? cf : cf ^ 1]);
    Scalars *__restrict__ sc = I.sc;
    const int nbx = I.nbxB, nby = I.nbyB;
    const int blk = (int)blockIdx.x - I.blkB0;
    using C = typename ThermalCfg<S>::C;
    constexpr int H = TY + 2 * HB;               // region rows
    constexpr int RPW = (H + NWB - 1) / NWB;     // region rows per wave
    __shared__ C T0[H][64];
    __shared__ C X[3][H][64];   // rho, vx, vy
    __shared__ C Ts[2][H][64];  // stage values T0 + c h (ping-pong); new T for the heat flux
    __shared__ double red[NWB];
    const long long t = sc->tB;
    if (blk == 0) {  // reduction of the LB launch's mass partials, first in the grid
        const double m = fixed_sum(I.mass_part, I.nbxA * P.ny, red);
        if (threadIdx.x == 0) {
            sc->rho_ave = m / ((double)P.nx * (double)P.ny);
            sc->tA = t + 1;
        }
        return;
    }
    const int tile = xcd_tile(blk - 1, nbx * nby);
    const int bx = tile % nbx, by = tile / nbx;
    const int x0 = bx * TXB, y0 = by * TY;
    const bool walls = !P.periodic_y;
    const bool run = P.mode != MODE_ISOTHERMAL;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gx = wrapi(x0 + lane - HB, P.nx);
    const unsigned gxu = (unsigned)gx;

    // lattice row of region row r; false beyond a wall
    auto row_of = [&](int r, int &gy) -> bool {
        gy = y0 + r - HB;
        if (P.periodic_y) {
            gy = wrapi(gy, P.ny);
            return true;
        }
        return gy >= 0 && gy < P.ny;
    };

#pragma unroll
    for (int m = 0; m < RPW; ++m) {
        const int r = wv + NWB * m;
        int gy;
        if (r >= H || !row_of(r, gy)) continue;
        const unsigned o = ((unsigned)gy * (unsigned)P.nx + gxu) * (unsigned)sizeof(S);
        T0[r][lane] = (C)ld_at(Tin, o);
        if (run) {
            X[0][r][lane] = (C)ld_at(rho_i, o);
            X[1][r][lane] = (C)ld_at(vx_i, o);
            X[2][r][lane] = (C)ld_at(vy_i, o);
        }
    }
    __syncthreads();

    C acc[RPW];
#pragma unroll
    for (int m = 0; m < RPW; ++m) acc[m] = C(0);

    // rows where K acts: in the lattice and not a wall row
    bool act[RPW];
#pragma unroll
    for (int m = 0; m < RPW; ++m) {
        int gy;
        act[m] = row_of(wv + NWB * m, gy) && !(walls && (gy == 0 || gy == P.ny - 1));
    }

    // Per-node coefficients of K on the region shrunk by one node, kept in
    // registers (each wave evaluates K only at its own rows).
    C cfr[4][RPW];
#pragma unroll
    for (int m = 0; m < RPW; ++m) cfr[0][m] = cfr[1][m] = cfr[2][m] = cfr[3][m] = C(0);
    if (run) {
#pragma unroll
        for (int m = 0; m < RPW; ++m) {
            const int r = wv + NWB * m;
            if (r < 1 || r >= H - 1 || !act[m]) continue;
            // column sums of the gradient stencils (see the stages below),
            // every lane for its own column, passed to the neighbours
            const C rc = X[0][r][lane], rN = X[0][r + 1][lane], rS = X[0][r - 1][lane];
            const C uc = X[1][r][lane], uN = X[1][r + 1][lane], uS = X[1][r - 1][lane];
            const C vN = X[2][r + 1][lane], vS = X[2][r - 1][lane];
            const C sr = (rN + rS) + C(4) * rc, dr = rN - rS;
            const C su = (uN + uS) + C(4) * uc, dv = vN - vS;
            const C srW = lane_from_left(sr), srE = lane_from_right(sr);
            const C drW = lane_from_left(dr), drE = lane_from_right(dr);
            const C suW = lane_from_left(su), suE = lane_from_right(su);
            const C dvW = lane_from_left(dv), dvE = lane_from_right(dv);
            if (lane < 1 || lane >= 63) continue;
            const double rho = (double)rc;
            // 12 d_x rho, 12 d_y rho and 12 div v from the column sums
            const C gx = srE - srW, gy = fma(C(4), dr, drW + drE);
            const double div12 = (double)((suE - suW) + fma(C(4), dv, dvW + dvE));
            // A w = (R/c_v) div v / D1 and B w = (a/c_v) rho div v / D2 with
            // D1 = 1 - b rho, D2 = 1 + 2 b rho - b^2 rho^2; one reciprocal
            // 1/(rho D1 D2) gives 1/rho, 1/D1 and 1/D2
            const double D1 = 1.0 - P.b * rho;
            const double D2 = 1.0 + 2.0 * P.b * rho - P.b * P.b * rho * rho;
            const double inv = rcp_nr(rho * D1 * D2);
            // the stages read the column sums unscaled: 12 d_x T and 12 d_y T,
            // so the advection coefficients carry the 1/12
            // (a_x/12 = (chi/rho) d_x rho/12 - v_x/12 = (chi/rho) gx/144 - v_x/12)
            const C k144 = (C)(P.chi * (1.0 / 144.0) * D1 * D2 * inv);
            cfr[0][m] = fma(k144, gx, -uc * C(1.0 / 12.0));
            cfr[1][m] = fma(k144, gy, -X[2][r][lane] * C(1.0 / 12.0));
            const double Aw = P.R_cv12 * div12 * (rho * D2 * inv), Bw = P.a_cv12 * rho * div12 * (rho * D1 * inv);
            cfr[2][m] = (C)(Bw * P.k2_Tc - Aw);
            cfr[3][m] = (C)(-Bw * P.k1k_rsTc);
        }

        const C Tref = (C)P.T_ref;
        const C chi6 = (C)(P.chi * (1.0 / 6.0));
        const C cst[3] = {C(0.5), C(0.5), C(1.0)};
        const C wst[4] = {C(1), C(2), C(2), C(1)};
        // stage st reads T0 (st = 0) or Ts[(st - 1) & 1] and writes Ts[st & 1]:
        // one barrier per stage
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int rad = HB - 1 - st;
            const C(*in)[64] = st == 0 ? T0 : Ts[(st - 1) & 1];
#pragma unroll
            for (int m = 0; m < RPW; ++m) {
                const int r = wv + NWB * m;
                if (r >= H || r < HB - rad || r >= HB + TY + rad) continue;
                // Column sums of the 3x3 stencil, formed by every lane for its
                // own column and passed to the neighbouring columns:
                // v = T_S + 4 T_c + T_N, w = T_N - T_S give
                //   d_x T = (v_E - v_W)/12, d_y T = (w_W + 4 w + w_E)/12,
                //   lap T = (v_W + v_E + 4 v - 36 T_c)/6,
                // the isotropic stencils of the gradient and the Laplacian
                // (the 1/12 and 1/6 are carried by the coefficients).
                const C tc = in[r][lane], tN = in[r + 1][lane], tS = in[r - 1][lane];
                const C v = fma(C(4), tc, tN + tS), w = tN - tS;
                const C vW = lane_from_left(v), vE = lane_from_right(v);
                const C wW = lane_from_left(w), wE = lane_from_right(w);
                if (lane < HB - rad || lane >= HB + TXB + rad) continue;
                C h = C(0);
                if (act[m]) {
                    const C T = Tref + tc;
                    const C lap6 = fma(C(-36), tc, fma(C(4), v, vW + vE));
                    h = cfr[2][m] * T;
                    h = fma(cfr[3][m], stage_sqrt(T), h);
                    h = fma(chi6, lap6, h);
                    h = fma(cfr[0][m], vE - vW, h);
                    h = fma(cfr[1][m], fma(C(4), w, wW + wE), h);
                    acc[m] = st == 0 ? h : fma(wst[st], h, acc[m]);
                }
                if (st < 3) Ts[st & 1][r][lane] = fma(cst[st], h, T0[r][lane]);
            }
            if (st < 3) __syncthreads();
        }
    }

    // new interior temperature (wall rows keep their Dirichlet values), into
    // the stage plane the last stage did not read
    C(*Tn_s)[64] = Ts[1];
#pragma unroll
    for (int m = 0; m < RPW; ++m) {
        const int r = wv + NWB * m;
        if (r < HB || r >= HB + TY || lane < HB || lane >= HB + TXB) continue;
        int gy;
        if (x0 + lane - HB >= P.nx || y0 + r - HB >= P.ny || !row_of(r, gy)) continue;
        C Tn = T0[r][lane];
        if (run && !(walls && (gy == 0 || gy == P.ny - 1))) {
            Tn = (C)(S)(T0[r][lane] + acc[m] * C(1.0 / 6.0));
            const double Tabs = P.T_ref + (double)Tn;
            if (!(Tabs > 0.0) || !(Tabs < 1e300)) flag_error(sc, t, ERR_T);
            st_at(Tout, ((unsigned)gy * (unsigned)P.nx + gxu) * (unsigned)sizeof(S), (S)Tn);
        }
        Tn_s[r][lane] = Tn;
    }
    __syncthreads();

    // heat-flux partials of the new state (bottom tile row only)
    if (walls && by == 0 && wv == 0) {
        double qw = 0.0;
        if (lane >= HB && lane < HB + TXB && x0 + lane - HB < P.nx) {
            const size_t N = (size_t)P.nx * P.ny;
            double fl[9];
            load_node(P, (const gmem<S> *)fnew, N, (size_t)gx, 0, fl);
            double r0 = fl[0];
#pragma unroll
            for (int a = 1; a < 9; ++a) r0 += fl[a];
            const double t0 = (double)T0[HB][lane], t1 = (double)Tn_s[HB + 1][lane], t2 = (double)Tn_s[HB + 2][lane];
            qw = -P.cv_chi * r0 * (-3.0 * t0 + 4.0 * t1 - t2) / 2.0;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) qw += __shfl_xor(qw, off, 64);
        if (lane == 0) I.hf_part[bx] = qw;
    }
}

// ---------------------------------------------------------------------------
// Set-up and read-back kernels.

// f = f_eq(rho, u), T as given (FP64 inputs), wall rows of T at T_b and T_s.
template <typename S>
__global__ void k_set_state(DevParams P, const double *__restrict__ rho, const double *__restrict__ ux,
                            const double *__restrict__ uy, const double *__restrict__ T,
                            const double *__restrict__ Tb, S *__restrict__ f, S *__restrict__ T0,
                            S *__restrict__ T1, Scalars *sc)
{
    const size_t N = (size_t)P.nx * P.ny;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < N; c += (size_t)gridDim.x * blockDim.x) {
        const int gy = (int)(c / P.nx), gx = (int)(c % P.nx);
        const bool wall_row = !P.periodic_y && (gy == 0 || gy == P.ny - 1);
        const double r = rho[c];
        const double u = (ux && !wall_row) ? ux[c] : 0.0, v = (uy && !wall_row) ? uy[c] : 0.0;
        const double u2 = u * u + v * v;
        const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
        for (int a = 0; a < 9; ++a) {
            const double eu = kEX[a] * u + kEY[a] * v;
            f[(size_t)a * N + c] = S(W[a] * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * u2));
        }
        double Tv = T ? T[c] : P.Ts;
        if (!P.periodic_y && gy == 0) Tv = Tb[gx];
        if (!P.periodic_y && gy == P.ny - 1) Tv = P.Ts;
        T0[c] = S(Tv - P.T_ref);
        T1[c] = S(Tv - P.T_ref);
        if (!(r > 0.0) || !(Tv > 0.0) || !(P.b * r < 1.0)) flag_error(sc, 0, ERR_RHO);
    }
}

// Mass partials of the current (post-streaming) state, plain sum of f.
template <typename S>
__global__ __launch_bounds__(NT) void k_mass(DevParams P, const S *__restrict__ f, double *__restrict__ part)
{
    __shared__ double red[NT / 64];
    const size_t N = (size_t)P.nx * P.ny;
    double m = 0.0;
    for (size_t c = blockIdx.x * (size_t)NT + threadIdx.x; c < N; c += (size_t)gridDim.x * NT) {
        double fl[9];
        load_node(P, f, N, c, (int)(c / P.nx), fl);
        double r = fl[0];
#pragma unroll
        for (int a = 1; a < 9; ++a) r += fl[a];
        m += r;
    }
    const double s = block_sum(m, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_reduce_mass(DevParams P, const double *__restrict__ part, int n, Scalars *sc)
{
    __shared__ double red[NT / 64];
    const double m = block_sum_array(part, n, red);
    if (threadIdx.x == 0) sc->rho_ave = m / ((double)P.nx * (double)P.ny);
}

// Heat-flux partials of the current state (set-up, heater change, load),
// with the lane layout of the thermal kernel: 64 threads per tile of TXB
// columns, lane = column + HB.
template <typename S>
__global__ void k_heat_flux_state(DevParams P, const S *__restrict__ f, const S *__restrict__ T,
                                  double *__restrict__ hf_part, double *__restrict__ q_local)
{
    const int lane = threadIdx.x;
    const int gx = blockIdx.x * TXB + lane - HB;
    double qw = 0.0;
    if (!P.periodic_y && lane >= HB && lane < HB + TXB && gx < P.nx) {
        const size_t N = (size_t)P.nx * P.ny;
        double fl[9];
        load_node(P, f, N, (size_t)gx, 0, fl);
        double r0 = fl[0];
#pragma unroll
        for (int a = 1; a < 9; ++a) r0 += fl[a];
        const double t0 = (double)T[gx], t1 = (double)T[P.nx + gx], t2 = (double)T[2 * P.nx + gx];
        qw = -P.cv_chi * r0 * (-3.0 * t0 + 4.0 * t1 - t2) / 2.0;
        if (q_local) q_local[gx] = qw;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) qw += __shfl_xor(qw, off, 64);
    if (lane == 0 && hf_part) hf_part[blockIdx.x] = qw;
}

// Heat-flux bookkeeping of the state after the last step, one block per lattice.
__global__ void k_flush_heat_flux(const Inst *__restrict__ insts)
{
    const Inst &I = insts[blockIdx.x];
    reduce_heat_flux(I.hf_part, I.nbxB, I.P.nx, I.sc, I.sc->tA);
}

// Read-back: rho, v of Eq. (6) with the force of the current state, T, and
// the completed f, all widened to FP64.
template <typename S>
__global__ __launch_bounds__(NT) void k_read(DevParams P, const S *__restrict__ fin, const S *__restrict__ Tin,
                                             double *__restrict__ rho_o, double *__restrict__ ux_o,
                                             double *__restrict__ uy_o, double *__restrict__ T_o,
                                             double *__restrict__ f_o, Scalars *sc, int nbx)
{
    __shared__ double psi_s[(TXR + 2) * (TYR + 2)];
    const int bx = blockIdx.x % nbx, by = blockIdx.x / nbx;
    const int x0 = bx * TXR, y0 = by * TYR;
    const size_t N = (size_t)P.nx * P.ny;
    const bool frozen = P.mode == MODE_THERMAL_ONLY;
    if (!frozen) tile_psi<S, TXR, TYR>(P, fin, Tin, x0, y0, psi_s, sc, sc->tA);
    __syncthreads();
    const double rho_ave = sc->rho_ave;
    const int tx = threadIdx.x % TXR;
    for (int ly = threadIdx.x / TXR; ly < TYR; ly += NT / TXR) {
        const int gx = x0 + tx, gy = y0 + ly;
        if (gx >= P.nx || gy >= P.ny) continue;
        const size_t c = (size_t)gy * P.nx + gx;
        double fl[9];
        load_node(P, fin, N, c, gy, fl);
        double rho = 0.0, jx = 0.0, jy = 0.0;
        {
            double r = fl[0];
#pragma unroll
            for (int a = 1; a < 9; ++a) r += fl[a];
            rho = r;
            jx = (double)(fl[1] - fl[3] + fl[5] - fl[6] - fl[7] + fl[8]);
            jy = (double)(fl[2] - fl[4] + fl[5] + fl[6] - fl[7] - fl[8]);
        }
        double Fx = 0.0, Fy = 0.0, Q = 0.0;
        if (!frozen) node_force<TXR + 2>(P, psi_s, tx, ly, gy, rho, rho_ave, Fx, Fy, Q);
        if (rho_o) rho_o[c] = rho;
        if (ux_o) ux_o[c] = (jx + 0.5 * Fx) / rho;
        if (uy_o) uy_o[c] = (jy + 0.5 * Fy) / rho;
        if (T_o) T_o[c] = P.T_ref + (double)Tin[c];
        if (f_o)
            for (int a = 0; a < 9; ++a) f_o[(size_t)a * N + c] = (double)fl[a];
    }
}

// Write the Zou-He completion into the stored wall rows (before a checkpoint).
template <typename S>
__global__ void k_complete_walls(DevParams P, S *__restrict__ f)
{
    const int gx = blockIdx.x * blockDim.x + threadIdx.x;
    if (P.periodic_y || P.mode == MODE_THERMAL_ONLY || gx >= P.nx) return;
    const size_t N = (size_t)P.nx * P.ny;
    for (int side = 0; side < 2; ++side) {
        const int gy = side ? P.ny - 1 : 0;
        const size_t c = (size_t)gy * P.nx + gx;
        double fl[9];
        load_node(P, f, N, c, gy, fl);
        for (int a = 0; a < 9; ++a) f[(size_t)a * N + c] = S(fl[a]);
    }
}

// Set the bottom-wall row of both temperature buffers.
template <typename S>
__global__ void k_set_heater(DevParams P, const double *__restrict__ Tb, S *__restrict__ T0, S *__restrict__ T1)
{
    const int gx = blockIdx.x * blockDim.x + threadIdx.x;
    if (P.periodic_y || gx >= P.nx) return;
    T0[gx] = S(Tb[gx] - P.T_ref);
    T1[gx] = S(Tb[gx] - P.T_ref);
}

}  // namespace lbb
