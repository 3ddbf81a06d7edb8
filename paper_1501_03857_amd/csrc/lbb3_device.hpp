// Device code of the three-dimensional path: the time step of the hybrid
// thermal pseudopotential LB boiling model (arXiv:1501.03857, Sec. 2) on the
// D3Q19 lattice, the extension the paper names as its future work (Sec. 4).
// gfx950, wave64.
//
// Data layout in HBM (structure of arrays, x fastest, then y, then z):
//   f[2][19][nz][ny][nx]  post-streaming populations, double-buffered; wall
//                         rows never store the five populations arriving
//                         from outside (completed by the Zou-He rule on read)
//   T[2][nz][ny][nx]      T - T_ref (T_ref = 0 in FP64, T_s in FP32)
//   rho, v[3]             density and the velocity the temperature equation
//                         sees (zero on wall rows), storage precision
//   psi                   pseudopotential, FP64
//   coef[5]               per-node coefficients of the temperature equation
//   Ts[2], acc            RK4 stage values and slope sum
// Walls at y = 0 and y = ny-1 (gravity along -y), periodic x and z.
//
// One step t -> t+1 is seven launches, one node per thread except the first
// RK4 stage:
//   k3_psi      rho (Eq. (6)) and psi (FP64 Peng-Robinson EOS, Eq. (21)) of
//               state t; per-block FP64 partials of the mass and, on the
//               bottom wall, of the heat flux of state t (Sec. 3.2)
//   k3_reduce   one block: rho_ave (Eq. (9)) and the heat-flux sample
//   k3_lb       forces (Eqs. (7), (9), (22)), velocity, MRT collision with
//               the improved forcing (Eqs. (2), (4), (5), (8)) and push
//               streaming (Eq. (3))
//   k3_stage0   the first RK4 stage (Eqs. (19)-(20)) of Eq. (18), one
//               thread a column of nodes marching along z with a ring of
//               planes in LDS; it also forms the per-node coefficients
//   k3_stage x3 the other three stages; the last writes T
// All reductions run in a fixed order, so results are reproducible bitwise.
#pragma once

#include "lbb_device.hpp"

namespace lbb3 {

using lbb::DevParams;
using lbb::gmem;
using lbb::rcp_nr;
using lbb::sqrt_pos;

constexpr int NT3 = 256;  // threads per block (4 waves)
constexpr int Q19 = 19;

// D3Q19 velocities: rest, +x, -x, +y, -y, +z, -z, then the edges
constexpr int EX3[Q19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int EY3[Q19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int EZ3[Q19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
// lattice weight of velocity a, times 36
constexpr int W36[Q19] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};

// Row k of the orthogonal D3Q19 moment basis at velocity a (rho, e,
// epsilon, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww, p_xy,
// p_yz, p_xz, m_x, m_y, m_z); all entries are integers.
constexpr int basis3(int k, int a)
{
    const int x = EX3[a], y = EY3[a], z = EZ3[a];
    const int e2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1;
    case 1: return 19 * e2 - 30;
    case 2: return (21 * e2 * e2 - 53 * e2 + 24) / 2;
    case 3: return x;
    case 4: return (5 * e2 - 9) * x;
    case 5: return y;
    case 6: return (5 * e2 - 9) * y;
    case 7: return z;
    case 8: return (5 * e2 - 9) * z;
    case 9: return 3 * x * x - e2;
    case 10: return (3 * e2 - 5) * (3 * x * x - e2);
    case 11: return y * y - z * z;
    case 12: return (3 * e2 - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
    }
}
// squared row norms: M M^T = diag(NORM3)
constexpr double NORM3[Q19] = {19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8};

// Velocities 2p+1 and 2p+2 (p = 0..8) are opposite.  A row of the basis is
// either even in e (rho, e, epsilon and the stress rows) or odd (the j, q and
// m rows), so an even row sees the pair sums f_a + f_abar only and an odd
// row the differences only: both transforms run on the nine pairs, which
// halves their additions.
constexpr bool odd_row(int k) { return (k >= 3 && k <= 8) || k >= 16; }

// c v added to an accumulator that holds nothing yet (first) or acc, with
// c a compile-time integer: zeros skipped, +-1 folded
__device__ __forceinline__ void acc_term(int c, double v, double &acc, bool &first)
{
    if (c == 0) return;
    if (first) acc = c == 1 ? v : (c == -1 ? -v : (double)c * v);
    else if (c == 1) acc += v;
    else if (c == -1) acc -= v;
    else acc = fma((double)c, v, acc);
    first = false;
}

// m_K = sum_a B_Ka f_a from f_0 and the pair sums s / differences d
template <int K>
__device__ __forceinline__ double row_dot(double f0, const double s[9], const double d[9])
{
    double acc = 0.0;
    bool first = true;
    if constexpr (!odd_row(K)) acc_term(basis3(K, 0), f0, acc, first);
#pragma unroll
    for (int p = 0; p < 9; ++p) acc_term(basis3(K, 2 * p + 1), odd_row(K) ? d[p] : s[p], acc, first);
    return acc;
}

template <int K = 0>
__device__ __forceinline__ void moments(double f0, const double s[9], const double d[9], double m[Q19])
{
    if constexpr (K < Q19) {
        m[K] = row_dot<K>(f0, s, d);
        moments<K + 1>(f0, s, d, m);
    }
}

__device__ __forceinline__ void moments(const double f[Q19], double m[Q19])
{
    double s[9], d[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        s[p] = f[2 * p + 1] + f[2 * p + 2];
        d[p] = f[2 * p + 1] - f[2 * p + 2];
    }
    moments(f[0], s, d, m);
}

// f_a = sum_k B_ka mh_k (mh = moments already divided by the row norms):
// the even rows give a part shared by a velocity and its opposite, the odd
// rows a part of opposite sign
__device__ __forceinline__ void from_moments(const double mh[Q19], double f[Q19])
{
    {
        double ev = 0.0;
        bool fe = true;
#pragma unroll
        for (int k = 0; k < Q19; ++k)
            if (!odd_row(k)) acc_term(basis3(k, 0), mh[k], ev, fe);
        f[0] = ev;
    }
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        double ev = 0.0, od = 0.0;
        bool fe = true, fo = true;
#pragma unroll
        for (int k = 0; k < Q19; ++k) {
            if (odd_row(k)) acc_term(basis3(k, 2 * p + 1), mh[k], od, fo);
            else acc_term(basis3(k, 2 * p + 1), mh[k], ev, fe);
        }
        f[2 * p + 1] = ev + od;
        f[2 * p + 2] = ev - od;
    }
}

__device__ __forceinline__ int wrap3(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Zou-He completion of a wall node with zero velocity: the unknowns are the
// reflected knowns, corrected by the transverse momentum of the populations
// parallel to the wall, so the node carries no momentum.
__device__ __forceinline__ void zou_he3(double f[Q19], bool bottom)
{
    const double Nx = 0.5 * (f[1] - f[2] + f[11] - f[12] + f[13] - f[14]);
    const double Nz = 0.5 * (f[5] - f[6] + f[11] - f[12] - f[13] + f[14]);
    if (bottom) {
        f[3] = f[4];
        f[7] = f[8] - Nx;
        f[10] = f[9] + Nx;
        f[15] = f[16] - Nz;
        f[17] = f[18] + Nz;
    } else {
        f[4] = f[3];
        f[8] = f[7] + Nx;
        f[9] = f[10] - Nx;
        f[16] = f[15] + Nz;
        f[18] = f[17] - Nz;
    }
}

// Node of a thread in the per-node launches.  Workgroups are dispatched to
// the 8 XCDs round-robin; block q takes the chunk lbb::xcd_tile(q, nb), so
// each XCD works through one contiguous run of the lattice and the rows and
// planes its stencils share stay in its own L2.
__device__ __forceinline__ unsigned node_of_thread()
{
    return (unsigned)lbb::xcd_tile((int)blockIdx.x, (int)gridDim.x) * 256u + threadIdx.x;
}

struct Geom3 {
    int nx, ny, nz;
    unsigned n;  // nx ny nz
};

// node c -> (x, y, z)
__device__ __forceinline__ void coords(const Geom3 &g, unsigned c, int &x, int &y, int &z)
{
    const unsigned xy = (unsigned)g.nx * (unsigned)g.ny;
    z = (int)(c / xy);
    const unsigned r = c - (unsigned)z * xy;
    y = (int)(r / (unsigned)g.nx);
    x = (int)(r - (unsigned)y * (unsigned)g.nx);
}

__device__ __forceinline__ unsigned node(const Geom3 &g, int x, int y, int z)
{
    return ((unsigned)z * (unsigned)g.ny + (unsigned)y) * (unsigned)g.nx + (unsigned)x;
}

// Node-index offsets of the neighbours of one node along each axis (-1, 0,
// +1), periodic wraps folded in: the neighbour along e_a is
// c + dx[e_ax + 1] + dy[e_ay + 1] + dz[e_az + 1].  Beyond a wall (y not
// periodic) the y offset is that of the node itself; has_s / has_n say
// whether the rows below and above exist.
struct Nb3 {
    int dx[3], dy[3], dz[3];
    bool has_s, has_n;
};

__device__ __forceinline__ Nb3 neighbours(const DevParams &P, const Geom3 &g, int x, int y, int z)
{
    Nb3 b;
    const int sy = g.nx, sz = g.nx * g.ny;
    b.dx[0] = x == 0 ? g.nx - 1 : -1;
    b.dx[1] = 0;
    b.dx[2] = x == g.nx - 1 ? 1 - g.nx : 1;
    b.dz[0] = (z == 0 ? g.nz - 1 : -1) * sz;
    b.dz[1] = 0;
    b.dz[2] = (z == g.nz - 1 ? 1 - g.nz : 1) * sz;
    b.has_s = P.periodic_y || y > 0;
    b.has_n = P.periodic_y || y < g.ny - 1;
    b.dy[0] = !b.has_s ? 0 : (y == 0 ? (g.ny - 1) * sy : -sy);
    b.dy[1] = 0;
    b.dy[2] = !b.has_n ? 0 : (y == g.ny - 1 ? (1 - g.ny) * sy : sy);
    return b;
}

template <int A>
__device__ __forceinline__ unsigned nb_at(const Nb3 &b, unsigned c)
{
    return (unsigned)((int)c + b.dx[EX3[A] + 1] + b.dy[EY3[A] + 1] + b.dz[EZ3[A] + 1]);
}

__device__ __forceinline__ unsigned nb_at(const Nb3 &b, unsigned c, int a)
{
    return (unsigned)((int)c + b.dx[EX3[a] + 1] + b.dy[EY3[a] + 1] + b.dz[EZ3[a] + 1]);
}

template <typename S>
__device__ __forceinline__ void load_f(const DevParams &P, const Geom3 &g, const S *__restrict__ f, unsigned c, int y,
                                       double fl[Q19])
{
#pragma unroll
    for (int a = 0; a < Q19; ++a) fl[a] = (double)lbb::ld_at(f + (size_t)a * g.n, c * (unsigned)sizeof(S));
    if (!P.periodic_y && P.mode != lbb::MODE_THERMAL_ONLY) {
        if (y == 0) zou_he3(fl, true);
        else if (y == g.ny - 1) zou_he3(fl, false);
    }
}

struct Scalars3 {
    double rho_ave;
    double q_now, q_sum;
    long long n_samples, last_counted, t;
    unsigned long long err_step;
    unsigned int err_code, pad;
};

__device__ __forceinline__ void flag3(Scalars3 *sc, long long t, unsigned code)
{
    atomicMin(&sc->err_step, (unsigned long long)t);
    atomicOr(&sc->err_code, code);
}

// block sum of one double per thread in a fixed order; valid in thread 0
__device__ __forceinline__ double block_sum3(double v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT3 / 64; ++k) s += red[k];
    return s;
}

// psi = sqrt(2 (p_EOS - rho/3) / G), FP64 (Eq. (21)); negative on a negative radicand
__device__ __forceinline__ double psi_of(const DevParams &P, double rho, double T)
{
    const double s = 1.0 + P.kappa * (1.0 - sqrt_pos(T * P.inv_Tc));
    const double phi = s * s;
    const double D1 = 1.0 - P.b * rho;
    const double D2 = 1.0 + 2.0 * P.b * rho - P.b * P.b * rho * rho;
    const double p = (rho * P.R * T * D2 - P.a * phi * rho * rho * D1) * rcp_nr(D1 * D2);
    const double r = P.two_over_G * (p - rho * (1.0 / 3.0));
    return r > 0.0 ? sqrt_pos(r) : (r == 0.0 ? 0.0 : -1.0);
}

// ---------------------------------------------------------------------------
// rho and psi of state t; mass and bottom-wall heat-flux partials per block.
// In THERMAL_ONLY mode (f frozen) it also writes v = sum e f / rho.
template <typename S>
__global__ __launch_bounds__(NT3) void k3_psi(DevParams P, Geom3 g, const S *__restrict__ f, const S *__restrict__ T,
                                             S *__restrict__ rho_o, double *__restrict__ psi_o, S *__restrict__ vx_o,
                                             S *__restrict__ vy_o, S *__restrict__ vz_o, double *__restrict__ mpart,
                                             double *__restrict__ hpart, Scalars3 *sc)
{
    __shared__ double red[NT3 / 64];
    const unsigned c = node_of_thread();
    double mass = 0.0, qw = 0.0;
    const long long t = sc->t;
    if (c < g.n) {
        int x, y, z;
        coords(g, c, x, y, z);
        double fl[Q19];
        load_f(P, g, f, c, y, fl);
        double r = fl[0];
#pragma unroll
        for (int a = 1; a < Q19; ++a) r += fl[a];
        mass = r;
        const double Tc_ = P.T_ref + (double)((const gmem<S> *)T)[c];
        if (!(r > 0.0) || !(r < 1e300)) flag3(sc, t, lbb::ERR_RHO);
        ((gmem<S> *)rho_o)[c] = S(r);
        if (P.mode == lbb::MODE_THERMAL_ONLY) {
            const bool wall = !P.periodic_y && (y == 0 || y == g.ny - 1);
            double j[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int a = 1; a < Q19; ++a) {
                j[0] += EX3[a] * fl[a];
                j[1] += EY3[a] * fl[a];
                j[2] += EZ3[a] * fl[a];
            }
            ((gmem<S> *)vx_o)[c] = wall ? S(0) : S(j[0] / r);
            ((gmem<S> *)vy_o)[c] = wall ? S(0) : S(j[1] / r);
            ((gmem<S> *)vz_o)[c] = wall ? S(0) : S(j[2] / r);
        } else {
            const double psi = psi_of(P, r, Tc_);
            if (!(psi >= 0.0) || !(psi < 1e300)) flag3(sc, t, lbb::ERR_PSI);
            ((gmem<double> *)psi_o)[c] = psi;
        }
        if (!P.periodic_y && y == 0) {
            const double t0 = (double)((const gmem<S> *)T)[c];
            const double t1 = (double)((const gmem<S> *)T)[c + (unsigned)g.nx];
            const double t2 = (double)((const gmem<S> *)T)[c + 2u * (unsigned)g.nx];
            qw = -P.cv_chi * r * (-3.0 * t0 + 4.0 * t1 - t2) / 2.0;
        }
    }
    const double ms = block_sum3(mass, red);
    __syncthreads();
    const double hs = block_sum3(qw, red);
    if (threadIdx.x == 0) {
        const int chunk = lbb::xcd_tile((int)blockIdx.x, (int)gridDim.x);
        mpart[chunk] = ms;
        hpart[chunk] = hs;
    }
}

// rho_ave of state t and its heat-flux sample (counted once per state index
// t >= 1), one block; with `advance` the state index then moves to t + 1,
// the state the rest of the step produces.
constexpr int NR3 = 1024;  // threads of the reduction block

// sum of one double per thread over a block of NR3 threads, fixed order;
// valid in thread 0
__device__ __forceinline__ double block_sum_r(double v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NR3 / 64; ++k) s += red[k];
    return s;
}

// Per thread: a[k0] + a[k0 + NR3] + ... (below n) and the same for b, each
// added in that order; the loads of 16 terms of both arrays are issued before
// the first of them is added, the last group's included (a step has about 13
// terms a thread, so a loop that waited per term would wait 26 times).
__device__ __forceinline__ void strided_sum2(const double *__restrict__ a_, const double *__restrict__ b_, int k0,
                                             int n, double &sa, double &sb)
{
    const gmem<double> *__restrict__ a = (const gmem<double> *)a_;
    const gmem<double> *__restrict__ b = (const gmem<double> *)b_;
    sa = sb = 0.0;
    for (int k = k0; k < n; k += 16 * NR3) {
        double va[16], vb[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const bool in = k + j * NR3 < n;
            va[j] = in ? a[k + j * NR3] : 0.0;
            vb[j] = in ? b[k + j * NR3] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (k + j * NR3 < n) {
                sa += va[j];
                sb += vb[j];
            }
    }
}

__global__ __launch_bounds__(NR3) void k3_reduce(Geom3 g, const double *__restrict__ mpart,
                                                 const double *__restrict__ hpart, int nb, Scalars3 *sc, int advance)
{
    __shared__ double red[NR3 / 64];
    double m, h;
    strided_sum2(mpart, hpart, threadIdx.x, nb, m, h);
    const double ms = block_sum_r(m, red);
    __syncthreads();
    const double hs = block_sum_r(h, red);
    if (threadIdx.x == 0) {
        sc->rho_ave = ms / (double)g.n;
        const double q = hs / ((double)g.nx * (double)g.nz);
        sc->q_now = q;
        if (sc->t > sc->last_counted) {
            sc->q_sum += q;
            sc->n_samples += 1;
            sc->last_counted = sc->t;
        }
        if (advance) sc->t += 1;
    }
}

// total force on a node of state t (Eq. (7) + Eq. (22) + Eq. (9)) and
// Q = |F_m|^2/psi^2 (Eq. (8)): none on the wall rows; the fluid-solid force
// on the rows next to them, the wall rows being the solid
__device__ __forceinline__ void force3(const DevParams &P, const Geom3 &g, const Nb3 &nb, const double *__restrict__ psi,
                                       int y, unsigned c, double rho, double rho_ave, double F[3], double &Q)
{
    F[0] = F[1] = F[2] = 0.0;
    Q = 0.0;
    if (!P.periodic_y && (y == 0 || y == g.ny - 1)) return;
    const double pc = lbb::ld_at(psi, c * 8u);
    double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
    for (int a = 1; a < Q19; ++a) {
        const double w = (a < 7 ? 1.0 / 6.0 : 1.0 / 12.0) * lbb::ld_at(psi, nb_at(nb, c, a) * 8u);
        if (EX3[a]) sx = fma((double)EX3[a], w, sx);
        if (EY3[a]) sy = fma((double)EY3[a], w, sy);
        if (EZ3[a]) sz = fma((double)EZ3[a], w, sz);
    }
    F[0] = -P.G * pc * sx;
    F[1] = -P.G * pc * sy;
    F[2] = -P.G * pc * sz;
    Q = P.G * P.G * (sx * sx + sy * sy + sz * sz);
    if (!P.periodic_y) {
        if (y == 1) F[1] += P.Gw_bottom * pc * pc * (1.0 / 6.0);
        if (y == g.ny - 2) F[1] -= P.Gw_top * pc * pc * (1.0 / 6.0);
    }
    F[1] -= (rho - rho_ave) * P.g;
}

// MRT collision of one node in the D3Q19 basis with the improved forcing,
// from its moments m = B f; writes the post-collision populations to f.
__device__ __forceinline__ void collide3(const DevParams &P, const double m[Q19], double rho, const double v[3],
                                         const double F[3], double Q, double s_nu, double f[Q19])
{
    const double vx = v[0], vy = v[1], vz = v[2];
    const double v2 = vx * vx + vy * vy + vz * vz, vF = vx * F[0] + vy * F[1] + vz * F[2];
    const double pxx = rho * (3.0 * vx * vx - v2), pww = rho * (vy * vy - vz * vz);
    const double Sxx = 2.0 * (3.0 * vx * F[0] - vF), Sww = 2.0 * (vy * F[1] - vz * F[2]);
    // equilibrium moments (M f_eq) and forcing moments (M F' of the Guo term)
    const double meq[Q19] = {rho, rho * (19.0 * v2 - 11.0), rho * (3.0 - 5.5 * v2), rho * vx, -(2.0 / 3.0) * rho * vx,
                             rho * vy, -(2.0 / 3.0) * rho * vy, rho * vz, -(2.0 / 3.0) * rho * vz, pxx, -0.5 * pxx,
                             pww, -0.5 * pww, rho * vx * vy, rho * vy * vz, rho * vx * vz, 0.0, 0.0, 0.0};
    const double S[Q19] = {0.0,
                           38.0 * vF + P.sig_e * 9.5 * Q,
                           -11.0 * vF - P.sig_z * 3.8 * Q,
                           F[0], -(2.0 / 3.0) * F[0], F[1], -(2.0 / 3.0) * F[1], F[2], -(2.0 / 3.0) * F[2],
                           Sxx, -0.5 * Sxx, Sww, -0.5 * Sww,
                           vx * F[1] + vy * F[0], vy * F[2] + vz * F[1], vx * F[2] + vz * F[0], 0.0, 0.0, 0.0};
    const double L[Q19] = {P.s_rho, P.s_e, P.s_zeta, P.s_j, P.s_q, P.s_j, P.s_q, P.s_j, P.s_q, s_nu,
                           P.s_zeta, s_nu, P.s_zeta, s_nu, s_nu, s_nu, P.s_q, P.s_q, P.s_q};
    double mh[Q19];
#pragma unroll
    for (int k = 0; k < Q19; ++k)
        mh[k] = (m[k] - L[k] * (m[k] - meq[k]) + (1.0 - 0.5 * L[k]) * S[k]) * (1.0 / NORM3[k]);
    // the density moment is conserved (m_eq = rho, S = 0), and rho/19 is
    // rounded once: 1/19 as its nearest double plus the remainder.  rho *
    // fl(1/19) alone is biased (fl(1/19) < 1/19); the outputs carry 19 times
    // this value, so every node would lose a fixed 5.6e-17 rho of mass per
    // step.
    mh[0] = fma(rho, 1.0 / 19.0, rho * 0x1.af286bca1af28p-59);
    from_moments(mh, f);
}

// forces, velocity, collision and push streaming of state t
template <typename S>
__global__ __launch_bounds__(NT3) void k3_lb(DevParams P, Geom3 g, const S *__restrict__ fin, S *__restrict__ fout,
                                            const double *__restrict__ psi, S *__restrict__ vx_o,
                                            S *__restrict__ vy_o, S *__restrict__ vz_o, const Scalars3 *sc)
{
    const unsigned c = node_of_thread();
    if (c >= g.n) return;
    int x, y, z;
    coords(g, c, x, y, z);
    double f[Q19], m[Q19];
    load_f(P, g, fin, c, y, f);
    moments(f, m);  // m_0 = rho, (m_3, m_5, m_7) = sum e f
    const double rho = m[0];
    const Nb3 nb = neighbours(P, g, x, y, z);
    double F[3], Q;
    force3(P, g, nb, psi, y, c, rho, sc->rho_ave, F, Q);
    const double inv = rcp_nr(rho);
    const double v[3] = {(m[3] + 0.5 * F[0]) * inv, (m[5] + 0.5 * F[1]) * inv, (m[7] + 0.5 * F[2]) * inv};
    const bool wall = !P.periodic_y && (y == 0 || y == g.ny - 1);
    ((gmem<S> *)vx_o)[c] = wall ? S(0) : S(v[0]);
    ((gmem<S> *)vy_o)[c] = wall ? S(0) : S(v[1]);
    ((gmem<S> *)vz_o)[c] = wall ? S(0) : S(v[2]);
    collide3(P, m, rho, v, F, Q, rcp_nr(P.tau_V + (rho - P.rho_V) * P.tau_slope), f);
#pragma unroll
    for (int a = 0; a < Q19; ++a) {
        const bool keep = EY3[a] < 0 ? nb.has_s : (EY3[a] > 0 ? nb.has_n : true);
        if (keep) lbb::st_at(fout + (size_t)a * g.n, nb_at(nb, c, a) * (unsigned)sizeof(S), S(f[a]));
    }
}

// ---------------------------------------------------------------------------
// Temperature equation (Eq. (18)) by RK4: K = -(a . grad T) + chi lap T +
// c1 T + c2 sqrt(T), with a = v - chi grad(rho)/rho and the pressure work
// -w T (dp/dT)_rho = c1 T + c2 sqrt(T), w = div v / (rho c_v) (the same
// split of (dp/dT)_rho as in two dimensions), on rows 1..ny-2; the wall rows
// keep their Dirichlet values in every stage.

// isotropic D3Q19 stencils at node c of field p: d_i p = 3 sum_a W_a e_ai
// p(c + e_a) for the directions i in the mask, and
// lap p = 6 sum_a W_a (p(c + e_a) - p(c)) when lap is non-null; only the
// velocities a stencil needs are read (interior rows only)
template <int MASK, typename T_>
__device__ __forceinline__ void stencil3(const Nb3 &nb, const T_ *__restrict__ p, unsigned c, double grad[3],
                                         double *lap)
{
    const double pc = (double)lbb::ld_at(p, c * (unsigned)sizeof(T_));
    double gx = 0.0, gy = 0.0, gz = 0.0, l = 0.0;
#pragma unroll
    for (int a = 1; a < Q19; ++a) {
        const bool need = lap || ((MASK & 1) && EX3[a]) || ((MASK & 2) && EY3[a]) || ((MASK & 4) && EZ3[a]);
        if (!need) continue;
        const double w = W36[a] * (1.0 / 36.0);
        const double val = (double)lbb::ld_at(p, nb_at(nb, c, a) * (unsigned)sizeof(T_));
        if ((MASK & 1) && EX3[a]) gx = fma(EX3[a] * w, val, gx);
        if ((MASK & 2) && EY3[a]) gy = fma(EY3[a] * w, val, gy);
        if ((MASK & 4) && EZ3[a]) gz = fma(EZ3[a] * w, val, gz);
        if (lap) l = fma(w, val - pc, l);
    }
    grad[0] = 3.0 * gx;
    grad[1] = 3.0 * gy;
    grad[2] = 3.0 * gz;
    if (lap) *lap = 6.0 * l;
}

// Stage K (1..3).  Reads the stage input Tin and the per-node coefficients
// the first stage formed, writes the next stage input Tout = T^t + c_{K+1} h
// (K < 3) or T^{t+1} (K = 3).
template <typename S, int K>
__global__ __launch_bounds__(NT3) void k3_stage(DevParams P, Geom3 g, const S *__restrict__ T0,
                                               const S *__restrict__ Tin, S *__restrict__ Tout,
                                               S *__restrict__ acc, const S *__restrict__ coef, Scalars3 *sc)
{
    static_assert(K >= 1 && K <= 3, "the first stage is k3_stage0");
    const unsigned c = node_of_thread();
    if (c >= g.n) return;
    int x, y, z;
    coords(g, c, x, y, z);
    const bool wall = !P.periodic_y && (y == 0 || y == g.ny - 1);
    const double t0 = (double)lbb::ld_at(T0, c * (unsigned)sizeof(S));
    double h = 0.0;
    if (!wall) {
        const Nb3 nb = neighbours(P, g, x, y, z);
        double a[3], c1, c2;
        a[0] = (double)lbb::ld_at(coef + 0 * (size_t)g.n, c * (unsigned)sizeof(S));
        a[1] = (double)lbb::ld_at(coef + 1 * (size_t)g.n, c * (unsigned)sizeof(S));
        a[2] = (double)lbb::ld_at(coef + 2 * (size_t)g.n, c * (unsigned)sizeof(S));
        c1 = (double)lbb::ld_at(coef + 3 * (size_t)g.n, c * (unsigned)sizeof(S));
        c2 = (double)lbb::ld_at(coef + 4 * (size_t)g.n, c * (unsigned)sizeof(S));
        double gT[3], lap;
        stencil3<7>(nb, Tin, c, gT, &lap);
        const double Tabs = P.T_ref + (double)lbb::ld_at(Tin, c * (unsigned)sizeof(S));
        h = -(a[0] * gT[0] + a[1] * gT[1] + a[2] * gT[2]) + P.chi * lap + c1 * Tabs + c2 * sqrt_pos(Tabs);
    }
    gmem<S> *ac = (gmem<S> *)acc;
    constexpr double wst = K == 3 ? 1.0 : 2.0;
    const double sum = (double)ac[c] + wst * h;
    if constexpr (K < 3) {
        constexpr double cst = K < 2 ? 0.5 : 1.0;
        ac[c] = S(sum);
        ((gmem<S> *)Tout)[c] = S(t0 + cst * h);
    } else {
        const double Tn = wall ? t0 : (double)S(t0 + sum * (1.0 / 6.0));
        if (!wall && !(P.T_ref + Tn > 0.0)) flag3(sc, sc->t, lbb::ERR_T);
        ((gmem<S> *)Tout)[c] = S(Tn);
    }
}

// First RK4 stage, marching along z.  Besides the temperature stencil it
// forms the per-node coefficients of the slope from the gradient of rho and
// the divergence of v: 66 neighbour values a node, which as gathers through
// the caches bound the launch.  A block owns RXZ x RYZ region columns (TXZ x
// TYZ interior columns and a halo of one in x and y), one thread a column, and
// a run of tl.zc planes.  It keeps three planes of rho, v and T in LDS as a
// ring, in the storage precision (so that in FP32 four blocks fit a CU), loads
// plane z + 2 into registers while it works on plane z, and then moves it into
// the slot of plane z - 1.  A value is loaded (32/30) (16/14) (zc + 2)/zc
// times, against 2.4 times for tiles with a halo in all three directions, and
// the loads of the next plane run under the stencils of the current one.  The
// stencils widen each value to FP64 and add the same terms in the same order as
// stencil3, so the arithmetic is that of the per-node stages.
constexpr int RXZ = 32, RYZ = 16;            // region columns along x and y
constexpr int TXZ = RXZ - 2, TYZ = RYZ - 2;  // interior columns
constexpr int NSZ = RXZ * RYZ;               // threads of a block, one a region column

struct Tiles3 {
    int ntx, nty, ntz;  // column tiles along x and y, plane runs along z
    int zc;             // planes of a run
};

// Stencil of a field at region cell `cell` of the middle plane, the planes
// below and above given apart (terms in the order of stencil3)
template <int MASK, typename L>
__device__ __forceinline__ void stencil3_ring(const L *pm, const L *pc, const L *pp, int cell, double grad[3],
                                              double *lap)
{
    const double v0 = (double)pc[cell];
    double gx = 0.0, gy = 0.0, gz = 0.0, l = 0.0;
#pragma unroll
    for (int a = 1; a < Q19; ++a) {
        const bool need = lap || ((MASK & 1) && EX3[a]) || ((MASK & 2) && EY3[a]) || ((MASK & 4) && EZ3[a]);
        if (!need) continue;
        const double w = W36[a] * (1.0 / 36.0);
        const L *pl = EZ3[a] < 0 ? pm : (EZ3[a] > 0 ? pp : pc);
        const double val = (double)pl[cell + EX3[a] + RXZ * EY3[a]];
        if ((MASK & 1) && EX3[a]) gx = fma(EX3[a] * w, val, gx);
        if ((MASK & 2) && EY3[a]) gy = fma(EY3[a] * w, val, gy);
        if ((MASK & 4) && EZ3[a]) gz = fma(EZ3[a] * w, val, gz);
        if (lap) l = fma(w, val - v0, l);
    }
    grad[0] = 3.0 * gx;
    grad[1] = 3.0 * gy;
    grad[2] = 3.0 * gz;
    if (lap) *lap = 6.0 * l;
}

template <typename S>
__global__ __launch_bounds__(NSZ) void k3_stage0(DevParams P, Geom3 g, Tiles3 tl, const S *__restrict__ T0,
                                                S *__restrict__ Tout, S *__restrict__ acc, S *__restrict__ coef,
                                                const S *__restrict__ rho, const S *__restrict__ vx,
                                                const S *__restrict__ vy, const S *__restrict__ vz)
{
    __shared__ S sh[3][5][NSZ];  // ring slot (plane) x field (rho, vx, vy, vz, T) x region column
    const int nt = tl.ntx * tl.nty * tl.ntz;
    const int tile = lbb::xcd_tile((int)blockIdx.x, nt);
    const int bx = tile % tl.ntx, by = (tile / tl.ntx) % tl.nty, bz = tile / (tl.ntx * tl.nty);
    const int x0 = bx * TXZ, y0 = by * TYZ, z0 = bz * tl.zc;
    const int z1 = min(z0 + tl.zc, g.nz);  // this block's planes are z0 .. z1-1
    const bool walls = !P.periodic_y;
    const int rx = (int)threadIdx.x % RXZ, ry = (int)threadIdx.x / RXZ;
    // this thread's region column: x periodic, y periodic or cut at the walls
    int x = (x0 + rx - 1) % g.nx, y = y0 + ry - 1;
    if (x < 0) x += g.nx;
    bool in = true;  // false beyond a wall: never read
    if (walls) in = y >= 0 && y < g.ny;
    else {
        y %= g.ny;
        if (y < 0) y += g.ny;
    }
    const unsigned col = in ? (unsigned)y * (unsigned)g.nx + (unsigned)x : 0u;
    const unsigned pl = (unsigned)g.nx * (unsigned)g.ny;
    const S *src[5] = {rho, vx, vy, vz, T0};
    auto load = [&](int z, S v[5]) {  // plane z in [-1, nz]
        const unsigned off = ((unsigned)wrap3(z, g.nz) * pl + col) * (unsigned)sizeof(S);
#pragma unroll
        for (int f = 0; f < 5; ++f) v[f] = in ? lbb::ld_at(src[f], off) : S(0);
    };
    auto put = [&](int slot, const S v[5]) {
#pragma unroll
        for (int f = 0; f < 5; ++f) sh[slot][f][threadIdx.x] = v[f];
    };
    S nxt[5];
    // plane q sits in slot (q - z0 + 1) mod 3
    load(z0 - 1, nxt);
    put(0, nxt);
    load(z0, nxt);
    put(1, nxt);
    load(z0 + 1, nxt);
    put(2, nxt);
    __syncthreads();

    const int xi = x0 + rx - 1, yi = y0 + ry - 1;
    const bool mine = rx >= 1 && rx <= TXZ && ry >= 1 && ry <= TYZ && xi < g.nx && yi < g.ny;
    const bool wall = walls && (yi == 0 || yi == g.ny - 1);
    const int cell = (int)threadIdx.x;
    int sm = 0;  // slot of plane z - 1
    for (int z = z0; z < z1; ++z) {
        const bool more = z + 2 <= z1;  // plane z + 2 is the upper neighbour of a plane of this run
        if (more) load(z + 2, nxt);
        const int sc = sm == 2 ? 0 : sm + 1, sp = sc == 2 ? 0 : sc + 1;
        if (mine) {
            const unsigned c = ((unsigned)z * (unsigned)g.ny + (unsigned)yi) * (unsigned)g.nx + (unsigned)xi;
            const double t0 = (double)sh[sc][4][cell];
            double h = 0.0;
            if (!wall) {
                // coefficients, once per step: grad rho, div v, A(rho), B(rho)
                const double r = (double)sh[sc][0][cell];
                double gr[3], dx_[3], dy_[3], dz_[3];
                stencil3_ring<7>(sh[sm][0], sh[sc][0], sh[sp][0], cell, gr, nullptr);
                stencil3_ring<1>(sh[sm][1], sh[sc][1], sh[sp][1], cell, dx_, nullptr);
                stencil3_ring<2>(sh[sm][2], sh[sc][2], sh[sp][2], cell, dy_, nullptr);
                stencil3_ring<4>(sh[sm][3], sh[sc][3], sh[sp][3], cell, dz_, nullptr);
                const double div = dx_[0] + dy_[1] + dz_[2];
                const double D1 = 1.0 - P.b * r, D2 = 1.0 + 2.0 * P.b * r - P.b * P.b * r * r;
                const double inv = rcp_nr(r * D1 * D2);
                const double chi_r = P.chi * D1 * D2 * inv;
                const double Aw = P.R_cv * div * (r * D2 * inv), Bw = P.a_cv * r * div * (r * D1 * inv);
                double a[3] = {(double)sh[sc][1][cell] - chi_r * gr[0], (double)sh[sc][2][cell] - chi_r * gr[1],
                               (double)sh[sc][3][cell] - chi_r * gr[2]};
                double c1 = Bw * P.k2_Tc - Aw;
                double c2 = -Bw * P.k1k_rsTc;
                gmem<S> *cf = (gmem<S> *)coef;
                cf[0 * (size_t)g.n + c] = S(a[0]);
                cf[1 * (size_t)g.n + c] = S(a[1]);
                cf[2 * (size_t)g.n + c] = S(a[2]);
                cf[3 * (size_t)g.n + c] = S(c1);
                cf[4 * (size_t)g.n + c] = S(c2);
                a[0] = (double)S(a[0]);
                a[1] = (double)S(a[1]);
                a[2] = (double)S(a[2]);
                c1 = (double)S(c1);
                c2 = (double)S(c2);
                double gT[3], lap;
                stencil3_ring<7>(sh[sm][4], sh[sc][4], sh[sp][4], cell, gT, &lap);
                const double Tabs = P.T_ref + t0;
                h = -(a[0] * gT[0] + a[1] * gT[1] + a[2] * gT[2]) + P.chi * lap + c1 * Tabs + c2 * sqrt_pos(Tabs);
            }
            ((gmem<S> *)acc)[c] = S(h);
            ((gmem<S> *)Tout)[c] = S(t0 + 0.5 * h);
        }
        __syncthreads();  // every read of plane z - 1 is done
        if (more) put(sm, nxt);
        __syncthreads();
        sm = sc;
    }
}

// ---------------------------------------------------------------------------
// Set-up and read-back.

template <typename S>
__global__ void k3_set_state(DevParams P, Geom3 g, const double *__restrict__ rho, const double *__restrict__ u,
                             const double *__restrict__ T, const double *__restrict__ Tb, S *__restrict__ f,
                             S *__restrict__ T0, S *__restrict__ T1, Scalars3 *sc)
{
    const unsigned c = node_of_thread();
    if (c >= g.n) return;
    int x, y, z;
    coords(g, c, x, y, z);
    const bool wall = !P.periodic_y && (y == 0 || y == g.ny - 1);
    const double r = rho[c];
    const double vx = (u && !wall) ? u[c] : 0.0, vy = (u && !wall) ? u[g.n + c] : 0.0,
                 vz = (u && !wall) ? u[2 * (size_t)g.n + c] : 0.0;
    const double v2 = vx * vx + vy * vy + vz * vz;
#pragma unroll
    for (int a = 0; a < Q19; ++a) {
        const double eu = EX3[a] * vx + EY3[a] * vy + EZ3[a] * vz;
        const double W = a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
        f[(size_t)a * g.n + c] = S(W * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * v2));
    }
    double Tv = T ? T[c] : P.Ts;
    if (!P.periodic_y && y == 0) Tv = Tb[(size_t)z * g.nx + x];
    if (!P.periodic_y && y == g.ny - 1) Tv = P.Ts;
    T0[c] = S(Tv - P.T_ref);
    T1[c] = S(Tv - P.T_ref);
    if (!(r > 0.0) || !(Tv > 0.0) || !(P.b * r < 1.0)) flag3(sc, 0, lbb::ERR_RHO);
}

// rho, v of Eq. (6) with the force of the current state (psi and rho_ave of
// the current state must be up to date), T and the completed f, in FP64
template <typename S>
__global__ __launch_bounds__(NT3) void k3_read(DevParams P, Geom3 g, const S *__restrict__ fin,
                                              const S *__restrict__ Tin, const double *__restrict__ psi,
                                              const Scalars3 *sc, double *__restrict__ rho_o, double *__restrict__ u_o,
                                              double *__restrict__ T_o, double *__restrict__ f_o,
                                              double *__restrict__ qloc)
{
    const unsigned c = node_of_thread();
    if (c >= g.n) return;
    int x, y, z;
    coords(g, c, x, y, z);
    double f[Q19];
    load_f(P, g, fin, c, y, f);
    double r = f[0];
#pragma unroll
    for (int a = 1; a < Q19; ++a) r += f[a];
    double F[3] = {0.0, 0.0, 0.0}, Q;
    if (P.mode != lbb::MODE_THERMAL_ONLY) force3(P, g, neighbours(P, g, x, y, z), psi, y, c, r, sc->rho_ave, F, Q);
    double j[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 1; a < Q19; ++a) {
        j[0] += EX3[a] * f[a];
        j[1] += EY3[a] * f[a];
        j[2] += EZ3[a] * f[a];
    }
    if (rho_o) rho_o[c] = r;
    if (u_o)
        for (int d = 0; d < 3; ++d) u_o[(size_t)d * g.n + c] = (j[d] + 0.5 * F[d]) / r;
    if (T_o) T_o[c] = P.T_ref + (double)Tin[c];
    if (f_o)
        for (int a = 0; a < Q19; ++a) f_o[(size_t)a * g.n + c] = f[a];
    if (qloc && !P.periodic_y && y == 0) {
        const double t0 = (double)Tin[c], t1 = (double)Tin[c + (unsigned)g.nx], t2 = (double)Tin[c + 2u * (unsigned)g.nx];
        qloc[(size_t)z * g.nx + x] = -P.cv_chi * r * (-3.0 * t0 + 4.0 * t1 - t2) / 2.0;
    }
}

template <typename S>
__global__ void k3_set_heater(DevParams P, Geom3 g, const double *__restrict__ Tb, S *__restrict__ T0,
                              S *__restrict__ T1)
{
    const unsigned k = blockIdx.x * NT3 + threadIdx.x;
    if (P.periodic_y || k >= (unsigned)g.nx * (unsigned)g.nz) return;
    const unsigned z = k / (unsigned)g.nx, x = k - z * (unsigned)g.nx;
    const unsigned c = node(g, (int)x, 0, (int)z);
    T0[c] = S(Tb[k] - P.T_ref);
    T1[c] = S(Tb[k] - P.T_ref);
}

}  // namespace lbb3
