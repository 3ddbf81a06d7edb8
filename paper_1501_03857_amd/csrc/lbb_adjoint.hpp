// Device code of the discrete adjoint: gradient of the time-averaged bottom
// wall heat flux J = (1/N) sum_{n=1..N} q^n (Sec. 3.2) with respect to the
// bottom-wall temperatures T_b(x) (Sec. 3.1) and the wall strength G_w
// (Eq. (22)).  One reverse step transposes the forward step of
// lbb_device.hpp stage by stage, in reverse order, over whole-lattice FP64
// work arrays.  A launch covers any number of lattices through a lattice
// table (one lattice, or every member of a batch); the per-node kernels work
// on 64 x 4 patches (lane = column, wave = row), the temperature kernel on
// tiles with a halo in LDS.  Three launches per reverse step of state
// t -> t+1:
//   a_theradj  forces (Eqs. (7), (9), (22)) and velocity (Eq. (6)) of the
//              state on the tile and its halo (rho_ave from the mass
//              partials of the state), the tile's own nodes stored for a_lb;
//              then the RK4 temperature step (Eqs. (18)-(20)) transposed:
//              div v and the coefficients of Eq. (18) formed on the tile and
//              its halo, stage inputs recomputed and the four stages
//              transposed in one tile
//   a_lb       stencil transposes of grad rho and div v (gather), push
//              streaming transposed (gather), MRT collision transposed in
//              moment space, velocity transposed, per-node force parts
//   a_final    interaction-force stencil transposed (gather), EOS transposed,
//              rho = sum f, Zou-He completion transposed, the heat-flux sample
//              of state t transposed, and rho, j, psi of state t-1 for the
//              next reverse step
// a_macro forms rho, j, psi of a state where no a_final precedes it, and
// a_hf the heat-flux source of the last state.  The state of a node is its
// stored populations: wall-row populations that arrive from outside are
// completions of the stored ones (Zou-He), so their adjoint is folded into
// the stored ones.  The adjoint covers lattices with walls (periodic x).
#pragma once

#include "lbb_device.hpp"

namespace lbb {

constexpr int NTA = 256;          // threads per adjoint block
constexpr int AXB = 64, AYB = 4;  // node patch of one block

// Work arrays of one lattice.  The per-node arrays are in the lattice's
// storage precision S (the forward values they hold are formed in FP64 from
// the stored state and rounded once; the adjoint parts are rounded once per
// reverse step), the partial sums and accumulators in FP64.  The host fills
// AdjW, whose per-node pointers are untyped; the kernels read the same
// pointers as AdjWG<S>, so every access is a global (not flat) memory
// instruction.
template <typename D, typename R>
struct AdjWT {
    // rho, j, psi and T of the state being reversed; a_final replaces them
    // by those of the state before it
    D *rho, *jx, *jy, *psi, *T1;
    D *sx, *sy, *Fx, *Fy, *vx, *vy;
    D *gDrx, *gDry, *gdiv, *grho, *gvx, *gvy, *gpsi, *gsx, *gsy;
    R *mpart;   // block mass partials of the state being reversed
    R *fpart;   // block partials of the force adjoint: [2b] rho_ave, [2b+1] G_w
    R *scal;    // [2] dJ/dG_w, accumulated over the steps
};
using AdjW = AdjWT<void, double>;
template <typename S>
using AdjWG = AdjWT<gmem<S>, gmem<double>>;

// a device array as a global-address-space pointer
template <typename T>
__device__ __forceinline__ gmem<T> *gp(T *p)
{
    return (gmem<T> *)p;
}

// One lattice of an adjoint launch: its parameters, work arrays, stored
// states and adjoint buffers, and its place in the launch grid.  A launch
// covers any number of lattices; a block finds its lattice through a block ->
// lattice table and its 64 x 4 patch from its index within the lattice.
struct AdjInst {
    DevParams P;
    AdjW w;
    const void *seg;          // stored states of the segment: slot k at 10 k nx ny elements
    void *lf[2];              // adjoint of f in the storage precision: [cur] the later state, [cur ^ 1] the earlier
    double *lT[2];            // adjoint of T (FP64), same parity
    double *gr[2];            // density adjoint of interior nodes not yet added to lf (same parity)
    int gx;                   // patches per lattice row
    int blk0;                 // first block of this lattice in the grid
    int nb;                   // blocks of this lattice
    int tgx, tblk0;           // temperature-adjoint tiles per row, first tile in its grid
};

#define A_INST                                            \
    const AdjInst &I = ai[amap[blockIdx.x]];              \
    const DevParams &P = I.P;                             \
    const AdjWG<S> &w = reinterpret_cast<const AdjWG<S> &>(I.w); \
    const int q = (int)blockIdx.x - I.blk0;               \
    (void)w;

#define A_NODE                                                 \
    const int gi = (q % I.gx) * AXB + (threadIdx.x & 63);      \
    const int gj = (q / I.gx) * AYB + (threadIdx.x >> 6);      \
    const bool on = gi < P.nx && gj < P.ny;                    \
    const size_t N = (size_t)P.nx * P.ny;                      \
    const size_t c = (size_t)gj * P.nx + gi;                   \
    (void)N;

// stored state k of lattice I (populations; T follows at 9 nx ny)
template <typename S>
__device__ __forceinline__ const gmem<S> *a_slot(const AdjInst &I, int k)
{
    return gp(static_cast<const S *>(I.seg)) + (size_t)k * 10 * (size_t)I.P.nx * I.P.ny;
}

#define A_ARGS const AdjInst *__restrict__ ai, const int *__restrict__ amap

__device__ __forceinline__ bool a_int(const DevParams &P, int j) { return j > 0 && j < P.ny - 1; }

// index of node (gi + dx, gj + dy) for a row known to lie in the lattice
__device__ __forceinline__ size_t a_at(const DevParams &P, int gi, int gj, int dx, int dy)
{
    int ii = gi + dx;
    ii = ii < 0 ? ii + P.nx : (ii >= P.nx ? ii - P.nx : ii);
    return (size_t)(gj + dy) * P.nx + ii;
}

// Neighbour c' = c - e_a of node (gi, gj) when it is an interior node (ok),
// else c itself: gathers load every neighbour without branching and weight
// the missing ones by zero.
__device__ __forceinline__ size_t a_src(const DevParams &P, int gi, int gj, int a, size_t c, bool &ok)
{
    const int jj = gj - kEY[a];
    ok = a_int(P, jj);
    return ok ? a_at(P, gi, gj, -kEX[a], -kEY[a]) : c;
}

__constant__ const double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
__constant__ const double kWpsi[9] = {0.0, 1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 3, 1.0 / 12, 1.0 / 12, 1.0 / 12, 1.0 / 12};

// Fixed-order sum of a[k * stride + off], k < n, returned to every thread of
// the block (every block forms the same value); all threads must call it.
__device__ __forceinline__ double block_sum_all(const gmem<double> *__restrict__ a, int n, int stride, int off,
                                                double *red /* [NTA / 64 + 1] */)
{
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += NTA) s += a[(size_t)k * stride + off];
    s = block_sum<NTA>(s, red);
    if (threadIdx.x == 0) red[NTA / 64] = s;
    __syncthreads();
    return red[NTA / 64];
}

// phi'(T) and phi''(T) of the Peng-Robinson alpha function (Eq. (21)), and
// u = sqrt(T / T_c).  One reciprocal square root y = 1/sqrt(T / T_c) gives
// u = (T / T_c) y and 1/(T_c u) = y / T_c.
__device__ __forceinline__ void phi_derivs(const DevParams &P, double T, double &d1, double &d2, double &u)
{
    const double x = T * P.inv_Tc;
    const double y = rsq_nr(x);
    u = x * y;
    const double iu = y * P.inv_Tc;
    d1 = -P.kappa * (1.0 + P.kappa * (1.0 - u)) * iu;
    d2 = 0.5 * P.kappa * (1.0 + P.kappa) * iu * iu * iu * P.Tc;
}

__device__ __forceinline__ void phi_derivs(const DevParams &P, double T, double &d1, double &d2)
{
    double u;
    phi_derivs(P, T, d1, d2, u);
}

// (dp/drho)_T and (dp/dT)_rho of Eq. (21); 1/D1 and 1/D2 from one reciprocal
__device__ __forceinline__ void eos_derivs(const DevParams &P, double r, double T, double &dpdr, double &dpdT)
{
    double d1, d2, u;
    phi_derivs(P, T, d1, d2, u);
    const double s = 1.0 + P.kappa * (1.0 - u);
    const double phi = s * s;
    const double D1 = 1.0 - P.b * r, D2 = 1.0 + 2.0 * P.b * r - P.b * P.b * r * r;
    const double i12 = rcp_nr(D1 * D2), i1 = D2 * i12, i2 = D1 * i12;
    dpdr = P.R * T * i1 * i1 - P.a * phi * 2.0 * r * (1.0 + P.b * r) * i2 * i2;
    dpdT = r * P.R * i1 - P.a * r * r * d1 * i2;
}

// Zou-He completion transposed: the adjoint of the completed populations of
// a wall node folded onto the stored (known) ones; the others are zeroed.
__device__ __forceinline__ void zou_he_T(double g[9], int bottom)
{
    if (bottom) {
        g[4] += g[2];
        g[7] += g[5];
        g[8] += g[6];
        g[1] += -0.5 * g[5] + 0.5 * g[6];
        g[3] += 0.5 * g[5] - 0.5 * g[6];
        g[2] = g[5] = g[6] = 0.0;
    } else {
        g[2] += g[4];
        g[5] += g[7];
        g[6] += g[8];
        g[1] += 0.5 * g[7] - 0.5 * g[8];
        g[3] += -0.5 * g[7] + 0.5 * g[8];
        g[4] = g[7] = g[8] = 0.0;
    }
}

// rho, j, psi and T of a stored state at node c; returns rho
template <typename S>
__device__ __forceinline__ double a_macro_node(const DevParams &P, const gmem<S> *__restrict__ f,
                                               const gmem<S> *__restrict__ T, size_t N, size_t c, int gj,
                                               const AdjWG<S> &w)
{
    double fl[9];
    load_node(P, f, N, c, gj, fl);
    double r = 0.0;
    for (int a = 0; a < 9; ++a) r += fl[a];
    const double Tv = P.T_ref + (double)T[c];
    w.rho[c] = r;
    w.jx[c] = fl[1] - fl[3] + fl[5] - fl[6] - fl[7] + fl[8];
    w.jy[c] = fl[2] - fl[4] + fl[5] + fl[6] - fl[7] - fl[8];
    w.T1[c] = Tv;
    w.psi[c] = pseudopotential(P, r, Tv);
    return r;
}

template <typename S>
__global__ __launch_bounds__(NTA) void a_macro(A_ARGS, int k)
{
    __shared__ double red[NTA / 64];
    A_INST
    A_NODE
    const gmem<S> *f = a_slot<S>(I, k);
    const double m = on ? a_macro_node<S>(P, f, f + 9 * N, N, c, gj, w) : 0.0;
    const double s = block_sum<NTA>(m, red);
    if (threadIdx.x == 0) w.mpart[q] = s;
}

// Force (Eqs. (7), (22), (9)) and velocity (Eq. (6)) of the stored state at
// node (gi, gj) from the state's psi and rho: the stencil sums sx, sy of
// psi, F, the isotropic gradient of rho and v.  Wall rows carry no force.
struct NodeForce {
    double sx, sy, Fx, Fy, rx, ry, vx, vy;
};

// isotropic gradient of rho at interior node (gi, gj)
template <typename WG>
__device__ __forceinline__ void grad_rho(const DevParams &P, const WG &w, int gi, int gj, double &rx, double &ry)
{
    rx = ry = 0.0;
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        const double rn = w.rho[a_at(P, gi, gj, kEX[a], kEY[a])];
        rx += 3.0 * kW[a] * kEX[a] * rn;
        ry += 3.0 * kW[a] * kEY[a] * rn;
    }
}

template <typename WG>
__device__ __forceinline__ NodeForce force_node(const DevParams &P, const WG &w, int gi, int gj, size_t c,
                                                double rho_ave)
{
    NodeForce o;
    o.sx = o.sy = o.Fx = o.Fy = o.rx = o.ry = 0.0;
    const double r = w.rho[c];
    if (a_int(P, gj)) {
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            const double pn = w.psi[a_at(P, gi, gj, kEX[a], kEY[a])];
            o.sx += kWpsi[a] * pn * kEX[a];
            o.sy += kWpsi[a] * pn * kEY[a];
        }
        grad_rho(P, w, gi, gj, o.rx, o.ry);
        const double ps = w.psi[c];
        o.Fx = -P.G * ps * o.sx;
        o.Fy = -P.G * ps * o.sy;
        if (gj == 1) o.Fy += P.Gw_bottom * ps * ps / 6.0;
        if (gj == P.ny - 2) o.Fy -= P.Gw_top * ps * ps / 6.0;
        o.Fy -= (r - rho_ave) * P.g;
    }
    const double ir = rcp_nr(r);
    o.vx = (w.jx[c] + 0.5 * o.Fx) * ir;
    o.vy = (w.jy[c] + 0.5 * o.Fy) * ir;
    return o;
}

// div v and the coefficients of Eq. (18) at interior node (gi, gj), formed
// where the temperature adjoint needs them (wall rows carry none):
// K(T) = AX d_x T + AY d_y T + chi lap T - IA divv T + IB divv T phi'(T) with
// AX = -vx + chi d_x rho / rho, IA = R / ((1 - b rho) c_v),
// IB = a rho / ((1 + 2 b rho - b^2 rho^2) c_v); E1, E2 give the rho
// derivative of the pressure-work factor.
struct DivCoef {
    double dv, ax, ay, IA, IB;
};

// From the velocity planes VX, VY of the tile region (region row r, lane l,
// both at least one node from the region's edge) and the node's own v_x, v_y,
// d_x rho, d_y rho and rho.
template <typename PT>
__device__ __forceinline__ DivCoef div_coef(const DevParams &P, const PT (*VX)[64], const PT (*VY)[64],
                                            int r, int l, int gj, double vx, double vy, double rx, double ry,
                                            double rho)
{
    double dv = 0.0;
#pragma unroll
    for (int a = 1; a < 9; ++a) {
        // the velocity the temperature equation sees is zero on the wall rows
        const double m = a_int(P, gj + kEY[a]) ? 3.0 * kW[a] : 0.0;
        dv += m * (kEX[a] * (double)VX[r + kEY[a]][l + kEX[a]] + kEY[a] * (double)VY[r + kEY[a]][l + kEX[a]]);
    }
    const double D1 = 1.0 - P.b * rho, D2 = 1.0 + 2.0 * P.b * rho - P.b * P.b * rho * rho;
    const double inv = rcp_nr(rho * D1 * D2);
    const double ri = D1 * D2 * inv, i1 = rho * D2 * inv, i2 = rho * D1 * inv;
    const double icv = P.inv_cv;
    DivCoef k;
    k.dv = dv;
    k.ax = -vx + P.chi * rx * ri;
    k.ay = -vy + P.chi * ry * ri;
    k.IA = P.R * i1 * icv;
    k.IB = P.a * rho * i2 * icv;
    return k;
}

// 1/rho and the rho derivatives E1 = R b i1^2 / c_v, E2 = a (1 + b^2 rho^2)
// i2^2 / c_v of the pressure-work coefficients at a node of density r
__device__ __forceinline__ void pw_derivs(const DevParams &P, double r, double &ri, double &E1, double &E2)
{
    const double D1 = 1.0 - P.b * r, D2 = 1.0 + 2.0 * P.b * r - P.b * P.b * r * r;
    const double inv = rcp_nr(r * D1 * D2);
    const double i1 = r * D2 * inv, i2 = r * D1 * inv;
    const double icv = P.inv_cv;
    ri = D1 * D2 * inv;
    E1 = P.R * P.b * i1 * i1 * icv;
    E2 = P.a * (1.0 + P.b * P.b * r * r) * i2 * i2 * icv;
}

// ---------------------------------------------------------------------------
// The temperature step transposed in one launch: the RK4 stage inputs
// T_2..T_4 recomputed (Eqs. (19)-(20)) and the four stages transposed, last
// first, on one tile with a halo of 7 (three forward stencil stages, four
// reverse ones), in LDS.  Lane = column (tile TAX = 50 wide, one wave64 with
// the halo), each of the TAW waves owns fixed region rows; tiles are TAY rows
// high (16 or 24, or 4 where 16-row tiles would leave the chip underfilled).  Stage k's slope
// adjoint is g_k = w_k lT^{t+1}/6 + c_{k+1} gT_{k+1} (RK4 weights w = (1, 2,
// 2, 1), g_3 = lT^{t+1}/6), gT_k being the adjoint of the stage input T_k,
// gathered from the slope adjoints of the node and its neighbours.  Outputs
// on the tile: the adjoint of T^t (lT^{t+1} plus the four gT_k) and the
// rho, grad rho, v and div v parts of the four stages.
constexpr int TAH = 7;
constexpr int TAX = 64 - 2 * TAH;

template <typename S, int TAY, int TAW>
__global__ __launch_bounds__(64 * TAW) void a_theradj(const AdjInst *__restrict__ ai, const int *__restrict__ tmap,
                                                      int cur)
{
    constexpr int H = TAY + 2 * TAH;          // region rows
    constexpr int RPW = (H + TAW - 1) / TAW;  // region rows per wave
    // planes 0..3: T_1..T_4; 4: lT^{t+1}; 5: g_2.  g_1 reuses plane 3 once
    // T_4 is dead, g_0 plane 2 once T_3 is.  The planes hold the storage
    // precision (the forward stages of an FP32 lattice run in FP32 too); the
    // arithmetic is FP64.  In FP32 they take half the LDS, which leaves room
    // for taller tiles.
    using LT = S;
    __shared__ LT sb[6][H][64];
    __shared__ LT sAX[H][64], sAY[H][64];
    __shared__ double s_rho_ave;
    const AdjInst &I = ai[tmap[blockIdx.x]];
    const DevParams P = I.P;
    const AdjWG<S> &w = reinterpret_cast<const AdjWG<S> &>(I.w);
    const int q = (int)blockIdx.x - I.tblk0;
    const int x0 = (q % I.tgx) * TAX, y0 = (q / I.tgx) * TAY;
    static_assert(RPW * TAW >= H, "every region row has a wave");
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gx = wrapi(x0 + lane - TAH, P.nx);
    const gmem<double> *__restrict__ lT1 = gp(I.lT[cur]);
    gmem<double> *__restrict__ lT0 = gp(I.lT[cur ^ 1]);
    const double chi = P.chi;

    // region row r of this wave's m-th slot: lattice row, in lattice, interior
    int gyr[RPW];
    bool inl[RPW], inr[RPW];
#pragma unroll
    for (int m = 0; m < RPW; ++m) {
        const int r = wv + TAW * m;
        const int gy = y0 + r - TAH;
        gyr[m] = gy;
        inl[m] = r < H && gy >= 0 && gy < P.ny;
        inr[m] = inl[m] && gy > 0 && gy < P.ny - 1;
    }

    // rho_ave of the stored state (Eq. (9)): every block sums the lattice's
    // mass partials in the same fixed order
    if (wv == 0) {
        double sm = 0.0;
        for (int k = lane; k < I.nb; k += 64) sm += w.mpart[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sm += __shfl_xor(sm, off, 64);
        if (lane == 0) s_rho_ave = sm / ((double)P.nx * (double)P.ny);
    }
    __syncthreads();
    const double rho_ave = s_rho_ave;

    // force and velocity of the stored state on the region: v into planes 1
    // and 2 (free until the first forward stage), grad rho into the
    // coefficient planes; the tile's own nodes also write the per-node
    // fields the LB adjoint reads
    const bool tile_col = lane >= TAH && lane < TAH + TAX;
#pragma unroll
    for (int m = 0; m < RPW; ++m) {
        const int r = wv + TAW * m;
        if (r >= H) continue;
        NodeForce o;
        o.vx = o.vy = o.rx = o.ry = 0.0;
        if (inl[m]) {
            const size_t c = (size_t)gyr[m] * P.nx + gx;
            o = force_node(P, w, gx, gyr[m], c, rho_ave);
            if (r >= TAH && r < TAH + TAY && tile_col && x0 + lane - TAH < P.nx) {
                w.sx[c] = o.sx;
                w.sy[c] = o.sy;
                w.Fx[c] = o.Fx;
                w.Fy[c] = o.Fy;
                w.vx[c] = o.vx;
                w.vy[c] = o.vy;
            }
        }
        sb[1][r][lane] = o.vx;
        sb[2][r][lane] = o.vy;
        sAX[r][lane] = o.rx;
        sAY[r][lane] = o.ry;
    }
    __syncthreads();

    // coefficients of K at the region nodes one node in from its edge (the
    // only ones any stage reads)
    double cdv[RPW], cIA[RPW], cIB[RPW], cE1[RPW], cE2[RPW];
#pragma unroll
    for (int m = 0; m < RPW; ++m) {
        const int r = wv + TAW * m;
        double t1 = 0.0, ax = 0.0, ay = 0.0, l1 = 0.0;
        cdv[m] = cIA[m] = cIB[m] = cE1[m] = cE2[m] = 0.0;
        if (inl[m]) {
            const size_t c = (size_t)gyr[m] * P.nx + gx;
            t1 = w.T1[c];
            l1 = lT1[c];
            if (inr[m] && r >= 1 && r < H - 1 && lane >= 1 && lane < 63) {
                const double rho = w.rho[c];
                const DivCoef k = div_coef(P, sb[1], sb[2], r, lane, gyr[m], sb[1][r][lane], sb[2][r][lane],
                                           sAX[r][lane], sAY[r][lane], rho);
                ax = k.ax;
                ay = k.ay;
                cdv[m] = k.dv;
                cIA[m] = k.IA;
                cIB[m] = k.IB;
                if (r >= TAH && r < TAH + TAY) {
                    double ri;
                    pw_derivs(P, rho, ri, cE1[m], cE2[m]);
                }
            }
        }
        // each node reads only its own grad rho entry before replacing it
        // with the advection coefficient; the neighbours' reads above go to
        // the velocity planes
        if (r < H) {
            sb[0][r][lane] = t1;
            sb[4][r][lane] = l1;
            sAX[r][lane] = ax;
            sAY[r][lane] = ay;
        }
    }
    __syncthreads();

    // forward stages: T_{s+1} = T_1 + c_s K(T_s) on the region shrunk by s
#pragma unroll
    for (int s = 1; s <= 3; ++s) {
        const double cs = s == 3 ? 1.0 : 0.5;
#pragma unroll
        for (int m = 0; m < RPW; ++m) {
            const int r = wv + TAW * m;
            if (r < s || r >= H - s) continue;
            // the gradient and Laplacian stencils from column sums shifted
            // between lanes, as in the forward thermal step
            const LT(*F)[64] = sb[s - 1];
            const double tc = F[r][lane], tN = F[r + 1][lane], tS = F[r - 1][lane];
            const double cv = (tN + tS) + 4.0 * tc, cw = tN - tS;
            const double vW = lane_from_left(cv), vE = lane_from_right(cv);
            const double wW = lane_from_left(cw), wE = lane_from_right(cw);
            if (lane < s || lane >= 64 - s) continue;
            double v = sb[0][r][lane];
            if (inr[m]) {
                const int l = lane;
                const double dTx = (vE - vW) * (1.0 / 12.0);
                const double dTy = (wW + wE + 4.0 * cw) * (1.0 / 12.0);
                const double lap = (vW + vE + 4.0 * cv - 36.0 * tc) * (1.0 / 6.0);
                double d1, d2;
                phi_derivs(P, tc, d1, d2);
                const double h = sAX[r][l] * dTx + sAY[r][l] * dTy + chi * lap - cIA[m] * cdv[m] * tc +
                                 cIB[m] * cdv[m] * tc * d1;
                v += cs * h;
            }
            sb[s][r][lane] = v;
        }
        __syncthreads();
    }

    // reverse stages k = 3..0 on the region shrunk by 7 - k
    double lt[RPW], acc[RPW][5];
#pragma unroll
    for (int m = 0; m < RPW; ++m) {
        lt[m] = 0.0;
#pragma unroll
        for (int j = 0; j < 5; ++j) acc[m][j] = 0.0;
    }
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        const int R = 7 - k;
        // slope adjoint of stage k at region nodes: plane and scale
        const int gp = k == 3 ? 4 : (k == 2 ? 5 : (k == 1 ? 3 : 2));
        const double gs = k == 3 ? 1.0 / 6.0 : 1.0;
        const int op = k == 3 ? 5 : (k == 2 ? 3 : 2);  // plane of the next slope adjoint
        const double ck = k == 3 ? 1.0 : 0.5;
        const double wk = (k == 1) ? 1.0 : 2.0;        // RK4 weight of slope k-1
        double gnext[RPW];
#pragma unroll
        for (int m = 0; m < RPW; ++m) {
            const int r = wv + TAW * m;
            gnext[m] = 0.0;
            if (r < R || r >= H - R || lane < R || lane >= 64 - R || !inl[m]) continue;
            const LT(*G)[64] = sb[gp];
            const int l = lane;
            double gT = 0.0;
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                const int rp = r - kEY[a], lp = l - kEX[a];
                const int gyp = gyr[m] - kEY[a];
                const double mk = (gyp > 0 && gyp < P.ny - 1) ? gs : 0.0;
                gT += mk * (double)G[rp][lp] *
                      (3.0 * kW[a] * ((double)sAX[rp][lp] * kEX[a] + (double)sAY[rp][lp] * kEY[a]) + 6.0 * kW[a] * chi);
            }
            if (inr[m]) {
                const double g = gs * G[r][l];
                const LT(*F)[64] = sb[k];
                const double Tv = F[r][l];
                double d1, d2;
                phi_derivs(P, Tv, d1, d2);
                gT += g * (-(10.0 / 3.0) * chi - cdv[m] * (cIA[m] - cIB[m] * (d1 + Tv * d2)));
                if (k > 0) gnext[m] = wk * sb[4][r][l] * (1.0 / 6.0) + ck * gT;
                const bool tile_row = r >= TAH && r < TAH + TAY;
                if (tile_row && tile_col) {
                    // this stage's part of the rho, grad rho, v, div v adjoints at the node
                    const double tE = F[r][l + 1], tW = F[r][l - 1], tN = F[r + 1][l], tS = F[r - 1][l];
                    const double tNE = F[r + 1][l + 1], tNW = F[r + 1][l - 1];
                    const double tSE = F[r - 1][l + 1], tSW = F[r - 1][l - 1];
                    const double dTx = (tE - tW) * (1.0 / 3.0) + (tNE - tNW + tSE - tSW) * (1.0 / 12.0);
                    const double dTy = (tN - tS) * (1.0 / 3.0) + (tNE + tNW - tSE - tSW) * (1.0 / 12.0);
                    acc[m][0] += g * dTx;       // chi RI applied at the end
                    acc[m][1] += g * dTy;
                    acc[m][2] += g * Tv;        // div v part: -g T (IA - IB d1)
                    acc[m][3] += g * Tv * d1;
                    acc[m][4] += g * Tv * (cE1[m] - cE2[m] * d1);
                }
            }
            lt[m] += gT;
        }
        if (k == 0) break;
        // plane op is read by no stage-k node (stage k reads planes gp, k and
        // 4), and its earlier contents (T_4 for k = 2, T_3 for k = 1) were last
        // read before the previous stage's closing barrier: the writes need no
        // barrier of their own before them
#pragma unroll
        for (int m = 0; m < RPW; ++m) {
            const int r = wv + TAW * m;
            if (r < R || r >= H - R || lane < R || lane >= 64 - R) continue;
            sb[op][r][lane] = gnext[m];
        }
        __syncthreads();
    }

    // outputs on the tile
#pragma unroll
    for (int m = 0; m < RPW; ++m) {
        const int r = wv + TAW * m;
        if (r < TAH || r >= TAH + TAY || !tile_col || !inl[m] || x0 + lane - TAH >= P.nx) continue;
        const size_t c = (size_t)gyr[m] * P.nx + gx;
        lT0[c] = lT1[c] + lt[m];
        double aDrx = 0.0, aDry = 0.0, avx = 0.0, avy = 0.0, adiv = 0.0, arho = 0.0;
        if (inr[m]) {
            double ri, e1, e2;
            pw_derivs(P, w.rho[c], ri, e1, e2);
            // grad rho is constant over the stages: its part of the rho
            // adjoint is grad rho . (sum of g grad T), formed here
            double rx, ry;
            grad_rho(P, w, gx, gyr[m], rx, ry);
            aDrx = chi * ri * acc[m][0];
            aDry = chi * ri * acc[m][1];
            avx = -acc[m][0];
            avy = -acc[m][1];
            adiv = -(cIA[m] * acc[m][2] - cIB[m] * acc[m][3]);
            arho = -chi * ri * ri * (rx * acc[m][0] + ry * acc[m][1]) - cdv[m] * acc[m][4];
        }
        w.gDrx[c] = aDrx;
        w.gDry[c] = aDry;
        w.gvx[c] = avx;
        w.gvy[c] = avy;
        w.gdiv[c] = adiv;
        w.grho[c] = arho;
    }
}

// Stencil transposes of grad rho and div v, then streaming and collision
// transposed at node c; writes the adjoint of the completed populations
// (before the density and completion parts), and the per-node force adjoints.
template <typename S>
__global__ __launch_bounds__(NTA) void a_lb(A_ARGS, int k, int cur)
{
    __shared__ double red[NTA / 64];
    A_INST
    A_NODE
    const gmem<S> *__restrict__ f = a_slot<S>(I, k);
    const gmem<S> *__restrict__ lf1 = gp(static_cast<const S *>(I.lf[cur]));
    const gmem<double> *__restrict__ gr1 = gp(I.gr[cur]);
    gmem<S> *__restrict__ lf0 = gp(static_cast<S *>(I.lf[cur ^ 1]));
    double pr = 0.0, pg = 0.0;
    if (on) {
        const bool in = a_int(P, gj);
        // grad rho and div v of the temperature equation transposed (only
        // interior nodes carry them; the velocity it sees is zero on walls)
        double gr = w.grho[c], gvx = 0.0, gvy = 0.0;
        {
            double tr = 0.0, tu = 0.0, tv = 0.0;
#pragma unroll
            for (int a = 1; a < 9; ++a) {
                bool ok;
                const size_t cp = a_src(P, gi, gj, a, c, ok);
                const double m = ok ? 3.0 * kW[a] : 0.0;
                tr += m * (kEX[a] * (double)w.gDrx[cp] + kEY[a] * (double)w.gDry[cp]);
                const double gd = w.gdiv[cp];
                tu += m * kEX[a] * gd;
                tv += m * kEY[a] * gd;
            }
            gr += tr;
            if (in) {
                gvx = w.gvx[c] + tu;
                gvy = w.gvy[c] + tv;
            }
        }
        // push streaming transposed: f'(c + e_a, a) = f*(c, a)
        double gfs[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) {
            const int jj = gj + kEY[a];
            const bool ok = jj >= 0 && jj < P.ny;
            // interior nodes keep their density adjoint apart (added here);
            // wall nodes hold the complete adjoint (Zou-He transposed)
            const size_t ct = ok ? a_at(P, gi, gj, kEX[a], kEY[a]) : c;
            const double v = (double)lf1[(size_t)a * N + ct] + (a_int(P, jj) ? gr1[ct] : 0.0);
            gfs[a] = ok ? v : 0.0;
        }
        double fl[9];
        load_node(P, f, N, c, gj, fl);
        const double r = w.rho[c], vx = w.vx[c], vy = w.vy[c], Fx = w.Fx[c], Fy = w.Fy[c];
        // moments of f and the equilibrium (Eq. (5)), forcing (Eq. (8))
        const double s14 = fl[1] + fl[2] + fl[3] + fl[4], s58 = fl[5] + fl[6] + fl[7] + fl[8];
        double m[9];
        m[0] = r;
        m[1] = -4.0 * fl[0] - s14 + 2.0 * s58;
        m[2] = 4.0 * fl[0] - 2.0 * s14 + s58;
        m[3] = w.jx[c];
        m[4] = -2.0 * fl[1] + 2.0 * fl[3] + fl[5] - fl[6] - fl[7] + fl[8];
        m[5] = w.jy[c];
        m[6] = -2.0 * fl[2] + 2.0 * fl[4] + fl[5] + fl[6] - fl[7] - fl[8];
        m[7] = fl[1] - fl[2] + fl[3] - fl[4];
        m[8] = fl[5] - fl[6] + fl[7] - fl[8];
        const double v2 = vx * vx + vy * vy;
        const double meq7 = r * (vx * vx - vy * vy), meq8 = r * vx * vy;
        const double S7 = 2.0 * (vx * Fx - vy * Fy), S8 = vx * Fy + vy * Fx;
        const double tau = P.tau_V + (r - P.rho_V) * P.tau_slope, s_nu = rcp_nr(tau);
        const double L[9] = {P.s_rho, P.s_e, P.s_zeta, P.s_j, P.s_q, P.s_j, P.s_q, s_nu, s_nu};
        // f* = M^T diag(1/n) m*  ->  gm* = diag(1/n) M gf*
        double gms[9];
        {
            const double g14 = gfs[1] + gfs[2] + gfs[3] + gfs[4], g58 = gfs[5] + gfs[6] + gfs[7] + gfs[8];
            double a0 = 0.0;
            for (int a = 0; a < 9; ++a) a0 += gfs[a];
            gms[0] = a0 * (1.0 / 9.0);
            gms[1] = (-4.0 * gfs[0] - g14 + 2.0 * g58) * (1.0 / 36.0);
            gms[2] = (4.0 * gfs[0] - 2.0 * g14 + g58) * (1.0 / 36.0);
            gms[3] = (gfs[1] - gfs[3] + gfs[5] - gfs[6] - gfs[7] + gfs[8]) * (1.0 / 6.0);
            gms[4] = (-2.0 * gfs[1] + 2.0 * gfs[3] + gfs[5] - gfs[6] - gfs[7] + gfs[8]) * (1.0 / 12.0);
            gms[5] = (gfs[2] - gfs[4] + gfs[5] + gfs[6] - gfs[7] - gfs[8]) * (1.0 / 6.0);
            gms[6] = (-2.0 * gfs[2] + 2.0 * gfs[4] + gfs[5] + gfs[6] - gfs[7] - gfs[8]) * (1.0 / 12.0);
            gms[7] = (gfs[1] - gfs[2] + gfs[3] - gfs[4]) * 0.25;
            gms[8] = (gfs[5] - gfs[6] + gfs[7] - gfs[8]) * 0.25;
        }
        // m* = m - L (m - m_eq) + (1 - L/2) S
        double gm[9], gq[9], gS[9];
        for (int k = 0; k < 9; ++k) {
            gm[k] = (1.0 - L[k]) * gms[k];
            gq[k] = L[k] * gms[k];
            gS[k] = (1.0 - 0.5 * L[k]) * gms[k];
        }
        const double gsnu = gms[7] * (-(m[7] - meq7) - 0.5 * S7) + gms[8] * (-(m[8] - meq8) - 0.5 * S8);
        // m = M f  ->  gf += M^T gm
        double gf[9];
        gf[0] = gm[0] - 4.0 * gm[1] + 4.0 * gm[2];
        gf[1] = gm[0] - gm[1] - 2.0 * gm[2] + gm[3] - 2.0 * gm[4] + gm[7];
        gf[2] = gm[0] - gm[1] - 2.0 * gm[2] + gm[5] - 2.0 * gm[6] - gm[7];
        gf[3] = gm[0] - gm[1] - 2.0 * gm[2] - gm[3] + 2.0 * gm[4] + gm[7];
        gf[4] = gm[0] - gm[1] - 2.0 * gm[2] - gm[5] + 2.0 * gm[6] - gm[7];
        gf[5] = gm[0] + 2.0 * gm[1] + gm[2] + gm[3] + gm[4] + gm[5] + gm[6] + gm[8];
        gf[6] = gm[0] + 2.0 * gm[1] + gm[2] - gm[3] - gm[4] + gm[5] + gm[6] - gm[8];
        gf[7] = gm[0] + 2.0 * gm[1] + gm[2] - gm[3] - gm[4] - gm[5] - gm[6] + gm[8];
        gf[8] = gm[0] + 2.0 * gm[1] + gm[2] + gm[3] + gm[4] - gm[5] - gm[6] - gm[8];
        // m_eq(rho, v) of Eq. (5)
        gr += gq[0] + gq[1] * (-2.0 + 3.0 * v2) + gq[2] * (1.0 - 3.0 * v2) + gq[3] * vx - gq[4] * vx +
              gq[5] * vy - gq[6] * vy + gq[7] * (vx * vx - vy * vy) + gq[8] * vx * vy;
        gvx += r * (6.0 * vx * (gq[1] - gq[2]) + gq[3] - gq[4] + 2.0 * vx * gq[7] + vy * gq[8]);
        gvy += r * (6.0 * vy * (gq[1] - gq[2]) + gq[5] - gq[6] - 2.0 * vy * gq[7] + vx * gq[8]);
        // S(v, F, Q) of Eq. (8)
        const double a6 = gS[1] - gS[2];
        double gFx = 6.0 * a6 * vx + gS[3] - gS[4] + 2.0 * vx * gS[7] + vy * gS[8];
        double gFy = 6.0 * a6 * vy + gS[5] - gS[6] - 2.0 * vy * gS[7] + vx * gS[8];
        gvx += 6.0 * a6 * Fx + 2.0 * Fx * gS[7] + Fy * gS[8];
        gvy += 6.0 * a6 * Fy - 2.0 * Fy * gS[7] + Fx * gS[8];
        const double gQ = P.sig_e * gS[1] - P.sig_z * gS[2];
        // s_nu = 1 / tau(rho)
        gr += gsnu * (-P.tau_slope * s_nu * s_nu);
        // v = (j + F/2)/rho
        const double ir = rcp_nr(r);
        const double gjx = gvx * ir, gjy = gvy * ir;
        gFx += 0.5 * gvx * ir;
        gFy += 0.5 * gvy * ir;
        gr += -(gvx * vx + gvy * vy) * ir;
        for (int a = 0; a < 9; ++a) lf0[(size_t)a * N + c] = S(gf[a] + kEX[a] * gjx + kEY[a] * gjy);
        // per-node force parts (no force on the wall rows)
        double gpsi = 0.0, gsx = 0.0, gsy = 0.0;
        if (in) {
            const double ps = w.psi[c];
            gr += -P.g * gFy;
            pr = P.g * gFy;
            if (gj == 1) {
                gpsi += gFy * P.Gw_bottom * ps / 3.0;
                pg = gFy * ps * ps / 6.0;
            }
            if (gj == P.ny - 2) gpsi += -gFy * P.Gw_top * ps / 3.0;
            gpsi += -P.G * (w.sx[c] * gFx + w.sy[c] * gFy);
            gsx = -P.G * ps * gFx + 2.0 * P.G * P.G * w.sx[c] * gQ;
            gsy = -P.G * ps * gFy + 2.0 * P.G * P.G * w.sy[c] * gQ;
        }
        w.grho[c] = gr;
        w.gpsi[c] = gpsi;
        w.gsx[c] = gsx;
        w.gsy[c] = gsy;
    }
    const double sr = block_sum<NTA>(pr, red);
    __syncthreads();
    const double sg = block_sum<NTA>(pg, red);
    if (threadIdx.x == 0) {
        w.fpart[2 * q] = sr;
        w.fpart[2 * q + 1] = sg;
    }
}

// Heat-flux sample q = -(c_v chi / nx) sum_i rho(i,0) (-3 T0 + 4 T1 - T2)/2
// of a stored state, transposed with weight wq, at node (gi, gj) of rows
// 0..2: the population part (row 0, Zou-He folded) and the temperature part.
template <typename S>
__device__ __forceinline__ void hf_source(const DevParams &P, const gmem<S> *__restrict__ f,
                                          const gmem<S> *__restrict__ T, double wq, size_t N, int gi, int gj,
                                          double gpop[9], double &gtem)
{
    const double k = -P.cv_chi / P.nx * wq;
    for (int a = 0; a < 9; ++a) gpop[a] = 0.0;
    gtem = 0.0;
    if (gj > 2) return;
    double fl[9];
    load_node(P, f, N, (size_t)gi, 0, fl);
    double r0 = 0.0;
    for (int a = 0; a < 9; ++a) r0 += fl[a];
    if (gj == 0) {
        const double t0 = (double)T[gi], t1 = (double)T[P.nx + gi], t2 = (double)T[2 * P.nx + gi];
        for (int a = 0; a < 9; ++a) gpop[a] = k * (-3.0 * t0 + 4.0 * t1 - t2) / 2.0;
        zou_he_T(gpop, 1);
    }
    gtem = k * r0 * (gj == 0 ? -1.5 : (gj == 1 ? 2.0 : -0.5));
}

// Interaction-force stencil transposed (gather of s over the neighbours),
// EOS transposed, rho = sum f, Zou-He completion transposed; the heat-flux
// source of state t (when it is a sample, wq > 0), and rho, j, psi of the
// state before (fp, Tp when given) with its mass partials.
template <typename S>
__global__ __launch_bounds__(NTA) void a_final(A_ARGS, int k, int cur, double wq, int prev)
{
    __shared__ double red[NTA / 64 + 1];
    A_INST
    const double sr = block_sum_all(w.fpart, I.nb, 2, 0, red);
    if (q == 0) {
        const double sg = block_sum_all(w.fpart, I.nb, 2, 1, red);
        if (threadIdx.x == 0) w.scal[2] += sg;
    }
    A_NODE
    const gmem<S> *__restrict__ f = a_slot<S>(I, k);
    const gmem<S> *__restrict__ T = f + 9 * N;
    const gmem<S> *__restrict__ fp = prev ? a_slot<S>(I, k - 1) : nullptr;
    const gmem<S> *__restrict__ Tp = prev ? fp + 9 * N : nullptr;
    gmem<S> *__restrict__ lf0 = gp(static_cast<S *>(I.lf[cur ^ 1]));
    gmem<double> *__restrict__ lT0 = gp(I.lT[cur ^ 1]);
    double m = 0.0;
    if (on) {
        double gpsi = w.gpsi[c];
#pragma unroll
        for (int a = 1; a < 9; ++a) {
            bool ok;
            const size_t cp = a_src(P, gi, gj, a, c, ok);
            const double m = ok ? kWpsi[a] : 0.0;
            gpsi += m * (kEX[a] * (double)w.gsx[cp] + kEY[a] * (double)w.gsy[cp]);
        }
        double gr = w.grho[c] + sr / ((double)P.nx * (double)P.ny);
        double gT = 0.0;
        if (gpsi != 0.0) {
            const double r = w.rho[c], Tv = w.T1[c];
            double dpdr, dpdT;
            eos_derivs(P, r, Tv, dpdr, dpdT);
            const double gq = gpsi * 0.5 * rcp_nr(w.psi[c]) * P.two_over_G;
            gr += gq * (dpdr - 1.0 / 3.0);
            gT = gq * dpdT;
        }
        double gpop[9], gtem = 0.0;
        if (wq != 0.0 && gj <= 2) hf_source<S>(P, f, T, wq, N, gi, gj, gpop, gtem);
        if (a_int(P, gj)) {
            // rho = sum f: the density adjoint joins every population of the
            // node; kept apart and added where the next step gathers lf
            gp(I.gr[cur ^ 1])[c] = gr;
        } else {
            double g[9];
            for (int a = 0; a < 9; ++a) g[a] = (double)lf0[(size_t)a * N + c] + gr;
            zou_he_T(g, gj == 0);
            if (wq != 0.0 && gj == 0)
                for (int a = 0; a < 9; ++a) g[a] += gpop[a];
            for (int a = 0; a < 9; ++a) lf0[(size_t)a * N + c] = S(g[a]);
        }
        lT0[c] += gT + gtem;
        // this thread's reads of the state-t values at c are done
        if (fp) m = a_macro_node<S>(P, fp, Tp, N, c, gj, w);
    }
    if (prev) {
        const double s = block_sum<NTA>(m, red);
        if (threadIdx.x == 0) w.mpart[q] = s;
    }
}

// T of a state copied into the T part of each of `slots` stored states
// (layout per state: 9 population planes, then T), so that every slot holds
// the Dirichlet wall rows the thermal launch does not rewrite.
template <typename S>
__global__ void a_bcast_T(const S *__restrict__ T, S *__restrict__ seg, size_t n, int slots)
{
    const size_t total = n * (size_t)slots;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
        const size_t s = k / n, c = k - s * n;
        seg[s * 10 * n + 9 * n + c] = T[c];
    }
}

// The heat-flux sample of stored state k transposed, weight wq, added to the
// adjoint [cur] of that state (nodes of rows 0..2 act).
template <typename S>
__global__ __launch_bounds__(NTA) void a_hf(A_ARGS, int k, double wq, int cur)
{
    A_INST
    A_NODE
    if (!on || gj > 2) return;
    const gmem<S> *f = a_slot<S>(I, k);
    double gpop[9], gtem;
    hf_source<S>(P, f, f + 9 * N, wq, N, gi, gj, gpop, gtem);
    if (gj == 0) {
        gmem<S> *lf = gp(static_cast<S *>(I.lf[cur]));
        for (int a = 0; a < 9; ++a) lf[(size_t)a * N + c] = S((double)lf[(size_t)a * N + c] + gpop[a]);
    }
    gp(I.lT[cur])[c] += gtem;
}

}  // namespace lbb
