// kernels.hip -- CDNA4 (gfx950) kernels and the C ABI of libbmhd.so.
//
// Hot path per stage (the GPU solver's block sweep, Algorithm 2, redesigned for MI355X):
//   k_halo_fill   ghost layers of faces that border another level (restriction / prolongation,
//                 Sec. 4.2), only on grids with two levels;
//   k_stage_wp    (default) one workgroup per slab of a block (8 x 8 x KS cells), one wavefront per
//   / k_stage     cell layer plus one (or, k_stage, one thread per face). It gathers the slab and its
//                 2-deep face halos from HBM straight into LDS as primitive variables (same-level
//                 neighbours are read in place: no separate ghost-fill pass), computes every face flux
//                 once (MC-limited reconstruction, Rusanov or HLLE), hands each flux to the cells on
//                 both sides (cross-lane permutes and LDS), adds the Powell source (Eqs. 2-4) and
//                 writes the stage result. The second stage also folds in the next time-step bound
//                 (wave-level max, one filtered 64-bit atomic per workgroup) and the positivity check;
//   k_flux_correct coarse cells next to a coarse-fine face swap their coarse flux for the mean of the
//                 four fine fluxes (FP64 in every precision form);
//   k_dt_finalize dt = CFL / max bound per simulation.
// Under local time stepping (steady-state sessions, Sec. 5.2) the first stage forms each cell's own CFL
// step from its FP64 stage input and stores it; the second stage and k_flux_correct read it.
// Between steps: k_remap moves a state onto an adapted grid (copy, prolongation, restriction).
// Workgroups are mapped XCD-aware: consecutive workgroup ids go to different XCDs, so each XCD is
// handed a contiguous run of the Morton-ordered block schedule and neighbouring blocks share an L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>

#include "bmhd_internal.h"

namespace bmhd {

constexpr double GAMMA = 5.0 / 3.0;

// ------------------------------------------------------------------------------------------------
// small device helpers

template <typename R>
__device__ __forceinline__ R rmin(R a, R b) { return fmin(a, b); }
template <typename R>
__device__ __forceinline__ R rmax(R a, R b) { return fmax(a, b); }

// Reciprocal and square root from the hardware approximations (about 26 correct bits) refined by
// Newton steps: two steps for 1/x, two corrections for sqrt. Inputs are positive normal numbers
// (densities, squared wave speeds, signal-speed spans); sqrt(0) returns 0.
__device__ __forceinline__ double frcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float frcp(float x) {
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double fsqrt(double x) {
    const double r = __builtin_amdgcn_rsq(fmax(x, 1e-300));
    double g = x * r, h = 0.5 * r;
    const double t = fma(-g, h, 0.5);
    g = fma(g, t, g);
    h = fma(h, t, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
}
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// One-step refinements for the face fluxes, measured on gfx950 over random positive inputs: 1/x within
// 11 ulp (hardware reciprocal plus one Newton step), sqrt within 35 ulp (hardware reciprocal square root
// plus one Goldschmidt step). Wave speeds and the HLLE weights carry these errors into the fluxes
// (relative 1e-14 at most), far inside the 1e-12 bound; dt and the primitive conversion keep the
// two-step forms above.
__device__ __forceinline__ double frcp1(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float frcp1(float x) { return frcp(x); }
__device__ __forceinline__ double fsqrt1(double x) {
    const double r = __builtin_amdgcn_rsq(fmax(x, 1e-300));
    const double g = x * r, h = 0.5 * r;
    return fma(g, fma(-g, h, 0.5), g);
}
__device__ __forceinline__ float fsqrt1(float x) { return fsqrt(x); }

// conserved -> primitive in FP64 (u = m / rho, p from the total energy of Eq. 5)
__device__ __forceinline__ void cons_to_prim(const double u[8], double w[8]) {
    const double rho = u[0];
    const double ir = frcp(rho);
    const double ux = u[1] * ir, uy = u[2] * ir, uz = u[3] * ir;
    const double ke = u[1] * ux + u[2] * uy + u[3] * uz;
    const double b2 = u[4] * u[4] + u[5] * u[5] + u[6] * u[6];
    w[0] = rho;
    w[1] = ux;
    w[2] = uy;
    w[3] = uz;
    w[4] = u[4];
    w[5] = u[5];
    w[6] = u[6];
    w[7] = (GAMMA - 1.0) * (u[7] - 0.5 * ke - 0.5 * b2);
}

// fast magnetosonic speed along axis D (largest root of the ideal-MHD dispersion relation)
template <typename R, int D, bool FACE = false>
__device__ __forceinline__ R fast_speed(const R w[8], R ir) {
    const R a2 = R(GAMMA) * w[7] * ir;
    const R bx = w[4], by = w[5], bz = w[6];
    const R b2 = (bx * bx + by * by + bz * bz) * ir;
    const R bn = w[4 + D];
    const R bn2 = bn * bn * ir;
    const R s = a2 + b2;
    R disc = s * s - R(4) * a2 * bn2;
    disc = rmax(disc, R(0));
    if constexpr (FACE) return fsqrt1(R(0.5) * (s + fsqrt1(disc)));
    return fsqrt(R(0.5) * (s + fsqrt(disc)));
}

// conserved state, physical flux along D, normal velocity and fast speed of one face state
template <typename R, int D>
__device__ __forceinline__ void face_side(const R w[8], R U[8], R F[8], R &un, R &cf) {
    const R rho = w[0], ux = w[1], uy = w[2], uz = w[3], bx = w[4], by = w[5], bz = w[6], p = w[7];
    const R u2 = ux * ux + uy * uy + uz * uz;
    const R b2 = bx * bx + by * by + bz * bz;
    const R ub = ux * bx + uy * by + uz * bz;
    const R pb = R(0.5) * b2;
    const R ptot = p + pb;
    const R e = p * R(1.5) + R(0.5) * rho * u2 + pb;
    un = w[1 + D];
    const R bn = w[4 + D];
    const R mn = rho * un;
    U[0] = rho;
    U[1] = rho * ux;
    U[2] = rho * uy;
    U[3] = rho * uz;
    U[4] = bx;
    U[5] = by;
    U[6] = bz;
    U[7] = e;
    F[0] = mn;
    F[1] = mn * ux - bx * bn;
    F[2] = mn * uy - by * bn;
    F[3] = mn * uz - bz * bn;
    F[1 + D] += ptot;
    F[4] = un * bx - bn * ux;
    F[5] = un * by - bn * uy;
    F[6] = un * bz - bn * uz;
    F[4 + D] = R(0);
    F[7] = un * (e + ptot) - bn * ub;
    const R ir = frcp1(rho);
    cf = fast_speed<R, D, true>(w, ir);
}

template <typename R, int D, int FLUX>
__device__ __forceinline__ void num_flux(const R wl[8], const R wr[8], R f[8]) {
    // Linde-type flux: the entropy wave's density jump (the part no pressure change explains, bounded by
    // the jump) and the mean velocity, formed before the face states' fluxes so that only these four
    // values stay live through them
    R delta = R(0), ub[3] = {R(0), R(0), R(0)};
    if constexpr (FLUX == BMHD_FLUX_LINDE) {
        const R drho = wr[0] - wl[0], dp = wr[7] - wl[7];
        const R c2 = R(GAMMA) * (wl[7] + wr[7]) * frcp1(wl[0] + wr[0]);
        const R t = drho - dp * frcp1(c2);
        delta = (t > R(0) && drho > R(0)) ? rmin(t, drho) : ((t < R(0) && drho < R(0)) ? rmax(t, drho) : R(0));
#pragma unroll
        for (int a = 0; a < 3; ++a) ub[a] = R(0.5) * (wl[1 + a] + wr[1 + a]);
    }
    R UL[8], FL[8], UR[8], FR[8], unl, cl, unr, cr;
    face_side<R, D>(wl, UL, FL, unl, cl);
    face_side<R, D>(wr, UR, FR, unr, cr);
    if constexpr (FLUX == BMHD_FLUX_RUSANOV) {
        const R cmax = rmax(fabs(unl) + cl, fabs(unr) + cr);
#pragma unroll
        for (int v = 0; v < 8; ++v) f[v] = R(0.5) * (FL[v] + FR[v]) - R(0.5) * cmax * (UR[v] - UL[v]);
    } else {
        // with sl' = min(sl, 0) and sr' = max(sr, 0) the single formula covers the three cases
        const R sl = rmin(rmin(unl - cl, unr - cr), R(0));
        const R sr = rmax(rmax(unl + cl, unr + cr), R(0));
        const R inv = frcp1(sr - sl);
        const R a = sr * inv, b = -sl * inv, c = sl * a;
#pragma unroll
        for (int v = 0; v < 8; ++v) f[v] = fma(a, FL[v], fma(b, FR[v], c * (UR[v] - UL[v])));
        if constexpr (FLUX == BMHD_FLUX_LINDE) {
            // anti-diffusion of the entropy (contact) wave: its jump carried at the mean velocity,
            // upwinded at the contact speed
            const R lam = rmin(rmax(ub[D], sl), sr);
            const R k = (sl * rmax(lam, R(0)) + sr * rmin(lam, R(0)) - sl * sr) * inv * delta;
            f[0] += k;
            f[1] += k * ub[0];
            f[2] += k * ub[1];
            f[3] += k * ub[2];
            f[7] += k * (R(0.5) * (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]));
        }
    }
}

// Half of the monotonized-central limited slope, minmod(2 dm, (dm + dp) / 2, 2 dp) / 2, from the two
// one-sided differences. With s = sign(dm + dp) it is s * max(0, min(|dm + dp| / 4, s dm, s dp)): the
// same value bit for bit (every scaling is by a power of two), without branches.
template <typename R>
__device__ __forceinline__ R mc_half(R dm, R dp) {
    const R c = dm + dp;
    const R s = copysign(R(1), c);
    const R q = rmax(R(0), rmin(rmin(R(0.25) * fabs(c), s * dm), s * dp));
    return s * q;
}

// body membership of a cell from its centre (no contraction: must agree bit for bit everywhere)
__device__ __noinline__ bool in_body(const DevSim &S, int level, const int32_t ijk[3], int i, int j, int k) {
#pragma clang fp contract(off)
    if (!(S.body_r > 0.0)) return false;
    const double dx = S.dx0 / double(1 << level);
    const int idx[3] = {i, j, k};
    double r2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long G = (long long)ijk[a] * 8 + idx[a];
        const double x = S.origin[a] + (double(G) + 0.5) * dx;
        const double t = x - S.body_c[a];
        r2 = r2 + t * t;
    }
    return r2 < S.body_r * S.body_r;
}

// ------------------------------------------------------------------------------------------------
// generic ghost-value rules (Sec. 4.2) on global cell indices; used by the halo and full ghost fills.
// Evaluated without contraction so that copy, restriction and prolongation are reproducible bit for bit.

struct Cursor {
    const Tables *T;
    const double *U;
    size_t vs;  // variable stride = nb * 512
};

__device__ __forceinline__ int32_t lut_at(const Tables &T, const DevSim &S, int l, long long bx, long long by,
                                          long long bz) {
    const long long nx = (long long)S.nroot[0] << l, ny = (long long)S.nroot[1] << l, nz = (long long)S.nroot[2] << l;
    if (bx < 0 || by < 0 || bz < 0 || bx >= nx || by >= ny || bz >= nz) return -1;
    return T.lut[S.lut_off[l] + (bz * ny + by) * nx + bx];
}

// boundary rule on a level-l global cell index; false means "inflow"
__device__ __forceinline__ bool apply_bounds(const DevSim &S, int l, long long G[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const long long n = ((long long)S.nroot[a] * 8) << l;
        if (G[a] < 0 || G[a] >= n) {
            const int side = G[a] >= n;
            const int t = S.bc[2 * a + side];
            if (t == BMHD_BC_PERIODIC) G[a] = ((G[a] % n) + n) % n;
            else if (t == BMHD_BC_OUTFLOW) G[a] = side ? n - 1 : 0;
            else return false;
        }
    }
    return true;
}

// The helpers below produce NV consecutive variables v0 .. v0 + NV - 1 of a cell (all eight by default; the
// level-change halo fill asks for four, so that two threads share a cell's loads).
template <int NV = 8>
__device__ __forceinline__ bool leaf_cell(const Cursor &c, const DevSim &S, int l, const long long G[3], double out[NV],
                                          int v0 = 0) {
    const int32_t b = lut_at(*c.T, S, l, G[0] >> 3, G[1] >> 3, G[2] >> 3);
    if (b < 0) return false;
    const size_t off = size_t(b) * 512 + size_t(((G[2] & 7) * 8 + (G[1] & 7)) * 8 + (G[0] & 7));
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = c.U[(v0 + v) * c.vs + off];
    return true;
}

template <int NV = 8>
__device__ __forceinline__ bool restricted_cell(const Cursor &c, const DevSim &S, const long long G[3], double out[NV],
                                                int v0 = 0) {
#pragma clang fp contract(off)
    size_t off[8];
    for (int q = 0; q < 8; ++q) {
        const long long F[3] = {2 * G[0] + (q & 1), 2 * G[1] + ((q >> 1) & 1), 2 * G[2] + (q >> 2)};
        const int32_t b = lut_at(*c.T, S, 1, F[0] >> 3, F[1] >> 3, F[2] >> 3);
        if (b < 0) return false;
        off[q] = size_t(b) * 512 + size_t(((F[2] & 7) * 8 + (F[1] & 7)) * 8 + (F[0] & 7));
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double *u = c.U + (v0 + v) * c.vs;
        const double s = ((u[off[0]] + u[off[1]]) + (u[off[2]] + u[off[3]])) +
                         ((u[off[4]] + u[off[5]]) + (u[off[6]] + u[off[7]]));
        out[v] = s * 0.125;
    }
    return true;
}

// level-0 value with boundary rule, from a level-0 leaf or restricted from level 1
template <int NV = 8>
__device__ __forceinline__ void coarse_cell(const Cursor &c, const DevSim &S, long long G[3], double out[NV], int v0 = 0) {
    if (!apply_bounds(S, 0, G)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v] = S.inflow_U[v0 + v];
        return;
    }
    if (leaf_cell<NV>(c, S, 0, G, out, v0)) return;
    restricted_cell<NV>(c, S, G, out, v0);
}

__device__ __forceinline__ double minmod2(double a, double b) {
    return (a > 0.0 && b > 0.0) ? fmin(a, b) : ((a < 0.0 && b < 0.0) ? fmax(a, b) : 0.0);
}

// any cell of a level-l grid, at a global index that may lie outside the domain. The ghost-rule helpers are
// inlined into their kernels: out of line, their arrays went through scratch memory and the call held 210
// registers (the level-change halo fill ran 19 % slower in FP64 two-level steps, 23 % with FP32 fluxes)
template <int NV = 8>
__device__ __forceinline__ void ghost_cell(const Cursor &c, const DevSim &S, int l, const long long G0[3], double out[NV],
                                           int v0 = 0) {
#pragma clang fp contract(off)
    long long G[3] = {G0[0], G0[1], G0[2]};
    if (!apply_bounds(S, l, G)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v] = S.inflow_U[v0 + v];
        return;
    }
    if (leaf_cell<NV>(c, S, l, G, out, v0)) return;
    if (l == 0) {
        restricted_cell<NV>(c, S, G, out, v0);
        return;
    }
    // prolongation from coarse cell C = G / 2
    long long C[3] = {G[0] >> 1, G[1] >> 1, G[2] >> 1};
    double uc[NV];
    leaf_cell<NV>(c, S, 0, C, uc, v0);
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = uc[v];
    for (int d = 0; d < 3; ++d) {
        long long Cm[3] = {C[0], C[1], C[2]}, Cp[3] = {C[0], C[1], C[2]};
        Cm[d] -= 1;
        Cp[d] += 1;
        double um[NV], up[NV];
        coarse_cell<NV>(c, S, Cm, um, v0);
        coarse_cell<NV>(c, S, Cp, up, v0);
        const double s = (G[d] & 1) ? 0.25 : -0.25;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = acc[v] + s * minmod2(uc[v] - um[v], up[v] - uc[v]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = acc[v];
}

// ------------------------------------------------------------------------------------------------
// kernels: state conversion, full ghost view, halo buffer

__global__ void k_set_state(const double *__restrict__ W, double *__restrict__ U, size_t n) {
    const size_t c = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double w[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) w[v] = W[v * n + c];
    const double rho = w[0];
    const double u2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    const double b2 = w[4] * w[4] + w[5] * w[5] + w[6] * w[6];
    U[c] = rho;
    U[n + c] = rho * w[1];
    U[2 * n + c] = rho * w[2];
    U[3 * n + c] = rho * w[3];
    U[4 * n + c] = w[4];
    U[5 * n + c] = w[5];
    U[6 * n + c] = w[6];
    U[7 * n + c] = w[7] * 1.5 + 0.5 * rho * u2 + 0.5 * b2;
}

__global__ void __launch_bounds__(256) k_fill_view(Tables T, const double *__restrict__ U, double *__restrict__ view) {
    const int b = blockIdx.x;
    const DevBlock &B = T.blocks[b];
    const DevSim &S = T.sims[B.sim];
    const size_t vs = size_t(T.nb) * 512, vv = size_t(T.nb) * 1728;
    Cursor cur{&T, U, vs};
    for (int c = threadIdx.x; c < 1728; c += blockDim.x) {
        const int i = c % 12 - 2, j = (c / 12) % 12 - 2, k = c / 144 - 2;
        double out[8];
        if ((unsigned)i < 8u && (unsigned)j < 8u && (unsigned)k < 8u) {
            const size_t off = size_t(b) * 512 + (k * 8 + j) * 8 + i;
#pragma unroll
            for (int v = 0; v < 8; ++v) out[v] = U[v * vs + off];
        } else {
            const long long G[3] = {(long long)B.ijk[0] * 8 + i, (long long)B.ijk[1] * 8 + j, (long long)B.ijk[2] * 8 + k};
            ghost_cell(cur, S, B.level, G, out);
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) view[v * vv + size_t(b) * 1728 + c] = out[v];
    }
}

// State remap after a refinement change: every cell of the new grid N takes the value that the ghost rules
// of the old grid F give at its level and global index -- the leaf's own value (block unchanged), the
// prolongation of a fine ghost cell (block refined from a level-0 parent) or the restriction of the 8
// children (block coarsened). One workgroup per new block, one thread per cell; no contraction (inside
// ghost_cell), so the result is exact to the oracle's.
__global__ void __launch_bounds__(512) k_remap(Tables F, const double *__restrict__ Uf, Tables N,
                                               double *__restrict__ Un) {
    const int b = blockIdx.x, c = threadIdx.x;
    const DevBlock &B = N.blocks[b];
    const DevSim &S = F.sims[B.sim];
    const Cursor cur{&F, Uf, size_t(F.nb) * 512};
    const long long G[3] = {(long long)B.ijk[0] * 8 + (c & 7), (long long)B.ijk[1] * 8 + ((c >> 3) & 7),
                            (long long)B.ijk[2] * 8 + (c >> 6)};
    double u[8];
    ghost_cell(cur, S, B.level, G, u);
    const size_t vs = size_t(N.nb) * 512, off = size_t(b) * 512 + c;
#pragma unroll
    for (int v = 0; v < 8; ++v) Un[v * vs + off] = u[v];
}

// Refinement indicator per block: the largest normalised jump, over its cells and the three axes, of the
// density and of |B|^2 between a cell's two face neighbours (neighbours outside the block by the ghost
// rules): |q+ - q-| / (q+ + q- + 1e-300). One workgroup per block, one thread per cell. No contraction: the
// value equals the host-side reference bit for bit.
__global__ void __launch_bounds__(512) k_block_indicator(Tables T, const double *__restrict__ U, double *__restrict__ ind) {
#pragma clang fp contract(off)
    __shared__ double red[8];
    const int b = blockIdx.x, c = threadIdx.x;
    const DevBlock &B = T.blocks[b];
    const DevSim &S = T.sims[B.sim];
    const size_t vs = size_t(T.nb) * 512;
    const Cursor cur{&T, U, vs};
    const int ii[3] = {c & 7, (c >> 3) & 7, c >> 6};
    double m = 0.0;
    for (int d = 0; d < 3; ++d) {
        double q[2][8];
        for (int side = 0; side < 2; ++side) {
            int n[3] = {ii[0], ii[1], ii[2]};
            n[d] += side ? 1 : -1;
            if ((unsigned)n[d] < 8u) {
                const size_t off = size_t(b) * 512 + (n[2] * 8 + n[1]) * 8 + n[0];
                for (int v = 0; v < 8; ++v) q[side][v] = U[v * vs + off];
            } else {
                const long long G[3] = {(long long)B.ijk[0] * 8 + n[0], (long long)B.ijk[1] * 8 + n[1],
                                        (long long)B.ijk[2] * 8 + n[2]};
                ghost_cell(cur, S, B.level, G, q[side]);
            }
        }
        const double rp = q[1][0], rm = q[0][0];
        const double bp = q[1][4] * q[1][4] + q[1][5] * q[1][5] + q[1][6] * q[1][6];
        const double bm = q[0][4] * q[0][4] + q[0][5] * q[0][5] + q[0][6] * q[0][6];
        const double jr = fabs(rp - rm) / (rp + rm + 1e-300);
        const double jb = fabs(bp - bm) / (bp + bm + 1e-300);
        m = fmax(m, fmax(jr, jb));
    }
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((c & 63) == 0) red[c >> 6] = m;
    __syncthreads();
    if (c == 0) {
        double r = red[0];
        for (int w = 1; w < 8; ++w) r = fmax(r, red[w]);
        ind[b] = r;
    }
}

// Ghost layers of one level-change face: item = (block << 3) | face; 256 threads = 2 halves of the
// variables x 2 layers x 64 cells. Two threads per cell repeat its index work and each loads four variables:
// on the two-level magnetosphere 1-2 % faster per step than one thread per cell (too few wavefronts to hide
// the chains of dependent loads) and than four or eight threads per cell (the repeated index work dominates).
__global__ void __launch_bounds__(256) k_halo_fill(Tables T, const double *__restrict__ U) {
    const int32_t item = T.halo_items[blockIdx.x];
    const int b = item >> 3, f = item & 7;
    const DevBlock &B = T.blocks[b];
    const DevSim &S = T.sims[B.sim];
    const int t = threadIdx.x, v = (t >> 7) * 4, cell = t & 127, layer = cell >> 6, t1 = cell & 7, t2 = (cell >> 3) & 7;
    const int a = f >> 1, side = f & 1;
    const int a1 = a == 0 ? 1 : 0, a2 = a == 2 ? 1 : 2;
    int idx[3];
    idx[a] = side ? 8 + layer : -1 - layer;
    idx[a1] = t1;
    idx[a2] = t2;
    const long long G[3] = {(long long)B.ijk[0] * 8 + idx[0], (long long)B.ijk[1] * 8 + idx[1],
                            (long long)B.ijk[2] * 8 + idx[2]};
    Cursor cur{&T, U, size_t(T.nb) * 512};
    double out[4];
    ghost_cell<4>(cur, S, B.level, G, out, v);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        T.halo[size_t(B.halo_slot) * HALO_SLOT + size_t(f) * HALO_FACE + (v + q) * 128 + layer * 64 + t2 * 8 + t1] = out[q];
}

// ------------------------------------------------------------------------------------------------
// time-step bound

__device__ __forceinline__ double cell_bound(const double w[8], double inv_dx) {
    const double ir = frcp(w[0]);
    const double cx = fast_speed<double, 0>(w, ir), cy = fast_speed<double, 1>(w, ir), cz = fast_speed<double, 2>(w, ir);
    return (fabs(w[1]) + cx) * inv_dx + (fabs(w[2]) + cy) * inv_dx + (fabs(w[3]) + cz) * inv_dx;
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
    return x;
}
__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// bits of a non-negative double order like the double; read first so that most workgroups skip the atomic
__device__ __forceinline__ void publish_max(unsigned long long *slot, double v) {
    if (!(v > 0.0)) {
        if (v != v) atomicMax(slot, 0x7ff8000000000000ull);
        return;
    }
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    if (__atomic_load_n(slot, __ATOMIC_RELAXED) < bits) atomicMax(slot, bits);
}

template <int NT>
__device__ __forceinline__ void block_publish(double lam, int nfault, double *red, int *redi, unsigned long long *slot,
                                              int32_t *faults) {
    lam = wave_max(lam);
    nfault = wave_sum(nfault);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[wid] = lam;
        redi[wid] = nfault;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        int n = redi[0];
        for (int w = 1; w < NT / 64; ++w) {
            m = fmax(m, red[w]);
            n += redi[w];
        }
        if (slot) publish_max(slot, m);
        if (n && faults) atomicAdd(faults, n);
    }
}

__global__ void __launch_bounds__(512) k_dt_reduce(Tables T, const double *__restrict__ U) {
    __shared__ double red[8];
    __shared__ int redi[8];
    const int b = blockIdx.x;
    const DevBlock &B = T.blocks[b];
    const DevSim &S = T.sims[B.sim];
    const size_t vs = size_t(T.nb) * 512;
    const int c = threadIdx.x;
    double u[8], w[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) u[v] = U[v * vs + size_t(b) * 512 + c];
    cons_to_prim(u, w);
    const double inv_dx = double(1 << B.level) / S.dx0;
    bool body = (B.flags & BF_NEAR_BODY) && in_body(S, B.level, B.ijk, c & 7, (c >> 3) & 7, c >> 6);
    const double lam = body ? 0.0 : cell_bound(w, inv_dx);
    block_publish<512>(lam, 0, red, redi, T.lam + B.sim, nullptr);
}

__global__ void k_dt_finalize(Tables T, double cfl, double *__restrict__ dt) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= T.ns) return;
    const double lam = __longlong_as_double((long long)T.lam[s]);
    dt[s] = cfl * (1.0 / lam);
    T.lam[s] = 0ull;
}

__global__ void k_lam_reset(Tables T) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < T.ns) T.lam[s] = 0ull;
}

// ------------------------------------------------------------------------------------------------
// the fused stage kernel

// LDS cell numbering of a slab with KS z-layers: [0, 64 KS) slab cells (k, j, i) = thread id; then the
// two z-halo layers below and above; then x-halo (k, j, 4) and y-halo (k, 4, i) columns.
template <int KS>
struct Slab {
    static constexpr int NCELLS = 64 * KS;  // cells of the slab, owned one per thread
    static constexpr int NFX = 72 * KS;
    static constexpr int NFZ = 64 * (KS + 1);
    static constexpr int NF = NFX > NFZ ? NFX : NFZ;
    // one face per thread in every sweep: 320 threads for KS = 4, 576 for KS = 8
    static constexpr int NT = (NF + 63) / 64 * 64;
    static constexpr int ZLO = 64 * KS;
    static constexpr int ZHI = 64 * KS + 128;
    static constexpr int XH = 64 * KS + 256;
    static constexpr int YH = 96 * KS + 256;
    static constexpr int NC = 128 * KS + 256;
    static constexpr int NPT = (NC + NT - 1) / NT;  // gathered cells per thread
    // (i, j, k) slab-local, at most one coordinate outside the slab
    __device__ static __forceinline__ int idx(int i, int j, int k) {
        if ((unsigned)i < 8u && (unsigned)j < 8u) {
            if ((unsigned)k < (unsigned)KS) return (k * 8 + j) * 8 + i;
            if (k < 0) return ZLO + ((k + 2) * 8 + j) * 8 + i;
            return ZHI + ((k - KS) * 8 + j) * 8 + i;
        }
        if ((unsigned)j < 8u) return XH + (k * 8 + j) * 4 + (i < 0 ? i + 2 : i - 6);
        return YH + (k * 4 + (j < 0 ? j + 2 : j - 6)) * 8 + i;
    }
    __device__ static __forceinline__ void decode(int c, int &i, int &j, int &k) {
        if (c < ZLO) {
            i = c & 7; j = (c >> 3) & 7; k = c >> 6;
        } else if (c < XH) {
            const int cc = c - ZLO, hi = cc >> 7, l = (cc >> 6) & 1;
            i = cc & 7; j = (cc >> 3) & 7; k = hi ? KS + l : l - 2;
        } else if (c < YH) {
            const int cc = c - XH, xh = cc & 3;
            k = cc >> 5; j = (cc >> 2) & 7; i = xh < 2 ? xh - 2 : xh + 6;
        } else {
            const int cc = c - YH, yh = (cc >> 3) & 3;
            k = cc >> 5; i = cc & 7; j = yh < 2 ? yh - 2 : yh + 6;
        }
    }
};

struct StageArgs {
    const double *Uin;
    const double *U0;
    double *Uout;
    double *dt;      // one step per simulation, or per cell with local_dt (written by the first stage)
    int32_t *faults;
    double alpha, beta;
    int use_u0;      // add alpha * U0 (second stage)
    int want_lam;    // accumulate the next dt bound
    int count_faults;
    int local_dt;    // local time stepping: dt holds one step per cell ([nB][512]) instead of one per simulation
    int write_dt;    // with local_dt: this stage forms each cell's step from its own input state and stores it
    double cfl;
    // learned correction (only read by the LEARN variants)
    const float *lrn_y;      // MLP outputs per face, normalised, face-normal frame
    const float *lrn_stats;  // in_mean[32], in_std[32], out_mean[8], out_std[8]
    uint8_t *lrn_flags;      // per cell: provisional state rejected
    int lrn_compact;         // lrn_y in the compact face layout (each face once) rather than bmhd_face_data's
    double tau;
    double floor_rel;        // the neighbourhood range is at least floor_rel times its largest magnitude
    // work list of the launch: a part of the Morton schedule (block ids), or null for all of T.order
    const int32_t *sched;
    int32_t n_sched;
    // ghost cells from a padded view [8][n][12][12][12] (one process's blocks after the exchange between
    // processes) instead of the neighbours' interiors, the boundary rules and the halo buffer: view_local[b]
    // is block b's index in the view, view_vs its variable stride; null: the usual gather
    const double *view;
    const int32_t *view_local;
    const int32_t *view_faces;  // per block: bit f, face f's ghost cells from the view (others in place)
    int64_t view_vs;
    // the coarse cells k_flux_correct takes: a list of n_fc_list cells, or null for all of T.fc_cells
    const DevFcCell *fc_list;
    int32_t n_fc_list;
};

__device__ __forceinline__ int sched_count(const Tables &T, const StageArgs &A) { return A.sched ? A.n_sched : T.nb; }
__device__ __forceinline__ int sched_block(const Tables &T, const StageArgs &A, int i) {
    return A.sched ? A.sched[i] : T.order[i];
}

// block-local index of face (i, j, z) of direction D (see bmhd_face_data)
template <int D>
__device__ __forceinline__ int face_index(int i, int j, int z) {
    return D == 0 ? (z * 8 + j) * 9 + i : (D == 1 ? (z * 9 + j) * 8 + i : (z * 8 + j) * 8 + i);
}

// Normalised learned correction of face (i, j, z) of direction D of block b (the face between cells
// (i, j, z) - e_D and (i, j, z), its coordinate along D in 0..8). In bmhd_face_data's layout every block
// holds its 576 faces per direction; in the compact layout of the network path every face is held once:
// [n_blocks][3][512] low faces (coordinate 0..7 along D, index (z 8 + j) 8 + i), then 64 faces per high
// face plane with no neighbour across it (DevBlock::hb_pos, index t2 8 + t1 over the two other axes in x,
// y, z order), so that a block's high face is its neighbour's low face.
template <int D>
__device__ __forceinline__ const float *lrn_y_at(const Tables &T, const StageArgs &A, int b, int i, int j, int z) {
    if (!A.lrn_compact) return A.lrn_y + ((size_t(b) * 3 + D) * 576 + face_index<D>(i, j, z)) * 8;
    const int a = D == 0 ? i : (D == 1 ? j : z);
    if (a < 8) return A.lrn_y + (size_t(b) * 1536 + D * 512 + (z * 8 + j) * 8 + i) * 8;
    const DevBlock &B = T.blocks[b];
    const int nbr = B.face[2 * D + 1];
    if (nbr >= 0) {
        const int i0 = D == 0 ? 0 : i, j0 = D == 1 ? 0 : j, z0 = D == 2 ? 0 : z;
        return A.lrn_y + (size_t(nbr) * 1536 + D * 512 + (z0 * 8 + j0) * 8 + i0) * 8;
    }
    const int t1 = D == 0 ? j : i, t2 = D == 2 ? j : z;
    return A.lrn_y + (size_t(T.nb) * 1536 + size_t(B.hb_pos[D]) * 64 + t2 * 8 + t1) * 8;
}

// learned flux increment of one face, de-normalised and rotated from the face-normal frame to x, y, z
template <typename R, int D>
__device__ __forceinline__ void learned_increment(const float *y, const float *stats, R dF[8]) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = y[q] * stats[72 + q] + stats[64 + q];
    dF[0] = R(v[0]);
    dF[7] = R(v[7]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        dF[1 + (D + a) % 3] = R(v[1 + a]);
        dF[4 + (D + a) % 3] = R(v[4 + a]);
    }
}

// The thread index, laundered through an empty asm statement so that index arithmetic derived from it
// is recomputed where it is used instead of being hoisted out of the persistent loop (where it would
// stay live across the whole slab computation and double the register footprint).
__device__ __forceinline__ int lane_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Body mask of the LDS cells of a slab: one byte per cell, or one bit per cell (32 cells per word).
struct ByteMask {
    const unsigned char *m;
    __device__ __forceinline__ bool operator()(int c) const { return m[c] != 0; }
};
struct BitMask {
    const uint32_t *m;
    __device__ __forceinline__ bool operator()(int c) const { return (m[c >> 5] >> (c & 31)) & 1u; }
};

// Record the flux of a face of direction D, (i, j, z) block-local (the face between cells (i-1, j, z) and
// (i, j, z) for D = 0, likewise j and z), if it lies on a block face that takes part in a flux correction.
template <int D, typename R>
__device__ __forceinline__ void record_fc(const Tables &T, const DevBlock &B, int i, int j, int z, const R fl[8]) {
    int bf = -1, t1 = 0, t2 = 0;
    if (D == 0) { if (i == 0) bf = 0; else if (i == 8) bf = 1; t1 = j; t2 = z; }
    if (D == 1) { if (j == 0) bf = 2; else if (j == 8) bf = 3; t1 = i; t2 = z; }
    if (D == 2) { if (z == 0) bf = 4; else if (z == 8) bf = 5; t1 = i; t2 = j; }
    if (bf >= 0 && B.fc_rec[bf] >= 0) {
        double *rec = T.fcbuf + size_t(B.fc_rec[bf]) * FC_REC;
        if ((B.fc_role >> bf) & 1) {
#pragma unroll
            for (int v = 0; v < 8; ++v) rec[v * 64 + t2 * 8 + t1] = double(fl[v]);
        } else {
            const int q = B.fc_quad[bf];
            const int g1 = 8 * (q & 1) + t1, g2 = 8 * (q >> 1) + t2;
#pragma unroll
            for (int v = 0; v < 8; ++v) rec[FC_COARSE + v * 256 + g2 * 16 + g1] = double(fl[v]);
        }
    }
}

// Flux through one face of direction D of a slab whose primitives are in LDS: the face between cells
// (i-1, j, k) and (i, j, k) for D = 0 (likewise j for D = 1, k for D = 2), slab-local coordinates, the face
// coordinate in 0..8 (0..KS along z). Returns the 8 flux components and the face-averaged normal field
// (for the divergence of the Powell source), and records the flux of block faces that take part in a
// flux correction.
template <int KS, typename R, int D, int FLUX, bool BODY, bool LEARN, typename Mask>
__device__ __forceinline__ void face_flux(const Tables &T, const StageArgs &A, const DevBlock &B, int b, int slab,
                                          R (*sW)[Slab<KS>::NC], Mask sM, int i, int j, int k, R fl[8], R &bbar) {
    using SL = Slab<KS>;
    int c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int o = q - 2;
        c[q] = D == 0 ? SL::idx(i + o, j, k) : (D == 1 ? SL::idx(i, j + o, k) : SL::idx(i, j, k + o));
    }
    // face values: W_L = W_{i-1} + slope/2, W_R = W_i - slope/2 (monotonized central)
    R wl[8], wr[8];
    bool m0 = false, m1 = false, m2 = false, m3 = false;
    if constexpr (BODY) {
        m0 = sM(c[0]); m1 = sM(c[1]); m2 = sM(c[2]); m3 = sM(c[3]);
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const R a = sW[v][c[0]], b = sW[v][c[1]], cc = sW[v][c[2]], d = sW[v][c[3]];
        const R d0 = b - a, d1 = cc - b, d2 = d - cc;
        R hl = mc_half(d0, d1), hr = mc_half(d1, d2);
        if constexpr (BODY) {
            hl = (m0 || m2) ? R(0) : hl;
            hr = (m1 || m3) ? R(0) : hr;
        }
        wl[v] = b + hl;
        wr[v] = cc - hr;
    }
    bool skip = false;
    if constexpr (BODY) {
        // a face between a fluid and a body cell reflects the first-order fluid state
        if (m1 && m2) {
            skip = true;
        } else if (m2) {
#pragma unroll
            for (int v = 0; v < 8; ++v) wr[v] = wl[v];
            wr[1 + D] = -wl[1 + D];
        } else if (m1) {
#pragma unroll
            for (int v = 0; v < 8; ++v) wl[v] = wr[v];
            wl[1 + D] = -wr[1 + D];
        }
    }
    num_flux<R, D, FLUX>(wl, wr, fl);
    if constexpr (LEARN) {
        // faces next to a body cell keep the plain (reflecting) flux
        if (!(m1 || m2)) {
            R dF[8];
            learned_increment<R, D>(lrn_y_at<D>(T, A, b, i, j, slab * KS + k), A.lrn_stats, dF);
#pragma unroll
            for (int v = 0; v < 8; ++v) fl[v] += dF[v];
        }
    }
    bbar = R(0.5) * (wl[4 + D] + wr[4 + D]);
    if constexpr (BODY) {
        if (skip) {
#pragma unroll
            for (int v = 0; v < 8; ++v) fl[v] = R(0);
            bbar = R(0);
        }
    }
    if (B.flags & BF_FC) record_fc<D>(T, B, i, j, slab * KS + k, fl);
}

// One sweep of the face-per-thread scheme: thread f takes face f of direction D and leaves its flux in
// sF for the two cells on either side.
template <int KS, typename R, int D, int FLUX, bool BODY>
__device__ __forceinline__ void sweep(const Tables &T, const StageArgs &A, const DevBlock &B, int b, int slab,
                                      R (*sW)[Slab<KS>::NC], const unsigned char *sM, R (*sF)[Slab<KS>::NF]) {
    using SL = Slab<KS>;
    constexpr int NF = D == 2 ? SL::NFZ : SL::NFX;
    const int f = lane_tid();
    if (f >= NF) return;
    int i, j, k;
    if (D == 0) { i = f % 9; j = (f / 9) & 7; k = f / 72; }
    else if (D == 1) { i = f & 7; j = (f >> 3) % 9; k = f / 72; }
    else { i = f & 7; j = (f >> 3) & 7; k = f >> 6; }
    R fl[8], bbar;
    face_flux<KS, R, D, FLUX, BODY, false>(T, A, B, b, slab, sW, ByteMask{sM}, i, j, k, fl, bbar);
#pragma unroll
    for (int v = 0; v < 8; ++v) sF[v][f] = fl[v];
    sF[8][f] = bbar;
}

template <int KS, typename R, int D>
__device__ __forceinline__ void accumulate(R (*sF)[Slab<KS>::NF], double rhs[8], double &divb, double inv_dx) {
    const int t = lane_tid(), i = t & 7, j = (t >> 3) & 7, k = t >> 6;
    int fl, fr;
    if (D == 0) { fl = k * 72 + j * 9 + i; fr = fl + 1; }
    else if (D == 1) { fl = k * 72 + j * 8 + i; fr = fl + 8; }
    else { fl = (k * 8 + j) * 8 + i; fr = fl + 64; }
#pragma unroll
    for (int v = 0; v < 8; ++v) rhs[v] += (double(sF[v][fl]) - double(sF[v][fr])) * inv_dx;
    divb += (double(sF[8][fr]) - double(sF[8][fl])) * inv_dx;
}

// Cells of a slab and its face halos gathered per thread by a workgroup of NTH threads.
template <int KS, int NTH>
constexpr int gather_npt() { return (Slab<KS>::NC + NTH - 1) / NTH; }

// Issue the global loads of one slab and its face halos (cells tid, tid + NTH, ...) into registers.
template <int KS, int NTH = Slab<KS>::NT, bool VIEW = false>
__device__ __forceinline__ void gather_issue(const Tables &T, const StageArgs &A, int b, int slab,
                                             double (&u)[gather_npt<KS, NTH>()][8]) {
    using SL = Slab<KS>;
    constexpr int NPT = gather_npt<KS, NTH>();
    const DevBlock &B = T.blocks[b];
    const DevSim &S = T.sims[B.sim];
    const size_t vs = size_t(T.nb) * 512;
    const int tid = lane_tid();
    // view gather: the ghost cells of faces whose neighbour is on another process or level come from the
    // process's padded view (received messages, restrictions, prolongations); the rest is read in place
    const int vfaces = VIEW ? A.view_faces[b] : 0;
    const double *vbase = VIEW ? A.view + size_t(A.view_local[b]) * 1728 : nullptr;
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
        const int c = tid + m * NTH;
        if (c >= SL::NC) break;
        int i, j, k;
        SL::decode(c, i, j, k);
        const int z = slab * KS + k;
        int fd = -1;
        if (i < 0) fd = 0; else if (i > 7) fd = 1;
        else if (j < 0) fd = 2; else if (j > 7) fd = 3;
        else if (z < 0) fd = 4; else if (z > 7) fd = 5;
        const int rel = fd < 0 ? b : B.face[fd];
        const double *p;
        size_t stride;
        if (VIEW && fd >= 0 && ((vfaces >> fd) & 1)) {
            p = vbase + ((z + 2) * 12 + (j + 2)) * 12 + (i + 2);
            stride = size_t(A.view_vs);
        } else if (rel >= 0 || rel == FACE_OUTFLOW) {
            int src = b, ii = i, jj = j, zz = z;
            if (rel >= 0) {
                src = rel;
                ii &= 7; jj &= 7; zz &= 7;
            } else {
                ii = ii < 0 ? 0 : (ii > 7 ? 7 : ii);
                jj = jj < 0 ? 0 : (jj > 7 ? 7 : jj);
                zz = zz < 0 ? 0 : (zz > 7 ? 7 : zz);
            }
            p = A.Uin + size_t(src) * 512 + (zz * 8 + jj) * 8 + ii;
            stride = vs;
        } else if (rel == FACE_INFLOW) {
            p = S.inflow_U;
            stride = 1;
        } else {
            const int a = fd >> 1;
            const int along = a == 0 ? i : (a == 1 ? j : z);
            const int layer = along < 0 ? -1 - along : along - 8;
            const int t1 = a == 0 ? j : i, t2 = a == 2 ? j : z;
            p = T.halo + size_t(B.halo_slot) * HALO_SLOT + size_t(fd) * HALO_FACE + layer * 64 + t2 * 8 + t1;
            stride = 128;
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) u[m][v] = p[v * stride];
    }
}

// Convert the gathered conserved values to primitives in LDS (and the body mask near a body).
template <int KS, typename R>
__device__ __forceinline__ void gather_store(const Tables &T, int b, int slab, const double (&u)[Slab<KS>::NPT][8],
                                             R (*sW)[Slab<KS>::NC], unsigned char *sM) {
    using SL = Slab<KS>;
    const DevBlock &B = T.blocks[b];
    const bool near_body = (B.flags & BF_NEAR_BODY) != 0;
    const int tid = lane_tid();
#pragma unroll
    for (int m = 0; m < SL::NPT; ++m) {
        const int c = tid + m * SL::NT;
        if (c >= SL::NC) break;
        double w[8];
        cons_to_prim(u[m], w);
#pragma unroll
        for (int v = 0; v < 8; ++v) sW[v][c] = R(w[v]);
        if (near_body) {
            int i, j, k;
            SL::decode(c, i, j, k);
            sM[c] = in_body(T.sims[B.sim], B.level, B.ijk, i, j, slab * KS + k) ? 1 : 0;
        }
    }
}

// Range of density and pressure over the old 7-point neighbourhood of slab cell tid (learned
// correction's acceptance test): rng = {rho min, rho max, p min, p max}, from the slab arrays `rho` and
// `p` (the LDS primitives, or their FP64 copies in the FP32-flux form).
template <int KS, typename V>
__device__ __forceinline__ void neighbour_range(const V *rho, const V *p, int tid, double rng[4]) {
    using SL = Slab<KS>;
    const int i = tid & 7, j = (tid >> 3) & 7, kk = tid >> 6;
    const int nb7[7] = {SL::idx(i, j, kk), SL::idx(i - 1, j, kk), SL::idx(i + 1, j, kk), SL::idx(i, j - 1, kk),
                        SL::idx(i, j + 1, kk), SL::idx(i, j, kk - 1), SL::idx(i, j, kk + 1)};
    double rlo = 1e300, rhi = -1e300, plo = 1e300, phi = -1e300;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const double r0 = double(rho[nb7[q]]), p0 = double(p[nb7[q]]);
        rlo = fmin(rlo, r0); rhi = fmax(rhi, r0);
        plo = fmin(plo, p0); phi = fmax(phi, p0);
    }
    rng[0] = rlo; rng[1] = rhi; rng[2] = plo; rng[3] = phi;
}

// Acceptance test of a provisional state under the learned correction: density r and pressure p positive
// and each inside [lo - tau h, hi + tau h] of its old neighbourhood range nr, where h is the range widened
// to at least floor_rel * max(|lo|, |hi|) (so that a uniform neighbourhood still admits a small change).
// Evaluated without contraction: the decision is the one plain FP64 arithmetic takes.
__device__ __forceinline__ bool learned_rejects(double r, double p, const double nr[4], double tau,
                                                double floor_rel) {
#pragma clang fp contract(off)
    bool bad = !(r > 0.0) || !(p > 0.0);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const double lo = nr[2 * m], hi = nr[2 * m + 1], v = m ? p : r;
        double h = hi - lo;
        const double fh = floor_rel * fmax(fabs(lo), fabs(hi));
        if (fh > h) h = fh;
        const double band = tau * h;
        bad = bad || v < lo - band || v > hi + band;
    }
    return bad;
}

// Powell source, stage update and write of the thread's own cell (threads below 64 KS own cell tid of
// the slab), then the end-of-step bookkeeping: positivity check and the next time-step bound. With the
// learned correction, `rng` (or the LDS primitives when it is null) gives the old neighbourhood range.
template <int KS, typename R, bool POWELL, bool LEARN, typename Mask, int NT = Slab<KS>::NT>
__device__ __forceinline__ void cell_update(const Tables &T, const StageArgs &A, int b, int slab, const double (&uin)[8],
                                            R (*sW)[Slab<KS>::NC], Mask sM, double (&rhs)[8], double divb,
                                            double inv_dx, double *red, int *redi, const double *rng = nullptr) {
    using SL = Slab<KS>;
    const DevBlock &B = T.blocks[b];
    const size_t vs = size_t(T.nb) * 512;
    const bool near_body = (B.flags & BF_NEAR_BODY) != 0;
    const int tid = lane_tid();
    const bool owner = tid < SL::NCELLS;
    const bool body = owner && near_body && sM(tid);
    const int cell = tid + slab * 64 * KS;
    const size_t off = size_t(b) * 512 + cell;
    double out[8];
    if (owner) {
        if (body) {
#pragma unroll
            for (int v = 0; v < 8; ++v) out[v] = uin[v];
            if (A.local_dt && A.write_dt) A.dt[off] = 0.0;
        } else {
            if (POWELL) {
                const double ux = double(sW[1][tid]), uy = double(sW[2][tid]), uz = double(sW[3][tid]);
                const double bx = double(sW[4][tid]), by = double(sW[5][tid]), bz = double(sW[6][tid]);
                const double ub = ux * bx + uy * by + uz * bz;
                rhs[1] -= divb * bx;
                rhs[2] -= divb * by;
                rhs[3] -= divb * bz;
                rhs[4] -= divb * ux;
                rhs[5] -= divb * uy;
                rhs[6] -= divb * uz;
                rhs[7] -= divb * ub;
            }
            double dtc;
            if (!A.local_dt) {
                dtc = A.dt[B.sim];
            } else if (A.write_dt) {
                // local time stepping: the cell's own CFL step from its stage input (the step's starting
                // state), the same expression as the global step of one cell
                double w[8];
                cons_to_prim(uin, w);
                dtc = A.cfl * (1.0 / cell_bound(w, inv_dx));
                A.dt[off] = dtc;
            } else {
                dtc = A.dt[off];
            }
            const double bdt = A.beta * dtc;
            if (A.use_u0) {
                const double a0 = A.alpha, a1 = 1.0 - A.alpha;
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    out[v] = a0 * __builtin_nontemporal_load(A.U0 + v * vs + off) + a1 * uin[v] + bdt * rhs[v];
            } else {
#pragma unroll
                for (int v = 0; v < 8; ++v) out[v] = uin[v] + bdt * rhs[v];
            }
        }
#pragma unroll
        // the stage result and U^n are streamed (stored / read once per stage): non-temporal, so that they
        // do not push the neighbours' halo cells out of L2
        for (int v = 0; v < 8; ++v) __builtin_nontemporal_store(out[v], A.Uout + v * vs + off);
        if constexpr (LEARN) {
            // reject the provisional state if it is not positive or leaves the widened range of the old
            // 7-point neighbourhood in density or pressure
            bool bad = false;
            if (!body) {
                double w[8];
                cons_to_prim(out, w);
                double nr[4];
                if (rng) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) nr[q] = rng[q];
                } else {
                    neighbour_range<KS, R>(sW[0], sW[7], tid, nr);
                }
                bad = learned_rejects(w[0], w[7], nr, A.tau, A.floor_rel);
            }
            A.lrn_flags[off] = bad ? 1 : 0;
        }
    }

    // end of a step: positivity check and the next time-step bound
    if (A.count_faults || A.want_lam) {
        double lam = 0.0;
        int nf = 0;
        if (owner && !body) {
            const int i = tid & 7, j = (tid >> 3) & 7, z = slab * KS + (tid >> 6);
            const int skipm = B.fc_skip;
            const bool later = skipm && (((skipm & 1) && i == 0) || ((skipm & 2) && i == 7) || ((skipm & 4) && j == 0) ||
                                         ((skipm & 8) && j == 7) || ((skipm & 16) && z == 0) || ((skipm & 32) && z == 7));
            if (!later) {
                double w[8];
                cons_to_prim(out, w);
                nf = !(w[0] > 0.0) || !(w[7] > 0.0) || !(w[7] < INFINITY);
                if (A.want_lam) lam = cell_bound(w, inv_dx);
            }
        }
        block_publish<NT>(lam, A.count_faults ? nf : 0, red, redi, A.want_lam ? T.lam + B.sim : nullptr,
                          A.faults);
    }
}

// Sweeps, source, update and end-of-step bookkeeping for one slab whose primitives are in LDS.
template <int KS, typename R, int FLUX, bool POWELL>
__device__ __forceinline__ void slab_compute(const Tables &T, const StageArgs &A, int b, int slab, const double (&uin)[8],
                                             R (*sW)[Slab<KS>::NC], unsigned char *sM, R (*sF)[Slab<KS>::NF],
                                             double *red, int *redi) {
    using SL = Slab<KS>;
    const DevBlock &B = T.blocks[b];
    const DevSim &S = T.sims[B.sim];
    const bool near_body = (B.flags & BF_NEAR_BODY) != 0;
    const int tid = lane_tid();
    const bool owner = tid < SL::NCELLS;

    // three flux sweeps, one face per thread; fluxes meet their two cells through LDS
    const double inv_dx = double(1 << B.level) / S.dx0;
    double rhs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double divb = 0.0;
    if (near_body) sweep<KS, R, 0, FLUX, true>(T, A, B, b, slab, sW, sM, sF);
    else sweep<KS, R, 0, FLUX, false>(T, A, B, b, slab, sW, sM, sF);
    __syncthreads();
    if (owner) accumulate<KS, R, 0>(sF, rhs, divb, inv_dx);
    __syncthreads();
    if (near_body) sweep<KS, R, 1, FLUX, true>(T, A, B, b, slab, sW, sM, sF);
    else sweep<KS, R, 1, FLUX, false>(T, A, B, b, slab, sW, sM, sF);
    __syncthreads();
    if (owner) accumulate<KS, R, 1>(sF, rhs, divb, inv_dx);
    __syncthreads();
    if (near_body) sweep<KS, R, 2, FLUX, true>(T, A, B, b, slab, sW, sM, sF);
    else sweep<KS, R, 2, FLUX, false>(T, A, B, b, slab, sW, sM, sF);
    __syncthreads();
    if (owner) accumulate<KS, R, 2>(sF, rhs, divb, inv_dx);
    cell_update<KS, R, POWELL, false>(T, A, b, slab, uin, sW, ByteMask{sM}, rhs, divb, inv_dx, red, redi);
}

// Work item -> (block, slab). Items are the slabs of the Morton-ordered block list. XCD x (workgroups
// w with w % 8 == x) owns the contiguous item range [first(x), first(x) + count(x)).
__device__ __forceinline__ int xcd_first(int nwork, int x) {
    const int q = nwork >> 3, r = nwork & 7;
    return x * q + (x < r ? x : r);
}
__device__ __forceinline__ int xcd_count(int nwork, int x) { return (nwork >> 3) + (x < (nwork & 7) ? 1 : 0); }

// One workgroup per slab (PERSIST = false: the grid has one workgroup per item) or a persistent grid
// (PERSIST = true: gridDim.x workgroups, a multiple of 8, each looping over the items of its XCD). The
// gather of a slab is issued at the top of its iteration: holding the next slab's 24 values per thread
// in registers across the flux sweeps would double the register footprint and halve occupancy, while
// two co-resident workgroups per CU already overlap one's gather with the other's sweeps.
template <int KS, typename R, int FLUX, bool POWELL, bool PERSIST>
__global__ void __launch_bounds__(Slab<KS>::NT) k_stage(Tables T, StageArgs A) {
    using SL = Slab<KS>;
    constexpr int S_PER_BLOCK = 8 / KS;
    __shared__ R sW[8][SL::NC];
    __shared__ R sF[9][SL::NF];
    __shared__ unsigned char sM[SL::NC];
    __shared__ double red[SL::NT / 64];
    __shared__ int redi[SL::NT / 64];

    const int nwork = T.nb * S_PER_BLOCK;
    const int wg = blockIdx.x, xcd = wg & 7, slot = wg >> 3;
    const int first = xcd_first(nwork, xcd), count = xcd_count(nwork, xcd);
    if constexpr (!PERSIST) {
        const int item = first + slot;
        const int b = T.order[item / S_PER_BLOCK], slab = item % S_PER_BLOCK;
        double u[SL::NPT][8];
        gather_issue<KS>(T, A, b, slab, u);
        gather_store<KS, R>(T, b, slab, u, sW, sM);
        __syncthreads();
        slab_compute<KS, R, FLUX, POWELL>(T, A, b, slab, u[0], sW, sM, sF, red, redi);
    } else {
        const int step = int(gridDim.x >> 3);
#pragma nounroll
        for (int it = slot; it < count; it += step) {
            const int item = first + it;
            const int b = T.order[item / S_PER_BLOCK], slab = item % S_PER_BLOCK;
            double u[SL::NPT][8];
            gather_issue<KS>(T, A, b, slab, u);
            gather_store<KS, R>(T, b, slab, u, sW, sM);
            __syncthreads();
            slab_compute<KS, R, FLUX, POWELL>(T, A, b, slab, u[0], sW, sM, sF, red, redi);
            __syncthreads();
            // keep the scheduler from overlapping iterations (that would hold two slabs' values live)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// ------------------------------------------------------------------------------------------------
// Wave-per-plane form of the stage kernel. A slab of KS z-layers is worked by KS + 1 waves: wave k < KS
// owns cell layer k (lane = (i, j)) and computes the face on the low side of each of its cells in every
// direction; wave KS computes the slab's high-side faces (x = 8, y = 8, z = KS). The flux through the
// high side of a cell then comes from the neighbouring lane (x: lane + 1, y: lane + 8, by cross-lane
// permute), from the next wave (z) or from the last wave (the slab's high faces), so no per-face flux
// array is kept: the z fluxes reuse the LDS space of the x and y halos, which is dead once the x and y
// faces are done, and one small buffer carries the last wave's high faces (x, then y, then the z faces'
// normal field). LDS per slab of four layers: 51.6 KB in FP64, small enough for three workgroups per CU.

// Convert the gathered conserved values to primitives in LDS and set one body-mask bit per cell.
template <int KS, typename R, bool RP = false>
__device__ __forceinline__ void gather_store_bits(const Tables &T, int b, int slab,
                                                  const double (&u)[Slab<KS>::NPT][8], R (*sW)[Slab<KS>::NC],
                                                  uint32_t *sMb, double *rp = nullptr) {
    using SL = Slab<KS>;
    const DevBlock &B = T.blocks[b];
    const bool near_body = (B.flags & BF_NEAR_BODY) != 0;
    const int tid = lane_tid();
#pragma unroll
    for (int m = 0; m < SL::NPT; ++m) {
        // NC and NT are multiples of 64: a wave's cells are all valid or all past the end
        const int c = tid + m * SL::NT;
        if (c >= SL::NC) break;
        double w[8];
        cons_to_prim(u[m], w);
#pragma unroll
        for (int v = 0; v < 8; ++v) sW[v][c] = R(w[v]);
        if constexpr (RP) {
            rp[c] = w[0];
            rp[SL::NC + c] = w[7];
        }
        if (near_body) {
            int i, j, k;
            SL::decode(c, i, j, k);
            const bool inb = in_body(T.sims[B.sim], B.level, B.ijk, i, j, slab * KS + k);
            const unsigned long long bits = __ballot(inb);
            if ((tid & 63) == 0) {
                sMb[c >> 5] = uint32_t(bits);
                sMb[(c >> 5) + 1] = uint32_t(bits >> 32);
            }
        }
    }
}

template <int KS, typename R, int D, int FLUX, bool LEARN>
__device__ __forceinline__ void wp_face(const Tables &T, const StageArgs &A, const DevBlock &B, int b, int slab,
                                        R (*sW)[Slab<KS>::NC], BitMask sM, bool near_body, int i, int j, int k,
                                        R fl[8], R &bbar) {
    if (near_body) face_flux<KS, R, D, FLUX, true, LEARN>(T, A, B, b, slab, sW, sM, i, j, k, fl, bbar);
    else face_flux<KS, R, D, FLUX, false, LEARN>(T, A, B, b, slab, sW, sM, i, j, k, fl, bbar);
}

template <typename R>
__device__ __forceinline__ R lane_down(R x, int delta) { return __shfl_down(x, delta, 64); }

template <int KS, typename R, int FLUX, bool POWELL, bool LEARN>
__device__ __forceinline__ void wp_compute(const Tables &T, const StageArgs &A, int b, int slab,
                                           R (*sW)[Slab<KS>::NC], R (*sH)[8 * KS], const uint32_t *sMb, double *red,
                                           int *redi, const double *rp = nullptr) {
    using SL = Slab<KS>;
    constexpr int NE = 8 * KS;
    const DevBlock &B = T.blocks[b];
    const DevSim &S = T.sims[B.sim];
    const bool near_body = (B.flags & BF_NEAR_BODY) != 0;
    const BitMask mk{sMb};
    const int tid = lane_tid();
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = tid & 63, ci = l & 7, cj = l >> 3;
    const bool cellw = w < KS;
    const double inv_dx = double(1 << B.level) / S.dx0;
    double rhs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double divb = 0.0;
    R fl[8], fr[8], bb, bbr;
    // learned correction: the old neighbourhood range, taken before the x/y halos are overwritten (from the
    // FP64 copies of density and pressure when the LDS primitives are FP32)
    double rng[4] = {0, 0, 0, 0};
    if constexpr (LEARN) {
        if (cellw) {
            if constexpr (sizeof(R) == 4) neighbour_range<KS, double>(rp, rp + SL::NC, tid, rng);
            else neighbour_range<KS, R>(sW[0], sW[7], tid, rng);
        }
    }

    // x: low-x face of each cell; the last wave takes the faces at x = 8 of the slab's 8 KS rows
    if (cellw) {
        wp_face<KS, R, 0, FLUX, LEARN>(T, A, B, b, slab, sW, mk, near_body, ci, cj, w, fl, bb);
#pragma unroll
        for (int v = 0; v < 8; ++v) fr[v] = lane_down(fl[v], 1);
        bbr = lane_down(bb, 1);
    } else if (l < NE) {
        wp_face<KS, R, 0, FLUX, LEARN>(T, A, B, b, slab, sW, mk, near_body, 8, l & 7, l >> 3, fl, bb);
#pragma unroll
        for (int v = 0; v < 8; ++v) sH[v][l] = fl[v];
        sH[8][l] = bb;
    }
    __syncthreads();
    if (cellw) {
        if (ci == 7) {
#pragma unroll
            for (int v = 0; v < 8; ++v) fr[v] = sH[v][w * 8 + cj];
            bbr = sH[8][w * 8 + cj];
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) rhs[v] += (double(fl[v]) - double(fr[v])) * inv_dx;
        divb += (double(bbr) - double(bb)) * inv_dx;
    }
    __syncthreads();  // sH is read: it takes the y faces next

    // y: low-y faces; the last wave takes the faces at y = 8
    if (cellw) {
        wp_face<KS, R, 1, FLUX, LEARN>(T, A, B, b, slab, sW, mk, near_body, ci, cj, w, fl, bb);
#pragma unroll
        for (int v = 0; v < 8; ++v) fr[v] = lane_down(fl[v], 8);
        bbr = lane_down(bb, 8);
    } else if (l < NE) {
        wp_face<KS, R, 1, FLUX, LEARN>(T, A, B, b, slab, sW, mk, near_body, l & 7, 8, l >> 3, fl, bb);
#pragma unroll
        for (int v = 0; v < 8; ++v) sH[v][l] = fl[v];
        sH[8][l] = bb;
    }
    __syncthreads();
    if (cellw) {
        if (cj == 7) {
#pragma unroll
            for (int v = 0; v < 8; ++v) fr[v] = sH[v][w * 8 + ci];
            bbr = sH[8][w * 8 + ci];
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) rhs[v] += (double(fl[v]) - double(fr[v])) * inv_dx;
        divb += (double(bbr) - double(bb)) * inv_dx;
    }
    // past this barrier no x or y halo cell is read again and sH is consumed: the z fluxes of face layer
    // p + 1 go to the x/y halo space of each variable (64 KS values per variable), their face-averaged
    // normal field to sH
    __syncthreads();

    // z: wave k < KS takes face layer k (low side of its cells), the last wave face layer KS
    R *zb = &sH[0][0];
    {
        const int kf = cellw ? w : KS;
        wp_face<KS, R, 2, FLUX, LEARN>(T, A, B, b, slab, sW, mk, near_body, ci, cj, kf, fl, bb);
        if (kf > 0) {
#pragma unroll
            for (int v = 0; v < 8; ++v) sW[v][SL::XH + (kf - 1) * 64 + l] = fl[v];
            zb[(kf - 1) * 64 + l] = bb;
        }
    }
    __syncthreads();
    double uin[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (cellw) {
#pragma unroll
        for (int v = 0; v < 8; ++v) fr[v] = sW[v][SL::XH + w * 64 + l];
        bbr = zb[w * 64 + l];
#pragma unroll
        for (int v = 0; v < 8; ++v) rhs[v] += (double(fl[v]) - double(fr[v])) * inv_dx;
        divb += (double(bbr) - double(bb)) * inv_dx;
        // the cell's own stage input, read again here rather than held in registers through the sweeps
        const size_t vs = size_t(T.nb) * 512, off = size_t(b) * 512 + slab * 64 * KS + tid;
#pragma unroll
        for (int v = 0; v < 8; ++v) uin[v] = A.Uin[v * vs + off];
    }
    cell_update<KS, R, POWELL, LEARN>(T, A, b, slab, uin, sW, mk, rhs, divb, inv_dx, red, redi, rng);
}

// One work item of the persistent form, kept out of line: inlined into the persistent loop the compiler
// keeps loop-carried copies live through the flux computation and spills (71 VGPRs at 128).
template <int KS, typename R, int FLUX, bool POWELL, bool LEARN>
__device__ __noinline__ void wp_item(const Tables &T, const StageArgs &A, int b, int slab, R (*sW)[Slab<KS>::NC],
                                     R (*sH)[8 * KS], uint32_t *sMb, double *red, int *redi) {
    using SL = Slab<KS>;
    {
        double u[SL::NPT][8];
        gather_issue<KS>(T, A, b, slab, u);
        gather_store_bits<KS, R>(T, b, slab, u, sW, sMb);
    }
    __syncthreads();
    wp_compute<KS, R, FLUX, POWELL, LEARN>(T, A, b, slab, sW, sH, sMb, red, redi);
}

// Waves per SIMD the register allocator aims for: four (at most 128 VGPRs), except for the FP64 tile of
// eight cell layers, whose LDS footprint already allows only one workgroup (three waves per SIMD) per CU.
template <int KS, typename R>
constexpr int wp_waves_per_simd() { return (KS == 8 && sizeof(R) == 8) ? 3 : 4; }

template <int KS, typename R, int FLUX, bool POWELL, bool PERSIST, bool LEARN = false, bool VIEW = false>
__global__ void __launch_bounds__(64 * (KS + 1), (wp_waves_per_simd<KS, R>())) k_stage_wp(Tables T, StageArgs A) {
    using SL = Slab<KS>;
    static_assert(SL::NT == 64 * (KS + 1), "one wave per cell layer plus one");
    static_assert(SL::NC - SL::XH == 64 * KS && 9 * 8 * KS >= 64 * KS, "z-flux exchange space");
    constexpr int S_PER_BLOCK = 8 / KS;
    __shared__ R sW[8][SL::NC];
    __shared__ R sH[9][8 * KS];
    __shared__ uint32_t sMb[SL::NC / 32];
    __shared__ double red[KS + 1];
    __shared__ int redi[KS + 1];
    // learned FP32-flux form: FP64 density and pressure of the gathered cells, for the acceptance test
    constexpr bool RP = LEARN && sizeof(R) == 4;
    __shared__ double sRP[RP ? 2 * SL::NC : 1];

    const int nwork = sched_count(T, A) * S_PER_BLOCK;
    const int wg = blockIdx.x, xcd = wg & 7, slot = wg >> 3;
    const int first = xcd_first(nwork, xcd), count = xcd_count(nwork, xcd);
    if constexpr (!PERSIST) {
        const int item = first + slot;
        const int b = sched_block(T, A, item / S_PER_BLOCK), slab = item % S_PER_BLOCK;
        {
            double u[SL::NPT][8];
            gather_issue<KS, SL::NT, VIEW>(T, A, b, slab, u);
            gather_store_bits<KS, R, RP>(T, b, slab, u, sW, sMb, sRP);
        }
        __syncthreads();
        wp_compute<KS, R, FLUX, POWELL, LEARN>(T, A, b, slab, sW, sH, sMb, red, redi, sRP);
    } else {
        static_assert(!LEARN && !VIEW, "the learned correction and the view gather run one workgroup per slab");
        const int step = int(gridDim.x >> 3);
#pragma nounroll
        for (int it = slot; it < count; it += step) {
            const int item = first + it;
            const int b = sched_block(T, A, item / S_PER_BLOCK), slab = item % S_PER_BLOCK;
            wp_item<KS, R, FLUX, POWELL, LEARN>(T, A, b, slab, sW, sH, sMb, red, redi);
            __syncthreads();
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// ------------------------------------------------------------------------------------------------
// Block form of the stage kernel: one workgroup of eight wavefronts per 8x8x8 block clear of any body,
// wavefront k owning cell layer k (lane = (i, j)). Each wavefront computes the low-side face of each of
// its cells in x, y and z, as the plane form does, and, in one more pass with the direction chosen per
// lane, its layer's eight faces at x = 8 and eight at y = 8 (each evaluated in the lane whose cell it
// bounds) plus eight of the block's 64 faces at z = 8: every wavefront does four face passes and no
// wavefront is set aside for the high faces. Flux differences enter each cell's sums as two multiply-adds
// (low side, then high side). LDS holds exactly the block and its face halos (80 KiB in FP64): the z
// fluxes travel through the x/y halo space and the top halo layer once those are dead, and the
// end-of-step reduction reuses the bottom halo layers, so two workgroups (sixteen wavefronts) share a
// CU (the plane form on 8x8x4 slabs: ten). Blocks near a body run on the plane form in a second launch.

constexpr int BLK_NT = 512;

// Convert the gathered conserved values of a block and its face halos to primitives in LDS.
template <typename R>
__device__ __forceinline__ void gather_store_blk(const double (&u)[gather_npt<8, BLK_NT>()][8], R (*sW)[Slab<8>::NC]) {
    const int tid = lane_tid();
#pragma unroll
    for (int m = 0; m < gather_npt<8, BLK_NT>(); ++m) {
        // 1,280 cells over 512 threads: a wavefront's cells are all valid or all past the end
        const int c = tid + m * BLK_NT;
        if (c >= Slab<8>::NC) break;
        double w[8];
        cons_to_prim(u[m], w);
#pragma unroll
        for (int v = 0; v < 8; ++v) sW[v][c] = R(w[v]);
    }
}

// Rotate the vector components of a state into the frame of normal direction d (normal first, then the
// other two in cyclic order), d chosen per lane.
template <typename R>
__device__ __forceinline__ void rotate_in(int d, R w[8]) {
#pragma unroll
    for (int base = 1; base <= 4; base += 3) {
        const R x = w[base], y = w[base + 1], z = w[base + 2];
        w[base] = d == 0 ? x : (d == 1 ? y : z);
        w[base + 1] = d == 0 ? y : (d == 1 ? z : x);
        w[base + 2] = d == 0 ? z : (d == 1 ? x : y);
    }
}

// Flux through a face whose direction d (0, 1, 2) is chosen per lane, away from any body cell: the face
// between the cells (i, j, k) - e_d and (i, j, k), block-local. The face states are reconstructed component
// by component (the limiter acts on each component alone) and then rotated into the face-normal frame, so
// one x-normal evaluation serves every direction; fr is the flux in that frame, bbar the face-averaged
// normal field.
template <typename R, int FLUX>
__device__ __forceinline__ void face_flux_any(R (*sW)[Slab<8>::NC], int d, int i, int j, int k, R fr[8], R &bbar) {
    using SL = Slab<8>;
    int c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int o = q - 2;
        c[q] = SL::idx(i + (d == 0 ? o : 0), j + (d == 1 ? o : 0), k + (d == 2 ? o : 0));
    }
    R wl[8], wr[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const R a = sW[v][c[0]], b = sW[v][c[1]], cc = sW[v][c[2]], dd = sW[v][c[3]];
        const R d0 = b - a, d1 = cc - b, d2 = dd - cc;
        wl[v] = b + mc_half(d0, d1);
        wr[v] = cc - mc_half(d1, d2);
    }
    rotate_in(d, wl);
    rotate_in(d, wr);
    num_flux<R, 0, FLUX>(wl, wr, fr);
    bbar = R(0.5) * (wl[4] + wr[4]);
}

// Flux of a face of direction D from the rotated frame of face_flux_any back to x, y, z.
template <int D, typename R>
__device__ __forceinline__ void unrotate(const R fr[8], R f[8]) {
    f[0] = fr[0];
    f[7] = fr[7];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f[1 + (D + a) % 3] = fr[1 + a];
        f[4 + (D + a) % 3] = fr[4 + a];
    }
}

// The value of the next lane (lane + 1) within each row of 16 lanes (DPP row shift; the last lane of a row
// receives its own value).
__device__ __forceinline__ int dpp_next(int x) { return __builtin_amdgcn_update_dpp(x, x, 0x101, 0xf, 0xf, false); }
__device__ __forceinline__ float lane_next(float x) { return __int_as_float(dpp_next(__float_as_int(x))); }
__device__ __forceinline__ double lane_next(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = dpp_next(int(v)), hi = dpp_next(int(v >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double lane_read(double x, int l) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane(int(v), l), hi = __builtin_amdgcn_readlane(int(v >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float lane_read(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// The four face passes, the source and the update of one block whose primitives are in LDS.
template <typename R, int FLUX, bool POWELL>
__device__ __forceinline__ void blk_compute(const Tables &T, const StageArgs &A, int b, R (*sW)[Slab<8>::NC]) {
    using SL = Slab<8>;
    const DevBlock &B = T.blocks[b];
    const DevSim &S = T.sims[B.sim];
    const BitMask mk{nullptr};  // no body cells in these blocks: never read
    const int tid = lane_tid();
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int l = tid & 63, ci = l & 7, cj = l >> 3;
    const double inv_dx = double(1 << B.level) / S.dx0;
    double rhs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double divb = 0.0;
    R f[8], bb;

    // x: the low-x face of each cell; its flux enters the cell and, from the next lane, the cell below
    face_flux<8, R, 0, FLUX, false, false>(T, A, B, b, 0, sW, mk, ci, cj, w, f, bb);
    // the next lane's flux enters with weight inv_dx, or 0 in the last column (its high face comes later)
    const double wx = ci < 7 ? inv_dx : 0.0, wy = cj < 7 ? inv_dx : 0.0;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const R g = lane_next(f[v]);
        rhs[v] = fma(double(f[v]), inv_dx, rhs[v]);
        rhs[v] = fma(-double(g), wx, rhs[v]);
    }
    {
        const R g = lane_next(bb);
        divb = fma(-double(bb), inv_dx, divb);
        divb = fma(double(g), wx, divb);
    }

    // y: the low-y face of each cell; the cell below is eight lanes on
    face_flux<8, R, 1, FLUX, false, false>(T, A, B, b, 0, sW, mk, ci, cj, w, f, bb);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const R g = __shfl_down(f[v], 8, 64);
        rhs[v] = fma(double(f[v]), inv_dx, rhs[v]);
        rhs[v] = fma(-double(g), wy, rhs[v]);
    }
    {
        const R g = __shfl_down(bb, 8, 64);
        divb = fma(-double(bb), inv_dx, divb);
        divb = fma(double(g), wy, divb);
    }

    // high faces: lane (7, j) takes face x = 8 of row j, lane (i, 7) face y = 8 of column i (i < 7; lane
    // (6, 6) takes column 7 for lane (7, 7)), lanes 0-6 and 8 eight faces z = 8 (row j = w of the top face
    // layer); the other lanes repeat face x = 8 of row 0
    R zf[8], zb;
    {
        int d = 0, fi = 8, fj = 0, fk = w;
        if (ci == 7) { fj = cj; }
        else if (cj == 7 || l == 54) { d = 1; fi = cj == 7 ? ci : 7; fj = 8; }
        else if (l < 7 || l == 8) { d = 2; fi = l == 8 ? 7 : l; fj = w; fk = 8; }
        R fr[8], bf;  // the flux in the face-normal frame
        face_flux_any<R, FLUX>(sW, d, fi, fj, fk, fr, bf);
        // the y = 8 face of column 7 moves from lane 54 to lane 63
        R yr[8], yb;
#pragma unroll
        for (int v = 0; v < 8; ++v) yr[v] = lane_read(fr[v], 54);
        yb = lane_read(bf, 54);
        if (ci == 7) {
            R fx[8];
            unrotate<0>(fr, fx);
#pragma unroll
            for (int v = 0; v < 8; ++v) rhs[v] = fma(-double(fx[v]), inv_dx, rhs[v]);
            divb = fma(double(bf), inv_dx, divb);
            if (B.flags & BF_FC) record_fc<0>(T, B, 8, cj, w, fx);
        }
        if (cj == 7) {
            R fy[8];
            if (ci == 7) unrotate<1>(yr, fy);
            else unrotate<1>(fr, fy);
            const R by = ci == 7 ? yb : bf;
#pragma unroll
            for (int v = 0; v < 8; ++v) rhs[v] = fma(-double(fy[v]), inv_dx, rhs[v]);
            divb = fma(double(by), inv_dx, divb);
            if (B.flags & BF_FC) record_fc<1>(T, B, ci, 8, w, fy);
        }
        if (l < 7 || l == 8) {
            unrotate<2>(fr, zf);
            zb = bf;
            if (B.flags & BF_FC) record_fc<2>(T, B, fi, w, 8, zf);
        }
    }
    // past this barrier the x/y halos and the top halo layer (z = 9) are dead: the z fluxes of face layers
    // 1-8 go to the x/y halo space of each variable (64 per layer), their normal field to the top layer
    __syncthreads();
    R *zbar = &sW[0][0] + SL::ZHI + 64;  // [face layer - 1] strided by NC, 64 lanes each
    if (l < 7 || l == 8) {
        const int q = 7 * 64 + w * 8 + (l == 8 ? 7 : l);
#pragma unroll
        for (int v = 0; v < 8; ++v) sW[v][SL::XH + q] = zf[v];
        zbar[7 * SL::NC + w * 8 + (l == 8 ? 7 : l)] = zb;
    }
    face_flux<8, R, 2, FLUX, false, false>(T, A, B, b, 0, sW, mk, ci, cj, w, f, bb);
#pragma unroll
    for (int v = 0; v < 8; ++v) rhs[v] = fma(double(f[v]), inv_dx, rhs[v]);
    divb = fma(-double(bb), inv_dx, divb);
    if (w > 0) {
#pragma unroll
        for (int v = 0; v < 8; ++v) sW[v][SL::XH + (w - 1) * 64 + l] = f[v];
        zbar[(w - 1) * SL::NC + l] = bb;
    }
    __syncthreads();
    double uin[8];
    {
#pragma unroll
        for (int v = 0; v < 8; ++v) rhs[v] = fma(-double(sW[v][SL::XH + w * 64 + l]), inv_dx, rhs[v]);
        divb = fma(double(zbar[w * SL::NC + l]), inv_dx, divb);
        const size_t vs = size_t(T.nb) * 512, off = size_t(b) * 512 + tid;
#pragma unroll
        for (int v = 0; v < 8; ++v) uin[v] = A.Uin[v * vs + off];
    }
    // the bottom halo layers are dead here: the end-of-step reduction uses them
    double *red = reinterpret_cast<double *>(&sW[0][SL::ZLO]);
    int *redi = reinterpret_cast<int *>(&sW[1][SL::ZLO]);
    cell_update<8, R, POWELL, false, BitMask, BLK_NT>(T, A, b, 0, uin, sW, mk, rhs, divb, inv_dx, red, redi);
}

// Wavefronts per SIMD the register allocation is sized for. FP64: four (126 VGPRs; the 80 KiB of LDS
// allow two workgroups per CU anyway). FP32 fluxes: six (80 VGPRs, 60 bytes of spills), so that three
// workgroups of 40 KiB share a CU: 24 wavefronts instead of 16, 9 % faster on the 256^3 magnetosphere
// than four per SIMD at 102 VGPRs; eight per SIMD (64 VGPRs) spills 116 bytes and is 26 % slower.
template <typename R>
constexpr int blk_waves_per_simd() { return sizeof(R) == 8 ? 4 : 6; }

template <typename R, int FLUX, bool POWELL, bool VIEW = false>
__global__ void __launch_bounds__(BLK_NT, (blk_waves_per_simd<R>())) k_stage_blk(Tables T, StageArgs A) {
    using SL = Slab<8>;
    static_assert(SL::NC - SL::XH >= 8 * 64, "z-flux exchange space");
    static_assert(sizeof(R) * 2 * 64 >= sizeof(double) * 8 + sizeof(int) * 8, "reduction space");
    __shared__ R sW[8][SL::NC];
    const int wg = blockIdx.x, xcd = wg & 7, slot = wg >> 3;
    const int b = sched_block(T, A, xcd_first(sched_count(T, A), xcd) + slot);
    {
        double u[gather_npt<8, BLK_NT>()][8];
        gather_issue<8, BLK_NT, VIEW>(T, A, b, 0, u);
        gather_store_blk<R>(u, sW);
    }
    __syncthreads();
    blk_compute<R, FLUX, POWELL>(T, A, b, sW);
}

// Flux-correction target of every face of a level-0 grid C from the same simulations refined everywhere
// (grid F, every block level 1): the mean of the 4 fine face fluxes covering the coarse face minus the
// coarse face flux, per component, with the face-data layout of both grids ([block][3][576][8], face-
// normal frame). The 4 fine faces lie in one child of the coarse block: along the face normal the coarse
// position a (0..8) is the fine position 2a, across it the coarse position t the fine positions 2t and
// 2t + 1; their mean is taken pairwise ((f00 + f10) + (f01 + f11)) / 4 with the first tangential index
// fastest, in FP64 without contraction, and rounded to FP32. One workgroup per coarse block, one thread per
// face of each direction.
__global__ void __launch_bounds__(576) k_face_targets(Tables F, const float *__restrict__ Ff, Tables C,
                                                      const float *__restrict__ Fc, float *__restrict__ Tout) {
#pragma clang fp contract(off)
    const int c = blockIdx.x, f = threadIdx.x;
    const DevBlock &B = C.blocks[c];
    const DevSim &S = F.sims[B.sim];
#pragma unroll
    for (int D = 0; D < 3; ++D) {
        int q[3];  // coarse face coordinates (x, y, z), the one along D in 0..8
        if (D == 0) { q[0] = f % 9; q[1] = (f / 9) & 7; q[2] = f / 72; }
        else if (D == 1) { q[0] = f & 7; q[1] = (f >> 3) % 9; q[2] = f / 72; }
        else { q[0] = f & 7; q[1] = (f >> 3) & 7; q[2] = f >> 6; }
        const int a1 = D == 0 ? 1 : 0, a2 = D == 2 ? 1 : 2;  // tangential axes, the first one fastest
        int child[3], fq[3];
        {
            const int g = 2 * q[D];
            child[D] = g >= 8 ? 1 : 0;
            fq[D] = g - 8 * child[D];
        }
        child[a1] = q[a1] >> 2;
        fq[a1] = 2 * q[a1] - 8 * child[a1];
        child[a2] = q[a2] >> 2;
        fq[a2] = 2 * q[a2] - 8 * child[a2];
        const int32_t fb = lut_at(F, S, 1, 2LL * B.ijk[0] + child[0], 2LL * B.ijk[1] + child[1],
                                  2LL * B.ijk[2] + child[2]);
        const float *src[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            int p[3] = {fq[0], fq[1], fq[2]};
            p[a1] += m & 1;
            p[a2] += m >> 1;
            const int idx = D == 0 ? face_index<0>(p[0], p[1], p[2])
                                   : (D == 1 ? face_index<1>(p[0], p[1], p[2]) : face_index<2>(p[0], p[1], p[2]));
            src[m] = Ff + ((size_t(fb) * 3 + D) * 576 + idx) * 8;
        }
        const size_t o = ((size_t(c) * 3 + D) * 576 + f) * 8;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const double mean = ((double(src[0][v]) + double(src[1][v])) + (double(src[2][v]) + double(src[3][v]))) * 0.25;
            Tout[o + v] = float(mean - double(Fc[o + v]));
        }
    }
}

// Per-face training data of a whole block (one workgroup of 576 threads = one face per thread and
// direction): stencil features in the face-normal frame (optionally z-scored) and the plain flux in the
// face-normal frame, FP64 arithmetic.
template <int FLUX>
__global__ void __launch_bounds__(Slab<8>::NT) k_face_data(Tables T, StageArgs A, const float *__restrict__ stats,
                                                           float *__restrict__ X, float *__restrict__ F) {
    using SL = Slab<8>;
    __shared__ double sW[8][SL::NC];
    __shared__ unsigned char sM[SL::NC];
    const int b = blockIdx.x;
    double u[SL::NPT][8];
    gather_issue<8>(T, A, b, 0, u);
    gather_store<8, double>(T, b, 0, u, sW, sM);
    __syncthreads();
    const DevBlock &B = T.blocks[b];
    const bool near_body = (B.flags & BF_NEAR_BODY) != 0;
    const int f = lane_tid();
    if (f >= 576) return;
#pragma unroll
    for (int D = 0; D < 3; ++D) {
        int i, j, k;
        if (D == 0) { i = f % 9; j = (f / 9) & 7; k = f / 72; }
        else if (D == 1) { i = f & 7; j = (f >> 3) % 9; k = f / 72; }
        else { i = f & 7; j = (f >> 3) & 7; k = f >> 6; }
        int c[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int o = q - 2;
            c[q] = D == 0 ? SL::idx(i + o, j, k) : (D == 1 ? SL::idx(i, j + o, k) : SL::idx(i, j, k + o));
        }
        const size_t g = (size_t(b) * 3 + D) * 576 + f;
        if (X) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float x[8];
                x[0] = float(sW[0][c[q]]);
                x[7] = float(sW[7][c[q]]);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    x[1 + a] = float(sW[1 + (D + a) % 3][c[q]]);
                    x[4 + a] = float(sW[4 + (D + a) % 3][c[q]]);
                }
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const int e = q * 8 + v;
                    X[g * 32 + e] = stats ? (x[v] - stats[e]) / stats[32 + e] : x[v];
                }
            }
        }
        if (F) {
            double wl[8], wr[8], fl[8];
            const bool m0 = near_body && sM[c[0]], m1 = near_body && sM[c[1]];
            const bool m2 = near_body && sM[c[2]], m3 = near_body && sM[c[3]];
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const double a = sW[v][c[0]], bb = sW[v][c[1]], cc = sW[v][c[2]], d = sW[v][c[3]];
                const double d0 = bb - a, d1 = cc - bb, d2 = d - cc;
                const double hl = (m0 || m2) ? 0.0 : mc_half(d0, d1), hr = (m1 || m3) ? 0.0 : mc_half(d1, d2);
                wl[v] = bb + hl;
                wr[v] = cc - hr;
            }
            if (m2 && !m1) {
#pragma unroll
                for (int v = 0; v < 8; ++v) wr[v] = wl[v];
                wr[1 + D] = -wl[1 + D];
            } else if (m1 && !m2) {
#pragma unroll
                for (int v = 0; v < 8; ++v) wl[v] = wr[v];
                wl[1 + D] = -wr[1 + D];
            }
            if (D == 0) num_flux<double, 0, FLUX>(wl, wr, fl);
            else if (D == 1) num_flux<double, 1, FLUX>(wl, wr, fl);
            else num_flux<double, 2, FLUX>(wl, wr, fl);
            if (m1 && m2) {
#pragma unroll
                for (int v = 0; v < 8; ++v) fl[v] = 0.0;
            }
            F[g * 8 + 0] = float(fl[0]);
            F[g * 8 + 7] = float(fl[7]);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                F[g * 8 + 1 + a] = float(fl[1 + (D + a) % 3]);
                F[g * 8 + 4 + a] = float(fl[4 + (D + a) % 3]);
            }
        }
    }
}

// Z-scored stencil features of the faces of a block for the learned correction's inference, in the
// compact face layout (see lrn_y_at), FP32 primitives in LDS (40 KB per block, so several blocks per CU); each
// thread takes one stencil cell of a face at a time (8 features), so a wavefront's stores cover
// contiguous memory. TX = __bf16 stores the features rounded as the BF16 network consumes them (half
// the bytes); TX = float keeps them for the FP32 network.
template <typename TX>
__global__ void __launch_bounds__(Slab<8>::NT) k_face_features(Tables T, StageArgs A, const float *__restrict__ stats,
                                                               TX *__restrict__ X) {
    using SL = Slab<8>;
    __shared__ float sW[8][SL::NC];
    __shared__ unsigned char sM[SL::NC];
    __shared__ float sMean[32], sInv[32];
    const int b = blockIdx.x;
    if (threadIdx.x < 32) {
        sMean[threadIdx.x] = stats[threadIdx.x];
        sInv[threadIdx.x] = 1.0f / stats[32 + threadIdx.x];
    }
    double u[SL::NPT][8];
    gather_issue<8>(T, A, b, 0, u);
    gather_store<8, float>(T, b, 0, u, sW, sM);
    __syncthreads();
    // task t = 4 f + q: stencil cell q of face f of the compact layout (each face once: the block's low
    // faces, then its high face planes with no neighbour across them), so consecutive lanes write
    // consecutive 32-byte pieces
    const DevBlock &B = T.blocks[b];
    const int tid = lane_tid();
#pragma unroll
    for (int D = 0; D < 3; ++D) {
        const bool hb = B.hb_pos[D] >= 0;
        const int ntask = hb ? 4 * (512 + 64) : 4 * 512;
        for (int t = tid; t < ntask; t += SL::NT) {
            const int f = t >> 2, q = t & 3;
            int p[3];  // face coordinates (x, y, z), the one along D in 0..8
            size_t row;
            if (f < 512) {
                p[0] = f & 7; p[1] = (f >> 3) & 7; p[2] = f >> 6;
                row = size_t(b) * 1536 + D * 512 + f;
            } else {
                const int h = f - 512, t1 = h & 7, t2 = h >> 3;
                p[D] = 8;
                p[D == 0 ? 1 : 0] = t1;
                p[D == 2 ? 1 : 2] = t2;
                row = size_t(T.nb) * 1536 + size_t(B.hb_pos[D]) * 64 + h;
            }
            const int o = q - 2;
            const int c = D == 0 ? SL::idx(p[0] + o, p[1], p[2]) : (D == 1 ? SL::idx(p[0], p[1] + o, p[2]) : SL::idx(p[0], p[1], p[2] + o));
            float x[8];
            x[0] = sW[0][c];
            x[7] = sW[7][c];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                x[1 + a] = sW[1 + (D + a) % 3][c];
                x[4 + a] = sW[4 + (D + a) % 3][c];
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) x[v] = (x[v] - sMean[q * 8 + v]) * sInv[q * 8 + v];
            TX *dst = X + row * 32 + q * 8;
            if constexpr (std::is_same<TX, __bf16>::value) {
                typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
                bf16x8_t hv;
#pragma unroll
                for (int v = 0; v < 8; ++v) hv[v] = __bf16(x[v]);
                *reinterpret_cast<bf16x8_t *>(dst) = hv;
            } else {
                float4 *out = reinterpret_cast<float4 *>(dst);
                out[0] = make_float4(x[0], x[1], x[2], x[3]);
                out[1] = make_float4(x[4], x[5], x[6], x[7]);
            }
        }
    }
}

// Learned-correction fallback: every face with a flagged cell on either side loses its learned
// increment on both sides (cell-centric, so each thread only writes its own cell). At the end of a step
// it also counts non-positive cells.
__global__ void __launch_bounds__(512) k_learn_fixup(Tables T, StageArgs A, int32_t *fallback_cells) {
    __shared__ double red[8];
    __shared__ int redi[8];
    const int b = blockIdx.x, c = threadIdx.x;
    const DevBlock &B = T.blocks[b];
    const DevSim &S = T.sims[B.sim];
    const size_t vs = size_t(T.nb) * 512, off = size_t(b) * 512 + c;
    const int ii[3] = {c & 7, (c >> 3) & 7, c >> 6};
    const bool near_body = (B.flags & BF_NEAR_BODY) != 0;
    const bool body = near_body && in_body(S, B.level, B.ijk, ii[0], ii[1], ii[2]);
    const bool self = A.lrn_flags[off] != 0;
    // faces whose learned increment the cell gives back: those with a flagged cell on either side and no
    // body cell across them (almost always none, and the cell's state is then read only to count faults)
    unsigned undo = 0;
    if (!body) {
#pragma unroll
        for (int fd = 0; fd < 6; ++fd) {
            const int a = fd >> 1, side = fd & 1;
            int nn[3] = {ii[0], ii[1], ii[2]};
            nn[a] += side ? 1 : -1;
            int nblk = b;
            if (nn[a] < 0 || nn[a] > 7) {
                nblk = B.face[fd];
                nn[a] &= 7;
            }
            bool other = false, nbody = false;
            if (nblk >= 0) {
                const DevBlock &NB = T.blocks[nblk];
                other = A.lrn_flags[size_t(nblk) * 512 + (nn[2] * 8 + nn[1]) * 8 + nn[0]] != 0;
                nbody = (NB.flags & BF_NEAR_BODY) && in_body(S, NB.level, NB.ijk, nn[0], nn[1], nn[2]);
            }
            if (!nbody && (self || other)) undo |= 1u << fd;
        }
    }
    double u[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (undo || (A.count_faults && !body)) {
#pragma unroll
        for (int v = 0; v < 8; ++v) u[v] = A.Uout[v * vs + off];
    }
    if (undo) {
        const double bdt = A.beta * A.dt[B.sim], inv_dx = double(1 << B.level) / S.dx0;
#pragma unroll
        for (int fd = 0; fd < 6; ++fd) {
            if (!((undo >> fd) & 1)) continue;
            const int a = fd >> 1, side = fd & 1;
            int fi[3] = {ii[0], ii[1], ii[2]};
            fi[a] += side;  // face index along a: the cell's own index (minus face) or one more (plus face)
            const float *y = a == 0 ? lrn_y_at<0>(T, A, b, fi[0], fi[1], fi[2])
                                    : (a == 1 ? lrn_y_at<1>(T, A, b, fi[0], fi[1], fi[2]) : lrn_y_at<2>(T, A, b, fi[0], fi[1], fi[2]));
            double dF[8];
            if (a == 0) learned_increment<double, 0>(y, A.lrn_stats, dF);
            else if (a == 1) learned_increment<double, 1>(y, A.lrn_stats, dF);
            else learned_increment<double, 2>(y, A.lrn_stats, dF);
            const double sg = side ? 1.0 : -1.0;
#pragma unroll
            for (int v = 0; v < 8; ++v) u[v] += bdt * sg * dF[v] * inv_dx;
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) A.Uout[v * vs + off] = u[v];
    }
    int nf = 0;
    if (A.count_faults && !body) {
        double w[8];
        cons_to_prim(u, w);
        nf = !(w[0] > 0.0) || !(w[7] > 0.0) || !(w[7] < INFINITY);
    }
    block_publish<512>(0.0, nf, red, redi, nullptr, A.faults);
    if (fallback_cells) {
        // reuse the reduction for the flagged-cell count
        __syncthreads();
        block_publish<512>(0.0, self ? 1 : 0, red, redi, nullptr, fallback_cells);
    }
}

// coarse cells at coarse-fine faces: swap the coarse flux for the mean of the four fine fluxes. A body
// cell on such a face is never updated and never enters dt or the fault count.
__global__ void __launch_bounds__(256) k_flux_correct(Tables T, StageArgs A) {
    __shared__ double red[4];
    __shared__ int redi[4];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const DevFcCell *cells = A.fc_list ? A.fc_list : T.fc_cells;
    const int ncells = A.fc_list ? A.n_fc_list : T.n_fc_cells;
    double lam = 0.0;
    int nf = 0;
    int sim = 0;
    bool body = false;
    if (e < ncells) {
        const DevFcCell C = cells[e];
        const DevBlock &B = T.blocks[C.block];
        const DevSim &S = T.sims[B.sim];
        sim = B.sim;
        body = (B.flags & BF_NEAR_BODY) && in_body(S, B.level, B.ijk, C.cell & 7, (C.cell >> 3) & 7, C.cell >> 6);
    }
    if (e < ncells && !body) {
        const DevFcCell C = cells[e];
        const DevBlock &B = T.blocks[C.block];
        const DevSim &S = T.sims[B.sim];
        const size_t vs = size_t(T.nb) * 512, off = size_t(C.block) * 512 + C.cell;
        const double inv_dx = 1.0 / S.dx0;
        const double bdt = A.beta * (A.local_dt ? A.dt[off] : A.dt[B.sim]);
        double u[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) u[v] = A.Uout[v * vs + off];
        for (int m = 0; m < C.n; ++m) {
            const double *rec = T.fcbuf + size_t(C.rec[m]) * FC_REC;
            const int t1 = C.t[m] & 7, t2 = C.t[m] >> 3;
            const double sg = (C.face[m] & 1) ? 1.0 : -1.0;
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                const double fc = rec[v * 64 + t2 * 8 + t1];
                const double *fn = rec + FC_COARSE + v * 256 + (2 * t2) * 16 + 2 * t1;
                const double fm = ((fn[0] + fn[1]) + (fn[16] + fn[17])) * 0.25;
                u[v] += bdt * sg * (fc - fm) * inv_dx;
            }
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) A.Uout[v * vs + off] = u[v];
        if (A.count_faults || A.want_lam) {
            double w[8];
            cons_to_prim(u, w);
            nf = !(w[0] > 0.0) || !(w[7] > 0.0) || !(w[7] < INFINITY);
            if (A.want_lam) lam = cell_bound(w, inv_dx);
        }
    }
    if (A.want_lam) {
        // a grid may mix simulations inside one workgroup here: publish per thread (few cells)
        if (e < ncells && !body) publish_max(T.lam + sim, lam);
    }
    if (A.count_faults) block_publish<256>(0.0, nf, red, redi, nullptr, A.faults);
}

}  // namespace bmhd

// ================================================================================================
// C ABI

using namespace bmhd;

bmhd_grid::~bmhd_grid() {
    if (h.graph_exec) (void)hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(h.graph_exec));
    if (h.graph) (void)hipGraphDestroy(reinterpret_cast<hipGraph_t>(h.graph));
    if (h.capture_stream) (void)hipStreamDestroy(reinterpret_cast<hipStream_t>(h.capture_stream));
    if (h.fork_event) (void)hipEventDestroy(reinterpret_cast<hipEvent_t>(h.fork_event));
    if (h.join_event) (void)hipEventDestroy(reinterpret_cast<hipEvent_t>(h.join_event));
    if (h.side_stream) (void)hipStreamDestroy(reinterpret_cast<hipStream_t>(h.side_stream));
}

namespace {
thread_local std::string g_err;

int32_t fail(int32_t code, const std::string &msg) {
    g_err = msg;
    return code;
}

int32_t hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return BMHD_OK;
    return fail(BMHD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int32_t launch_check(const char *what) { return hip_check(hipGetLastError(), what); }

int32_t record_event(void *ev, hipStream_t s) {
    return ev ? hip_check(hipEventRecord(reinterpret_cast<hipEvent_t>(ev), s), "event") : BMHD_OK;
}

bool ptr_ok(const void *p) { return p && (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

// The side stream for work that may run beside the next launch on s: the grid's side stream, made to wait
// for everything enqueued on s so far, or s itself while s is being captured into a graph (the launches
// then stay in order on s). join_side makes s wait for what was enqueued on the side stream.
int32_t fork_side(const HostGrid &h, hipStream_t s, hipStream_t &side) {
    side = s;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (int32_t rc = hip_check(hipStreamIsCapturing(s, &cs), "capture status")) return rc;
    if (cs != hipStreamCaptureStatusNone) return BMHD_OK;
    if (!h.side_stream) {  // all three or none
        hipStream_t ss = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        int32_t rc = hip_check(hipStreamCreateWithFlags(&ss, hipStreamNonBlocking), "side stream");
        if (!rc) rc = hip_check(hipEventCreateWithFlags(&e0, hipEventDisableTiming), "fork event");
        if (!rc) rc = hip_check(hipEventCreateWithFlags(&e1, hipEventDisableTiming), "join event");
        if (rc) {
            if (e0) (void)hipEventDestroy(e0);
            if (ss) (void)hipStreamDestroy(ss);
            return rc;
        }
        h.side_stream = ss;
        h.fork_event = e0;
        h.join_event = e1;
    }
    hipStream_t ss = reinterpret_cast<hipStream_t>(h.side_stream);
    hipEvent_t e0 = reinterpret_cast<hipEvent_t>(h.fork_event);
    if (int32_t rc = hip_check(hipEventRecord(e0, s), "fork")) return rc;
    if (int32_t rc = hip_check(hipStreamWaitEvent(ss, e0, 0), "fork wait")) return rc;
    side = ss;
    return BMHD_OK;
}

int32_t join_side(const HostGrid &h, hipStream_t s, hipStream_t side) {
    if (side == s) return BMHD_OK;
    hipEvent_t e1 = reinterpret_cast<hipEvent_t>(h.join_event);
    if (int32_t rc = hip_check(hipEventRecord(e1, side), "join")) return rc;
    return hip_check(hipStreamWaitEvent(s, e1, 0), "join wait");
}

// Launch shape of the stage kernel: work split (face per thread or wave per cell layer), tile depth (4
// or 8 cells) and persistent grid size (0: one workgroup per slab).
struct Shape {
    int scheme;
    int ks;
    int persist_wgs;
};

template <int KS, typename R, int FLUX, bool POWELL>
int32_t launch_stage_shape(const HostGrid &h, const StageArgs &a, int scheme, int persist_wgs, void *ev0, void *ev1,
                           hipStream_t s, const double *halo_in) {
    constexpr int nt = Slab<KS>::NT;
    const int items = h.nb * (8 / KS);
    int grid = items;
    if (persist_wgs > 0) {
        grid = persist_wgs < items ? persist_wgs : items;
        grid = (grid + 7) & ~7;
    }
    if (scheme == BMHD_SCHEME_BLOCK) {
        // Blocks clear of any body on the block form (the dominant launch) and blocks near a body on the
        // plane form; with split_level, the clear blocks with a face on another level are launched apart
        // once the level-change halo fill (halo_in: its input; null when the caller has enqueued it
        // already) is done, and the others at once. The launches that wait for the halo fill, and the few
        // workgroups near a body, go to a side stream beside the first launch, which would otherwise wait
        // for them with most of the chip idle. The launches write disjoint blocks of the output. The
        // events bracket the first launch alone.
        const int np = h.n_clear_plain, nc = h.n_clear, nl = nc - np, nn = h.nb - nc;
        StageArgs ap = a, al = a, an = a;
        ap.sched = h.dev.order_split;
        ap.n_sched = np;
        al.sched = h.dev.order_split + np;
        al.n_sched = nl;
        an.sched = h.dev.order_split + nc;
        an.n_sched = nn;
        const bool halo = halo_in && !h.halo_items.empty();
        if (halo && !h.split_level) {  // every clear block may read the halo buffer: fill it first
            k_halo_fill<<<unsigned(h.halo_items.size()), 256, 0, s>>>(h.dev, halo_in);
            if (int32_t rc = launch_check("level-change halo fill")) return rc;
        }
        hipStream_t side = s;
        if (np && ((halo && h.split_level) || nl || nn))
            if (int32_t rc = fork_side(h, s, side)) return rc;
        if (halo && h.split_level) {
            k_halo_fill<<<unsigned(h.halo_items.size()), 256, 0, side>>>(h.dev, halo_in);
            if (int32_t rc = launch_check("level-change halo fill")) return rc;
        }
        if (nn) {
            k_stage_wp<4, R, FLUX, POWELL, false><<<nn * 2, Slab<4>::NT, 0, side>>>(h.dev, an);
            if (int32_t rc = launch_check("stage kernel (blocks near a body)")) return rc;
        }
        if (nl) {
            k_stage_blk<R, FLUX, POWELL><<<nl, BLK_NT, 0, side>>>(h.dev, al);
            if (int32_t rc = launch_check("stage kernel (blocks at a level change)")) return rc;
        }
        if (int32_t rc = record_event(ev0, s)) return rc;
        if (np) k_stage_blk<R, FLUX, POWELL><<<np, BLK_NT, 0, s>>>(h.dev, ap);
        if (int32_t rc = record_event(ev1, s)) return rc;
        if (int32_t rc = launch_check("stage kernel")) return rc;
        return join_side(h, s, side);
    }
    if (halo_in && !h.halo_items.empty()) {
        k_halo_fill<<<unsigned(h.halo_items.size()), 256, 0, s>>>(h.dev, halo_in);
        if (int32_t rc = launch_check("level-change halo fill")) return rc;
    }
    if (int32_t rc = record_event(ev0, s)) return rc;
    if (scheme == BMHD_SCHEME_PLANE) {
        if (persist_wgs > 0) k_stage_wp<KS, R, FLUX, POWELL, true><<<grid, nt, 0, s>>>(h.dev, a);
        else k_stage_wp<KS, R, FLUX, POWELL, false><<<grid, nt, 0, s>>>(h.dev, a);
    } else {
        if (persist_wgs > 0) k_stage<KS, R, FLUX, POWELL, true><<<grid, nt, 0, s>>>(h.dev, a);
        else k_stage<KS, R, FLUX, POWELL, false><<<grid, nt, 0, s>>>(h.dev, a);
    }
    if (int32_t rc = record_event(ev1, s)) return rc;
    return launch_check("stage kernel");
}

template <int KS, typename R>
int32_t launch_stage_prec(const HostGrid &h, const StageArgs &a, int flux, bool powell, const Shape &sh, void *ev0,
                          void *ev1, hipStream_t s, const double *halo_in) {
    const int sc = sh.scheme, pw = sh.persist_wgs;
    if (flux == BMHD_FLUX_RUSANOV) {
        if (powell) return launch_stage_shape<KS, R, BMHD_FLUX_RUSANOV, true>(h, a, sc, pw, ev0, ev1, s, halo_in);
        return launch_stage_shape<KS, R, BMHD_FLUX_RUSANOV, false>(h, a, sc, pw, ev0, ev1, s, halo_in);
    }
    if (flux == BMHD_FLUX_LINDE) {
        if (powell) return launch_stage_shape<KS, R, BMHD_FLUX_LINDE, true>(h, a, sc, pw, ev0, ev1, s, halo_in);
        return launch_stage_shape<KS, R, BMHD_FLUX_LINDE, false>(h, a, sc, pw, ev0, ev1, s, halo_in);
    }
    if (powell) return launch_stage_shape<KS, R, BMHD_FLUX_HLLE, true>(h, a, sc, pw, ev0, ev1, s, halo_in);
    return launch_stage_shape<KS, R, BMHD_FLUX_HLLE, false>(h, a, sc, pw, ev0, ev1, s, halo_in);
}

Shape pick_shape(const bmhd_opts &o) {
    Shape sh;
    // measured on the 256^3 magnetosphere: the block form in both precisions (FP64: 1.25 / 1.40 ms per
    // stage against 1.74 / 2.07 for the plane form on 8x8x4 slabs and 1.91 / 2.16 for the face form on
    // full blocks; FP32 flux: 0.94 / 1.14 against 1.04 / 1.26). A persistent grid or a tile of four
    // layers asks for the plane form, and so does the Linde-type flux (its block form does not fit 128
    // registers: 4.46 against 3.98 ms per step on the same grid). With the face form, full blocks for FP64.
    if (o.scheme == 0)
        sh.scheme = (o.persist_wgs > 0 || o.slab == 4 || o.flux == BMHD_FLUX_LINDE) ? BMHD_SCHEME_PLANE : BMHD_SCHEME_BLOCK;
    else sh.scheme = o.scheme;
    sh.ks = o.slab == 0 ? ((o.precision == BMHD_FP64 && sh.scheme == BMHD_SCHEME_FACE) || sh.scheme == BMHD_SCHEME_BLOCK
                               ? 8 : 4)
                        : o.slab;
    sh.persist_wgs = o.persist_wgs;
    return sh;
}

// The stage kernel of the chosen shape; ev0 / ev1 (hipEvent_t, may be null) are recorded right before and
// after the dominant kernel.
// The stage kernels of one stage; halo_in, when not null, is the input of the level-change halo fill, which
// the launches then enqueue themselves ahead of the blocks that read it.
int32_t launch_stage(const HostGrid &h, const StageArgs &a, const bmhd_opts &o, void *ev0, void *ev1, hipStream_t s,
                     const double *halo_in) {
    const Shape sh = pick_shape(o);
    if (o.precision == BMHD_FP64) {
        if (sh.ks == 4) return launch_stage_prec<4, double>(h, a, o.flux, o.powell, sh, ev0, ev1, s, halo_in);
        return launch_stage_prec<8, double>(h, a, o.flux, o.powell, sh, ev0, ev1, s, halo_in);
    }
    if (sh.ks == 4) return launch_stage_prec<4, float>(h, a, o.flux, o.powell, sh, ev0, ev1, s, halo_in);
    return launch_stage_prec<8, float>(h, a, o.flux, o.powell, sh, ev0, ev1, s, halo_in);
}

template <typename R, int FLUX>
int32_t launch_learn_flux(const HostGrid &h, const StageArgs &a, bool powell, hipStream_t s) {
    constexpr int nt = Slab<4>::NT;
    if (powell) k_stage_wp<4, R, FLUX, true, false, true><<<h.nb * 2, nt, 0, s>>>(h.dev, a);
    else k_stage_wp<4, R, FLUX, false, false, true><<<h.nb * 2, nt, 0, s>>>(h.dev, a);
    return launch_check("learned stage kernel");
}

int32_t launch_learn(const HostGrid &h, const StageArgs &a, const bmhd_opts &o, hipStream_t s) {
    if (o.precision == BMHD_FP64) {
        if (o.flux == BMHD_FLUX_RUSANOV) return launch_learn_flux<double, BMHD_FLUX_RUSANOV>(h, a, o.powell, s);
        return launch_learn_flux<double, BMHD_FLUX_HLLE>(h, a, o.powell, s);
    }
    if (o.flux == BMHD_FLUX_RUSANOV) return launch_learn_flux<float, BMHD_FLUX_RUSANOV>(h, a, o.powell, s);
    return launch_learn_flux<float, BMHD_FLUX_HLLE>(h, a, o.powell, s);
}

int32_t check_opts(const bmhd_opts &o) {
    if (o.flux != BMHD_FLUX_RUSANOV && o.flux != BMHD_FLUX_HLLE && o.flux != BMHD_FLUX_LINDE)
        return fail(BMHD_EINVAL, "unknown flux");
    if (o.precision != BMHD_FP64 && o.precision != BMHD_FP32_FLUX) return fail(BMHD_EINVAL, "unknown precision");
    if (o.slab != 0 && o.slab != 4 && o.slab != 8) return fail(BMHD_EINVAL, "slab must be 0, 4 or 8");
    if (o.scheme != 0 && o.scheme != BMHD_SCHEME_FACE && o.scheme != BMHD_SCHEME_PLANE && o.scheme != BMHD_SCHEME_BLOCK)
        return fail(BMHD_EINVAL, "unknown scheme");
    if (o.scheme == BMHD_SCHEME_BLOCK && (o.slab == 4 || o.persist_wgs != 0))
        return fail(BMHD_EUNSUPPORTED, "the block scheme takes whole blocks, one workgroup each");
    if (o.persist_wgs < 0 || o.persist_wgs > (1 << 20)) return fail(BMHD_EINVAL, "persist_wgs out of range");
    if (o.recompute_dt && !(o.cfl > 0.0)) return fail(BMHD_EINVAL, "cfl must be positive");
    if (o.learned) {
        const bmhd_learned &L = *o.learned;
        if (L.hidden != 32 && L.hidden != 64 && L.hidden != 128) return fail(BMHD_EINVAL, "learned: hidden must be 32, 64 or 128");
        if (L.mode != 0 && L.mode != 1 && L.mode != 2) return fail(BMHD_EINVAL, "learned: mode must be 0, 1 or 2");
        if (!L.stats || !L.y_buf || !L.flags || (L.mode != 2 && (!L.params || !L.params_bf16 || !L.x_buf)))
            return fail(BMHD_EINVAL, "learned: null buffer");
        if (L.mode == 0 && (reinterpret_cast<uintptr_t>(L.x_buf) & 15u))
            return fail(BMHD_EINVAL, "learned: x_buf must be 16-byte aligned");
        if (!(L.tau >= 0.0)) return fail(BMHD_EINVAL, "learned: tau must be >= 0");
        if (!(L.floor_rel >= 0.0)) return fail(BMHD_EINVAL, "learned: floor_rel must be >= 0");
        if (o.use_graph) return fail(BMHD_EUNSUPPORTED, "learned correction is not captured in graphs");
        if (o.local_dt) return fail(BMHD_EUNSUPPORTED, "learned correction with local time stepping");
        if (o.flux == BMHD_FLUX_LINDE) return fail(BMHD_EUNSUPPORTED, "learned correction is added to the HLLE or Rusanov flux");
    }
    if (o.local_dt != 0 && o.local_dt != 1) return fail(BMHD_EINVAL, "local_dt must be 0 or 1");
    return BMHD_OK;
}

// One stage for a subset of blocks whose ghost cells come from a padded view (one process after the
// ghost exchange between processes): the block form for the subset's blocks clear of a body and the plane
// form for the others (the plane form for all of them with the Linde-type flux, as in bmhd_advance). No
// level-change halos (the view holds every ghost cell), no flux correction (flux_correct_subset, once the
// stage has run for every process) and no next-dt bound.
template <typename R, int FLUX, bool POWELL>
int32_t launch_view_stage(const HostGrid &h, const StageArgs &a, const ViewStage &v, hipStream_t s) {
    StageArgs ac = a, an = a;
    if constexpr (FLUX == BMHD_FLUX_LINDE) {
        an.sched = v.split;
        an.n_sched = v.n_total;
        if (v.n_total) k_stage_wp<4, R, FLUX, POWELL, false, false, true><<<v.n_total * 2, Slab<4>::NT, 0, s>>>(h.dev, an);
        return launch_check("stage kernel");
    } else {
        const int nn = v.n_total - v.n_clear;
        ac.sched = v.split;
        ac.n_sched = v.n_clear;
        an.sched = v.split + v.n_clear;
        an.n_sched = nn;
        if (nn) k_stage_wp<4, R, FLUX, POWELL, false, false, true><<<nn * 2, Slab<4>::NT, 0, s>>>(h.dev, an);
        if (v.n_clear) k_stage_blk<R, FLUX, POWELL, true><<<v.n_clear, BLK_NT, 0, s>>>(h.dev, ac);
        return launch_check("stage kernel");
    }
}

template <typename R, int FLUX>
int32_t launch_view_stage_p(const HostGrid &h, const StageArgs &a, const ViewStage &v, bool powell, hipStream_t s) {
    return powell ? launch_view_stage<R, FLUX, true>(h, a, v, s) : launch_view_stage<R, FLUX, false>(h, a, v, s);
}

template <typename R>
int32_t launch_view_stage_f(const HostGrid &h, const StageArgs &a, const ViewStage &v, const bmhd_opts &o, hipStream_t s) {
    if (o.flux == BMHD_FLUX_RUSANOV) return launch_view_stage_p<R, BMHD_FLUX_RUSANOV>(h, a, v, o.powell, s);
    if (o.flux == BMHD_FLUX_LINDE) return launch_view_stage_p<R, BMHD_FLUX_LINDE>(h, a, v, o.powell, s);
    return launch_view_stage_p<R, BMHD_FLUX_HLLE>(h, a, v, o.powell, s);
}

int32_t check_view_stage(const HostGrid &h, int e, const bmhd_opts &o) {
    if (!h.d_work) return fail(BMHD_EINVAL, "grid not uploaded (call bmhd_grid_upload first)");
    if (e != 0 && e != 1) return fail(BMHD_EINVAL, "stage must be 0 or 1");
    if (int32_t rc = check_opts(o)) return rc;
    if (o.learned || o.local_dt || o.persist_wgs)
        return fail(BMHD_EUNSUPPORTED, "the stage from an exchanged view takes no learned correction, local time "
                                       "stepping or persistent grid");
    return BMHD_OK;
}

int32_t stage_from_view_impl(const HostGrid &h, const ViewStage &v, int e, const double *U0, const double *Uin,
                             double *Uout, const double *dt, const bmhd_opts &o, int32_t *faults, void *stream) {
    if (int32_t rc = check_view_stage(h, e, o)) return rc;
    if (v.n_total == 0) return BMHD_OK;
    StageArgs a;
    std::memset(&a, 0, sizeof a);
    a.Uin = Uin;
    a.U0 = U0;
    a.Uout = Uout;
    a.dt = const_cast<double *>(dt);  // read only: no local stepping here
    a.faults = faults;
    a.alpha = o.alpha[e];
    a.beta = o.beta[e];
    a.use_u0 = o.alpha[e] != 0.0 ? 1 : 0;
    a.count_faults = (e == 1 && faults) ? 1 : 0;
    a.view = v.view;
    a.view_local = v.view_local;
    a.view_faces = v.view_faces;
    a.view_vs = v.view_vs;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (o.precision == BMHD_FP64) return launch_view_stage_f<double>(h, a, v, o, s);
    return launch_view_stage_f<float>(h, a, v, o, s);
}

int32_t flux_correct_subset_impl(const HostGrid &h, const ViewStage &v, int e, double *Uout, const double *dt,
                                 const bmhd_opts &o, int32_t *faults, void *stream) {
    if (int32_t rc = check_view_stage(h, e, o)) return rc;
    if (v.n_fc == 0) return BMHD_OK;
    StageArgs a;
    std::memset(&a, 0, sizeof a);
    a.Uout = Uout;
    a.dt = const_cast<double *>(dt);
    a.faults = faults;
    a.beta = o.beta[e];
    a.count_faults = (e == 1 && faults) ? 1 : 0;
    a.fc_list = v.fc_cells;
    a.n_fc_list = v.n_fc;
    k_flux_correct<<<unsigned((v.n_fc + 255) / 256), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(h.dev, a);
    return launch_check("flux correction");
}

// One stage: level-change halos, the stage kernel (optionally bracketed by events), flux correction.
// With the learned correction: face features, the MLP, the corrected stage, and the fallback.
int32_t enqueue_stage(const HostGrid &h, const bmhd_opts &o, int e, double *d_U0, double *d_U1, double *d_dt,
                      int32_t *d_faults, bool want_lam, void *ev0, void *ev1, hipStream_t s) {
    const double *in = e ? d_U1 : d_U0;
    double *out = e ? d_U0 : d_U1;
    // the plain stage enqueues the level-change halo fill with its launches (beside the blocks that do not
    // read it); the learned form fills it first
    if (!h.halo_items.empty() && o.learned) k_halo_fill<<<unsigned(h.halo_items.size()), 256, 0, s>>>(h.dev, in);
    StageArgs a;
    std::memset(&a, 0, sizeof a);
    a.Uin = in;
    a.U0 = d_U0;
    a.Uout = out;
    a.dt = d_dt;
    a.faults = d_faults;
    a.alpha = o.alpha[e];
    a.beta = o.beta[e];
    a.use_u0 = o.alpha[e] != 0.0 ? 1 : 0;
    a.want_lam = want_lam ? 1 : 0;
    a.count_faults = (e == 1 && d_faults) ? 1 : 0;
    if (o.local_dt) {
        a.local_dt = 1;
        a.write_dt = (e == 0 && o.recompute_dt) ? 1 : 0;
        a.cfl = o.cfl;
        a.want_lam = 0;
    }
    if (o.learned) {
        const bmhd_learned &L = *o.learned;
        a.lrn_y = L.y_buf;
        a.lrn_stats = L.stats;
        a.lrn_flags = L.flags;
        a.tau = L.tau;
        a.floor_rel = L.floor_rel;
        a.want_lam = 0;
        const int count = a.count_faults;
        a.count_faults = 0;
        // the network path evaluates every face once (compact layout); given corrections (mode 2) come in
        // bmhd_face_data's layout
        a.lrn_compact = L.mode != 2 ? 1 : 0;
        const int nrows = h.nb * 1536 + h.n_hb * 64;
        if (L.mode == 0) {  // BF16 network: features stored in BF16 in the first half of x_buf
            uint16_t *xb = reinterpret_cast<uint16_t *>(L.x_buf);
            k_face_features<__bf16><<<h.nb, Slab<8>::NT, 0, s>>>(h.dev, a, L.stats, reinterpret_cast<__bf16 *>(xb));
            if (int32_t rc = launch_check("face features")) return rc;
            std::string err;
            if (int32_t rc = mlp_infer_bf16_inputs(L.params, L.params_bf16, L.hidden, nrows, xb, L.y_buf, s, err))
                return fail(rc, err);
        } else if (L.mode == 1) {  // FP32 network; mode 2: y_buf is given
            k_face_features<float><<<h.nb, Slab<8>::NT, 0, s>>>(h.dev, a, L.stats, L.x_buf);
            if (int32_t rc = launch_check("face features")) return rc;
            if (int32_t rc = bmhd_mlp_forward(L.params, L.params_bf16, L.hidden, nrows, L.x_buf, L.y_buf,
                                              nullptr, L.mode, s))
                return fail(rc, bmhd_mlp_last_error());
        }
        if (ev0)
            if (int32_t rc = hip_check(hipEventRecord(reinterpret_cast<hipEvent_t>(ev0), s), "event")) return rc;
        if (int32_t rc = launch_learn(h, a, o, s)) return rc;
        if (ev1)
            if (int32_t rc = hip_check(hipEventRecord(reinterpret_cast<hipEvent_t>(ev1), s), "event")) return rc;
        a.count_faults = count;
        k_learn_fixup<<<h.nb, 512, 0, s>>>(h.dev, a, L.fallback_cells);
        return launch_check("learned fallback");
    }
    if (int32_t rc = launch_stage(h, a, o, ev0, ev1, s, in)) return rc;
    if (!h.fc_cells.empty()) {
        k_flux_correct<<<unsigned((h.fc_cells.size() + 255) / 256), 256, 0, s>>>(h.dev, a);
        if (int32_t rc = launch_check("flux correction")) return rc;
    }
    return BMHD_OK;
}

// Capture (once per buffer set and options) a graph of one whole step after the first: dt from the
// previous step's bound, both stages, the next bound. Kernels only: no memset or copy nodes.
int32_t ensure_step_graph(HostGrid &h, const bmhd_opts &o, double *d_U0, double *d_U1, double *d_dt,
                          int32_t *d_faults) {
    bmhd_opts ko = o;
    ko.events = nullptr;
    ko.n_events = 0;
    std::vector<unsigned char> key(sizeof(ko) + 4 * sizeof(void *));
    std::memcpy(key.data(), &ko, sizeof(ko));
    void *ptrs[4] = {d_U0, d_U1, d_dt, d_faults};
    std::memcpy(key.data() + sizeof(ko), ptrs, sizeof(ptrs));
    if (h.graph_exec && key == h.graph_key) return BMHD_OK;
    if (h.graph_exec) (void)hipGraphExecDestroy(reinterpret_cast<hipGraphExec_t>(h.graph_exec));
    if (h.graph) (void)hipGraphDestroy(reinterpret_cast<hipGraph_t>(h.graph));
    h.graph_exec = h.graph = nullptr;
    if (!h.capture_stream) {
        hipStream_t cs;
        if (int32_t rc = hip_check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream")) return rc;
        h.capture_stream = cs;
    }
    hipStream_t cs = reinterpret_cast<hipStream_t>(h.capture_stream);
    if (int32_t rc = hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture")) return rc;
    int32_t rc = BMHD_OK;
    if (o.recompute_dt && !o.local_dt) k_dt_finalize<<<(h.ns + 63) / 64, 64, 0, cs>>>(h.dev, o.cfl, d_dt);
    for (int e = 0; e < 2 && rc == BMHD_OK; ++e)
        rc = enqueue_stage(h, ko, e, d_U0, d_U1, d_dt, d_faults, e == 1 && o.recompute_dt && !o.local_dt, nullptr,
                           nullptr, cs);
    hipGraph_t graph = nullptr;
    const int32_t rc2 = hip_check(hipStreamEndCapture(cs, &graph), "end capture");
    if (rc) return rc;
    if (rc2) return rc2;
    hipGraphExec_t ex = nullptr;
    if (int32_t rc3 = hip_check(hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0), "instantiate")) {
        (void)hipGraphDestroy(graph);
        return rc3;
    }
    h.graph = graph;
    h.graph_exec = ex;
    h.graph_key = key;
    return BMHD_OK;
}

// block id of level-l block (bx, by, bz) of simulation s in the host lookup table, or -1
int32_t host_lut(const HostGrid &g, int s, int l, long long bx, long long by, long long bz) {
    const DevSim &S = g.sims[s];
    const long long nx = (long long)S.nroot[0] << l, ny = (long long)S.nroot[1] << l, nz = (long long)S.nroot[2] << l;
    if (bx < 0 || by < 0 || bz < 0 || bx >= nx || by >= ny || bz >= nz) return -1;
    return g.lut[S.lut_off[l] + (bz * ny + by) * nx + bx];
}

bool remap_compatible(const HostGrid &f, const HostGrid &t) {
    if (f.ns != t.ns) return false;
    for (int s = 0; s < f.ns; ++s) {
        const bmhd_sim_desc &a = f.sdesc[s], &b = t.sdesc[s];
        for (int q = 0; q < 3; ++q)
            if (a.nroot[q] != b.nroot[q] || a.origin[q] != b.origin[q] || a.body_c[q] != b.body_c[q]) return false;
        for (int q = 0; q < 6; ++q)
            if (a.bc[q] != b.bc[q]) return false;
        for (int q = 0; q < 8; ++q)
            if (a.inflow_W[q] != b.inflow_W[q]) return false;
        if (a.dx0 != b.dx0 || a.body_r != b.body_r) return false;
    }
    return true;
}

// a new block can be filled from the old grid: same block, child of an old level-0 block, or parent of 8
// old level-1 blocks
bool remap_source(const HostGrid &f, int s, int l, const int32_t *ijk) {
    if (host_lut(f, s, l, ijk[0], ijk[1], ijk[2]) >= 0) return true;
    if (l == 1) return host_lut(f, s, 0, ijk[0] >> 1, ijk[1] >> 1, ijk[2] >> 1) >= 0;
    for (int q = 0; q < 8; ++q)
        if (host_lut(f, s, 1, 2 * ijk[0] + (q & 1), 2 * ijk[1] + ((q >> 1) & 1), 2 * ijk[2] + (q >> 2)) < 0)
            return false;
    return true;
}

// Autotuner cache key: device (architecture, CU count), grid (sizes and an FNV-1a hash of its block list)
// and the options that change the work (flux, Powell, precision, learned, local dt, graphs, step count).
int32_t autotune_key(const HostGrid &h, const bmhd_opts &o, int n_steps, int dev, int cus, std::string &key) {
    hipDeviceProp_t prop;
    if (int32_t rc = hip_check(hipGetDeviceProperties(&prop, dev), "device properties")) return rc;
    uint64_t hsh = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *c = static_cast<const unsigned char *>(p);
        for (size_t q = 0; q < n; ++q) hsh = (hsh ^ c[q]) * 1099511628211ull;
    };
    mix(h.level.data(), h.level.size() * sizeof(int32_t));
    mix(h.ijk.data(), h.ijk.size() * sizeof(int32_t));
    mix(h.sim.data(), h.sim.size() * sizeof(int32_t));
    char buf[512];
    snprintf(buf, sizeof buf, "%s/%d/nb%d/ns%d/h%016llx/f%d/p%d/q%d/l%d/t%d/g%d/s%d", prop.gcnArchName, cus, h.nb, h.ns,
             (unsigned long long)hsh, o.flux, o.powell, o.precision, o.learned ? 1 : 0, o.local_dt, o.use_graph,
             n_steps);
    key = buf;
    for (char &c : key)
        if (c == ' ') c = '_';
    return BMHD_OK;
}

bool autotune_lookup(const char *path, const std::string &key, int &scheme, int &slab, int &persist) {
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[1024];
    bool hit = false;
    while (fgets(line, sizeof line, f)) {
        char k[600];
        int a = 0, b = 0, c = 0;
        if (sscanf(line, "%599s %d %d %d", k, &a, &b, &c) == 4 && key == k &&
            (a == BMHD_SCHEME_FACE || a == BMHD_SCHEME_PLANE) && (b == 4 || b == 8) && (c == 0 || c == 2 || c == 4)) {
            scheme = a;
            slab = b;
            persist = c;
            hit = true;
        }
    }
    fclose(f);
    return hit;
}

int32_t need_upload(const bmhd_grid *g) {
    if (!g) return fail(BMHD_EINVAL, "null grid");
    if (!g->h.d_work) return fail(BMHD_EINVAL, "grid not uploaded (call bmhd_grid_upload first)");
    return BMHD_OK;
}
}  // namespace

namespace bmhd {
int32_t set_last_error(int32_t code, const std::string &msg) { return fail(code, msg); }
int32_t stage_from_view(const HostGrid &h, const ViewStage &v, int e, const double *U0, const double *Uin,
                        double *Uout, const double *dt, const bmhd_opts &o, int32_t *faults, void *stream) {
    return stage_from_view_impl(h, v, e, U0, Uin, Uout, dt, o, faults, stream);
}
int32_t flux_correct_subset(const HostGrid &h, const ViewStage &v, int e, double *Uout, const double *dt,
                            const bmhd_opts &o, int32_t *faults, void *stream) {
    return flux_correct_subset_impl(h, v, e, Uout, dt, o, faults, stream);
}
}  // namespace bmhd

extern "C" {

int32_t bmhd_version(void) { return 100; }

const char *bmhd_last_error(void) { return g_err.c_str(); }

int32_t bmhd_grid_create(const bmhd_grid_desc *desc, bmhd_grid **out) {
    g_err.clear();
    if (!out) return fail(BMHD_EINVAL, "null output handle");
    *out = nullptr;
    bmhd_grid *g = new (std::nothrow) bmhd_grid;
    if (!g) return fail(BMHD_ENOMEM, "out of host memory");
    std::string err;
    int32_t rc;
    try {
        rc = build_grid(desc, g->h, err);
    } catch (const std::bad_alloc &) {
        rc = BMHD_ENOMEM;
        err = "out of host memory";
    }
    if (rc != BMHD_OK) {
        delete g;
        return fail(rc, err);
    }
    *out = g;
    return BMHD_OK;
}

void bmhd_grid_destroy(bmhd_grid *g) { delete g; }

int32_t bmhd_grid_info_get(const bmhd_grid *g, bmhd_grid_info *info) {
    if (!g || !info) return fail(BMHD_EINVAL, "null argument");
    info->n_blocks = g->h.nb;
    info->n_sims = g->h.ns;
    info->n_level_faces = int32_t(g->h.halo_items.size());
    info->n_flux_faces = g->h.n_fc_rec;
    info->work_bytes = g->h.work_bytes;
    return BMHD_OK;
}

int32_t bmhd_grid_neighbors(const bmhd_grid *g, int32_t *h_out) {
    if (!g || !h_out) return fail(BMHD_EINVAL, "null argument");
    std::memcpy(h_out, g->h.nbr.data(), sizeof(int32_t) * g->h.nbr.size());
    return BMHD_OK;
}

int32_t bmhd_grid_upload(bmhd_grid *g, void *d_work, size_t work_bytes, void *stream) {
    if (!g || !d_work) return fail(BMHD_EINVAL, "null argument");
    if ((reinterpret_cast<uintptr_t>(d_work) & 255u) != 0) return fail(BMHD_EINVAL, "workspace not 256-byte aligned");
    HostGrid &h = g->h;
    if (work_bytes < h.work_bytes)
        return fail(BMHD_ENOMEM, "workspace too small: need " + std::to_string(h.work_bytes) + " bytes");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char *base = static_cast<unsigned char *>(d_work);
    int32_t rc = hip_check(hipMemcpyAsync(base, h.blob.data(), h.table_bytes, hipMemcpyHostToDevice, s), "upload tables");
    if (rc) return rc;
    rc = hip_check(hipMemsetAsync(base + h.table_bytes, 0, h.work_bytes - h.table_bytes, s), "clear scratch");
    if (rc) return rc;
    rc = hip_check(hipStreamSynchronize(s), "upload sync");
    if (rc) return rc;
    h.d_work = d_work;
    Tables &t = h.dev;
    t.blocks = reinterpret_cast<const DevBlock *>(base + h.off_blocks);
    t.sims = reinterpret_cast<const DevSim *>(base + h.off_sims);
    t.lut = reinterpret_cast<const int32_t *>(base + h.off_lut);
    t.order = reinterpret_cast<const int32_t *>(base + h.off_order);
    t.order_split = reinterpret_cast<const int32_t *>(base + h.off_order_split);
    t.halo_items = reinterpret_cast<const int32_t *>(base + h.off_halo_items);
    t.fc_cells = reinterpret_cast<const DevFcCell *>(base + h.off_fc_cells);
    t.lam = reinterpret_cast<unsigned long long *>(base + h.off_lam);
    t.halo = reinterpret_cast<double *>(base + h.off_halo);
    t.fcbuf = reinterpret_cast<double *>(base + h.off_fcbuf);
    t.nb = h.nb;
    t.ns = h.ns;
    t.n_halo_items = int32_t(h.halo_items.size());
    t.n_fc_cells = int32_t(h.fc_cells.size());
    t.n_clear = h.n_clear;
    return BMHD_OK;
}

int32_t bmhd_set_state(const bmhd_grid *g, const double *d_W, double *d_U, void *stream) {
    if (int32_t rc = need_upload(g)) return rc;
    if (!ptr_ok(d_W) || !ptr_ok(d_U)) return fail(BMHD_EINVAL, "null or misaligned state pointer");
    const size_t n = size_t(g->h.nb) * 512;
    if (n == 0) return BMHD_OK;
    k_set_state<<<unsigned((n + 255) / 256), 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(d_W, d_U, n);
    return launch_check("set_state");
}

int32_t bmhd_fill_ghosts(const bmhd_grid *g, const double *d_U, double *d_view, void *stream) {
    if (int32_t rc = need_upload(g)) return rc;
    if (!ptr_ok(d_U) || !ptr_ok(d_view)) return fail(BMHD_EINVAL, "null or misaligned pointer");
    if (g->h.nb == 0) return BMHD_OK;
    k_fill_view<<<g->h.nb, 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(g->h.dev, d_U, d_view);
    return launch_check("fill_ghosts");
}

int32_t bmhd_remap(const bmhd_grid *from, const double *d_U_from, const bmhd_grid *to, double *d_U_to,
                   void *stream) {
    if (int32_t rc = need_upload(from)) return rc;
    if (int32_t rc = need_upload(to)) return rc;
    if (!ptr_ok(d_U_from) || !ptr_ok(d_U_to) || d_U_from == d_U_to)
        return fail(BMHD_EINVAL, "remap: null, misaligned or aliased state pointers");
    const HostGrid &f = from->h, &t = to->h;
    if (!remap_compatible(f, t)) return fail(BMHD_EINVAL, "remap: the grids differ in their simulations");
    for (int b = 0; b < t.nb; ++b)
        if (!remap_source(f, t.sim[b], t.level[b], &t.ijk[3 * b]))
            return fail(BMHD_EINVAL, "remap: a block of the new grid is neither a block of the old one, a child of "
                                     "an old level-0 block nor the parent of 8 old level-1 blocks");
    if (t.nb == 0) return BMHD_OK;
    k_remap<<<t.nb, 512, 0, reinterpret_cast<hipStream_t>(stream)>>>(f.dev, d_U_from, t.dev, d_U_to);
    return launch_check("remap");
}

int32_t bmhd_face_targets(const bmhd_grid *fine, const float *d_Ff, const bmhd_grid *coarse, const float *d_Fc,
                          float *d_T, void *stream) {
    if (int32_t rc = need_upload(fine)) return rc;
    if (int32_t rc = need_upload(coarse)) return rc;
    if (!d_Ff || !d_Fc || !d_T) return fail(BMHD_EINVAL, "face_targets: null buffer");
    const HostGrid &f = fine->h, &c = coarse->h;
    if (!remap_compatible(f, c)) return fail(BMHD_EINVAL, "face_targets: the grids differ in their simulations");
    if (f.nb != 8 * c.nb) return fail(BMHD_EINVAL, "face_targets: the fine grid must be the coarse grid refined everywhere");
    for (int b = 0; b < c.nb; ++b) {
        if (c.level[b] != 0) return fail(BMHD_EINVAL, "face_targets: the coarse grid must be all level 0");
        for (int q = 0; q < 8; ++q)
            if (host_lut(f, c.sim[b], 1, 2LL * c.ijk[3 * b] + (q & 1), 2LL * c.ijk[3 * b + 1] + ((q >> 1) & 1),
                         2LL * c.ijk[3 * b + 2] + (q >> 2)) < 0)
                return fail(BMHD_EINVAL, "face_targets: a coarse block lacks its 8 level-1 children in the fine grid");
    }
    if (c.nb == 0) return BMHD_OK;
    k_face_targets<<<c.nb, 576, 0, reinterpret_cast<hipStream_t>(stream)>>>(f.dev, d_Ff, c.dev, d_Fc, d_T);
    return launch_check("face targets");
}

int32_t bmhd_block_indicator(const bmhd_grid *g, const double *d_U, double *d_ind, void *stream) {
    if (int32_t rc = need_upload(g)) return rc;
    if (!ptr_ok(d_U) || !ptr_ok(d_ind)) return fail(BMHD_EINVAL, "block_indicator: null or misaligned buffer");
    if (g->h.nb == 0) return BMHD_OK;
    k_block_indicator<<<g->h.nb, 512, 0, reinterpret_cast<hipStream_t>(stream)>>>(g->h.dev, d_U, d_ind);
    return launch_check("block indicator");
}

int32_t bmhd_adapt(const bmhd_grid *g, const double *h_ind, double r_refine, double r_coarsen, int32_t *h_level,
                   int32_t *h_ijk, int32_t *h_sim, int32_t max_blocks, int32_t *n_out) {
    if (!g || !h_ind || !n_out || !(r_coarsen <= r_refine)) return fail(BMHD_EINVAL, "adapt: bad arguments");
    const HostGrid &h = g->h;
    int64_t n = 0;
    for (int s = 0; s < h.ns; ++s) {
        const DevSim &S = h.sims[s];
        for (int64_t z = 0; z < S.nroot[2]; ++z)
            for (int64_t y = 0; y < S.nroot[1]; ++y)
                for (int64_t x = 0; x < S.nroot[0]; ++x) {
                    const int32_t root = host_lut(h, s, 0, x, y, z);
                    bool refine;
                    if (root >= 0) {
                        refine = h_ind[root] >= r_refine;
                    } else {
                        double m = 0.0;
                        for (int q = 0; q < 8; ++q) {
                            const int32_t c = host_lut(h, s, 1, 2 * x + (q & 1), 2 * y + ((q >> 1) & 1), 2 * z + (q >> 2));
                            if (c < 0) return fail(BMHD_EINVAL, "adapt: a root is neither a block nor 8 children");
                            m = std::max(m, h_ind[c]);
                        }
                        refine = !(m < r_coarsen);
                    }
                    const int add = refine ? 8 : 1;
                    if (h_level && n + add > max_blocks) return fail(BMHD_ENOMEM, "adapt: output arrays too small");
                    for (int q = 0; q < add; ++q, ++n) {
                        if (!h_level) continue;
                        h_level[n] = refine ? 1 : 0;
                        h_ijk[3 * n + 0] = int32_t(refine ? 2 * x + (q & 1) : x);
                        h_ijk[3 * n + 1] = int32_t(refine ? 2 * y + ((q >> 1) & 1) : y);
                        h_ijk[3 * n + 2] = int32_t(refine ? 2 * z + (q >> 2) : z);
                        h_sim[n] = s;
                    }
                }
    }
    *n_out = int32_t(n);
    return BMHD_OK;
}

int32_t bmhd_reduce_dt(const bmhd_grid *g, const double *d_U, double cfl, double *d_dt, void *stream) {
    if (int32_t rc = need_upload(g)) return rc;
    if (!ptr_ok(d_U) || !ptr_ok(d_dt)) return fail(BMHD_EINVAL, "null or misaligned pointer");
    if (!(cfl > 0.0)) return fail(BMHD_EINVAL, "cfl must be positive");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const HostGrid &h = g->h;
    const int sb = (h.ns + 63) / 64;
    k_lam_reset<<<sb, 64, 0, s>>>(h.dev);
    if (h.nb) k_dt_reduce<<<h.nb, 512, 0, s>>>(h.dev, d_U);
    k_dt_finalize<<<sb, 64, 0, s>>>(h.dev, cfl, d_dt);
    return launch_check("reduce_dt");
}

int32_t bmhd_advance(const bmhd_grid *g, double *d_U0, double *d_U1, double *d_dt, int32_t n_stages,
                     const bmhd_opts *opts, int32_t *d_faults, void *stream) {
    if (int32_t rc = need_upload(g)) return rc;
    if (!opts) return fail(BMHD_EINVAL, "null options");
    if (!ptr_ok(d_U0) || !ptr_ok(d_U1) || !ptr_ok(d_dt) || d_U0 == d_U1)
        return fail(BMHD_EINVAL, "null, misaligned or aliased state pointers");
    if (d_faults && (reinterpret_cast<uintptr_t>(d_faults) & 3u)) return fail(BMHD_EINVAL, "misaligned fault counter");
    if (n_stages < 0) return fail(BMHD_EINVAL, "n_stages must be >= 0");
    const bmhd_opts &o = *opts;
    if (int32_t rc = check_opts(o)) return rc;
    if (o.use_graph && (n_stages & 1)) return fail(BMHD_EINVAL, "use_graph needs whole steps (even n_stages)");
    HostGrid &h = const_cast<bmhd_grid *>(g)->h;
    if (o.learned && !h.halo_items.empty())
        return fail(BMHD_EUNSUPPORTED, "the learned correction needs a single-level grid");
    // the fused next-dt bound is taken before the learned fallback, so the learned form reduces dt anew
    const bool fused_dt = !o.learned;
    if (h.nb == 0 || n_stages == 0) return BMHD_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int n_steps = (n_stages + 1) / 2;
    const bool timed = !o.use_graph && o.events && o.n_events >= 2 * n_stages;
    // the first step (and every step without a graph) is launched directly
    const int direct_steps = o.use_graph ? 1 : n_steps;
    for (int step = 0; step < direct_steps; ++step) {
        for (int e = 0; e < 2; ++e) {
            const int st = 2 * step + e;
            if (st >= n_stages) break;
            if (e == 0 && o.recompute_dt && !o.local_dt) {
                const int sb = (h.ns + 63) / 64;
                if (st == 0 || !fused_dt) {
                    k_lam_reset<<<sb, 64, 0, s>>>(h.dev);
                    k_dt_reduce<<<h.nb, 512, 0, s>>>(h.dev, d_U0);
                }
                k_dt_finalize<<<sb, 64, 0, s>>>(h.dev, o.cfl, d_dt);
            }
            void *ev0 = timed ? o.events[2 * st] : nullptr, *ev1 = timed ? o.events[2 * st + 1] : nullptr;
            const bool want_lam = fused_dt && e == 1 && o.recompute_dt && !o.local_dt && st + 1 < n_stages;
            if (int32_t rc = enqueue_stage(h, o, e, d_U0, d_U1, d_dt, d_faults, want_lam, ev0, ev1, s)) return rc;
        }
    }
    if (o.use_graph && n_steps > 1) {
        if (int32_t rc = ensure_step_graph(h, o, d_U0, d_U1, d_dt, d_faults)) return rc;
        hipGraphExec_t ex = reinterpret_cast<hipGraphExec_t>(h.graph_exec);
        for (int step = 1; step < n_steps; ++step)
            if (int32_t rc = hip_check(hipGraphLaunch(ex, s), "graph launch")) return rc;
    }
    return launch_check("advance");
}

int32_t bmhd_face_data(const bmhd_grid *g, const double *d_U, int32_t flux, const float *d_stats, float *d_X,
                       float *d_F, void *stream) {
    if (int32_t rc = need_upload(g)) return rc;
    if (!ptr_ok(d_U) || (!d_X && !d_F)) return fail(BMHD_EINVAL, "face_data: bad pointers");
    if (flux != BMHD_FLUX_RUSANOV && flux != BMHD_FLUX_HLLE) return fail(BMHD_EINVAL, "unknown flux");
    const HostGrid &h = g->h;
    if (!h.halo_items.empty()) return fail(BMHD_EUNSUPPORTED, "face_data needs a single-level grid");
    if (h.nb == 0) return BMHD_OK;
    StageArgs a;
    std::memset(&a, 0, sizeof a);
    a.Uin = d_U;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (flux == BMHD_FLUX_RUSANOV) k_face_data<BMHD_FLUX_RUSANOV><<<h.nb, Slab<8>::NT, 0, s>>>(h.dev, a, d_stats, d_X, d_F);
    else k_face_data<BMHD_FLUX_HLLE><<<h.nb, Slab<8>::NT, 0, s>>>(h.dev, a, d_stats, d_X, d_F);
    return launch_check("face_data");
}

int32_t bmhd_autotune(const bmhd_grid *g, double *d_U0, double *d_U1, double *d_dt, const bmhd_opts *base,
                      int32_t n_steps, bmhd_opts *best, float *h_ms, void *stream) {
    if (int32_t rc = need_upload(g)) return rc;
    if (!base || !best || n_steps <= 0) return fail(BMHD_EINVAL, "bad autotune arguments");
    if (int32_t rc = check_opts(*base)) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int dev = 0, cus = 0;
    if (int32_t rc = hip_check(hipGetDevice(&dev), "device")) return rc;
    if (int32_t rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "attr")) return rc;
    // on-disk cache (opt-in): one line per tuned configuration, the last matching line wins
    const char *cache = getenv("BMHD_AUTOTUNE_CACHE");
    std::string key;
    if (cache && *cache) {
        if (int32_t rc = autotune_key(g->h, *base, n_steps, dev, cus, key)) return rc;
        int sc = 0, sl = 0, pp = 0;
        if (autotune_lookup(cache, key, sc, sl, pp)) {
            *best = *base;
            best->scheme = sc;
            best->slab = sl;
            best->persist_wgs = pp * cus;
            if (h_ms)
                for (int c = 0; c < BMHD_AUTOTUNE_SHAPES; ++c) h_ms[c] = -1.0f;
            return BMHD_OK;
        }
    }
    hipEvent_t e0, e1;
    if (int32_t rc = hip_check(hipEventCreate(&e0), "event")) return rc;
    if (int32_t rc = hip_check(hipEventCreate(&e1), "event")) return rc;
    const int shapes[6][2] = {{4, 0}, {4, 2}, {4, 4}, {8, 0}, {8, 2}, {8, 4}};
    float best_ms = 1e30f;
    int32_t rc = BMHD_OK;
    *best = *base;
    for (int c = 0; c < BMHD_AUTOTUNE_SHAPES && rc == BMHD_OK; ++c) {
        bmhd_opts o = *base;
        if (c < 12) {
            o.scheme = c < 6 ? BMHD_SCHEME_FACE : BMHD_SCHEME_PLANE;
            o.slab = shapes[c % 6][0];
            o.persist_wgs = shapes[c % 6][1] * cus;
        } else {  // the block form: whole blocks, one workgroup each
            o.scheme = BMHD_SCHEME_BLOCK;
            o.slab = 8;
            o.persist_wgs = 0;
        }
        o.events = nullptr;
        o.n_events = 0;
        rc = bmhd_advance(g, d_U0, d_U1, d_dt, 2, &o, nullptr, stream);  // warm-up
        if (rc) break;
        rc = hip_check(hipEventRecord(e0, s), "event");
        if (!rc) rc = bmhd_advance(g, d_U0, d_U1, d_dt, 2 * n_steps, &o, nullptr, stream);
        if (!rc) rc = hip_check(hipEventRecord(e1, s), "event");
        if (!rc) rc = hip_check(hipEventSynchronize(e1), "event sync");
        float ms = 0.f;
        if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
        if (rc) break;
        if (h_ms) h_ms[c] = ms;
        if (ms < best_ms) {
            best_ms = ms;
            *best = o;
            best->events = base->events;
            best->n_events = base->n_events;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == BMHD_OK && !key.empty()) {
        if (FILE *f = fopen(cache, "a")) {
            fprintf(f, "%s %d %d %d\n", key.c_str(), best->scheme, best->slab, cus ? best->persist_wgs / cus : 0);
            fclose(f);
        }
    }
    return rc;
}

}  // extern "C"
