// HIP kernels (gfx950) and C-ABI host code of libsedg: the sub-element adaptive
// blended DG/FV right-hand side of arXiv:2011.03338 and its SSP Runge-Kutta stages (SSP-RK3, SSP-RK(5,4)).
//
// Work decomposition (per RK stage, three launches plus a tiny reduction):
//   analyse  : one thread per subcell, EPB elements per workgroup, all element
//              data staged in LDS.  Reconstructs every level (eq. reco-*),
//              computes the squeezing parameters (eq. calc-squeezing-parameter),
//              the blending factors with level pruning (eq. calc-blending-factor,
//              App. multi-level algorithm) and the blended interface states on
//              the element's own faces (App. eq. 3D-prolongation, multi-level
//              cascade of Sec. 2.6).  Writes alpha, beta and the face buffer
//              (the only data another element reads), plus per-block maxima of
//              the CFL eigenvalue estimate (eq. euler-max-eigenvalue).
//   eface    : one wavefront per element.  The common flux of every element
//              face (App. eq. 3D-blend-interface-fluxes on the element
//              boundary) is computed once, by the element whose low face it
//              is (or by the boundary element at the high end of a
//              non-periodic axis), and stored in a flux buffer that
//              both neighbours read, so the scheme is conservative by
//              construction and without atomics.
//   residual : same decomposition as analyse.  Per axis: blended interface
//              states of every interior subcell face, unique common fluxes
//              there (FV candidate plus per-level DG candidates projected along
//              the face), then the FV and level DG right-hand sides (eq.
//              multilevel-blending-scheme) blended with the weights of eq.
//              blending-weights; the Runge-Kutta combination is fused into the
//              store.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/sedg.h"
#include "sedg_internal.h"

#define MAXLEV 3
#define LAM_SLOTS 256   // slots of the per-step CFL eigenvalue maximum

// ---------------------------------------------------------------------------
// kernel arguments
// ---------------------------------------------------------------------------

struct ProbDesc;

// Level tables are read-only for the lifetime of every launch.  Kernels read them
// through the constant address space, so that the compiler may treat the loads as
// invariant: reads of a wave-uniform address become scalar loads, and per-lane
// reads may be scheduled across barriers.
typedef const __attribute__((address_space(4))) sedg_level_tab CTab;
typedef const __attribute__((address_space(4))) double CDbl;

struct KArgs {
    const double *u;        // stage state (read)
    const double *u0;       // u^n for RK stages 2, 3
    double *out;            // dudt or the next stage state
    double *alpha;          // nel * A
    double *beta;           // nel * A
    const double *alpha_in; // EXTERNAL mode
    double *fbuf;           // face buffer
    double *ef;             // common fluxes on the element faces (face-buffer layout), or null
    double *scale;          // nel * 2: largest mean density and |mean energy| per element
    double *mean;           // nel * NV * A: sub-element means per level
    CTab *tabs;                  // per level index
    double *lam_part;       // per-block CFL eigenvalue maxima (nullable)
    const double *dt;       // device scalar step (RK stages)
    int *err;               // smallest bad element index (INT_MAX = none)
    const double *lam;      // adjoint: input adjoint state
    double *gfb;            // adjoint: per element, its own share of the flux adjoints on its faces
    double *gsb, *gdb;      // adjoint: interface-state and mean-fallback adjoints of the element faces
    double *acc;            // adjoint RK: running adjoint of the step's initial state
    int lam_mask;           // CFL slots - 1 (slot = tile & lam_mask)
    int err_base;           // added to the element index reported through err
    // batched ensembles
    const ProbDesc *probs;  // per problem
    const int *tile_prob;   // problem of every tile
    const int *ftile_prob;  // problem of every element-face tile
    int ntiles;             // tiles of the whole ensemble
    int tile_base;          // first tile of a launch that covers the problems of one K
    // CFL step size formed by workgroup 0 of the element-face kernel (fin_lam non-null):
    // the maximum of the per-block eigenvalue maxima, fin_num / it into *dt, and the log
    double *fin_lam;
    double fin_num;
    double *fin_dt;
    double *fin_dt_log;
    const int *fin_ctr;
    int chunk;              // consecutive tiles per workgroup
    int xcd_map;            // remap workgroups to contiguous tile ranges per XCD
    long long dof;
    int nel;
    int ne[3];
    int G[3];
    int bc[3];
    double dx[3];
    int nlev;
    int lev_n[MAXLEV];
    int lev_off[MAXLEV];
    int A;
    int mode;
    unsigned level_mask;
    int stage;              // 0: write dudt; 1, 2, 3: SSP-RK3 stage
    double gamma, gm1, tau_A, tau_S, alpha_H, alpha_L, beta_L;
    double sigma_floor;     // floor of the smoothness-measure denominator (1 in the paper)
    // 0.99 tau_S when tau_A is finite and >= 0 and tau_S > 0, else 0: a relative change of
    // the smoothness measures below it clamps the blending factor's ramp to 0 for certain
    double ind_quick;
    // RANDOM mode: generator seed and the device counter of right-hand-side draws
    unsigned long long seed;
    const long long *draw;
    int *fbc;               // interface-safety fallback counter (diagnostics; nullable)
    // generic Shu-Osher stage (stage code 5): out = rk[0] u0 + rk[1] u + rk[2] dt L(u)
    // + rk[3] x1, and, where yout is given, yout = rk[4] y0 + rk[5] u + rk[6] dt L(u)
    const double *x1, *y0;
    double *yout;
    double rk[7];
};

// Per-axis mesh data by run-time axis.  A kernel may hold its arguments in a local
// copy, which must only be read at constant offsets to stay in registers; a plain
// select of the three fields is folded by the optimiser into one load at a
// selected offset, so the fields are blended arithmetically (exact: the other
// terms are multiplied by zero and every value is finite).
__device__ __forceinline__ int arg_ne(const KArgs &P, int a)
{
    return (a == 0) * P.ne[0] + (a == 1) * P.ne[1] + (a == 2) * P.ne[2];
}
__device__ __forceinline__ int arg_bc(const KArgs &P, int a)
{
    return (a == 0) * P.bc[0] + (a == 1) * P.bc[1] + (a == 2) * P.bc[2];
}
__device__ __forceinline__ double arg_dx(const KArgs &P, int a)
{
    return (a == 0 ? 1.0 : 0.0) * P.dx[0] + (a == 1 ? 1.0 : 0.0) * P.dx[1] + (a == 2 ? 1.0 : 0.0) * P.dx[2];
}

// Random blending factors (stress test of Sec. 3.3): the k-th output of SplitMix64
// (Steele, Lea & Flood, OOPSLA 2014) seeded with `seed`, i.e. its output function
// applied to seed + (k + 1) * 0x9e3779b97f4a7c15, mapped to [0, 1) by its top 53 bits.
// k = (draw * nel + element) * A + slot enumerates every factor of every draw.
__device__ __forceinline__ double splitmix_u01(unsigned long long seed, unsigned long long k)
{
    unsigned long long z = seed + (k + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// physics (Sec. 3.1) - same formulas as the HLL-Einfeldt flux of Sec. 3
// ---------------------------------------------------------------------------

// The axis a is a run-time value in the kernels: components along a are picked and
// scattered over the unrolled component loop, never by indexing a register array with
// a.  The pick masks the bit patterns of the components (exact for every value): a
// chain of selects between array elements can be turned by the compiler into one load
// from a computed address, which puts the array into scratch memory (it did so in 3-D,
// where the axis differs between the lanes of the element-face kernel).
template <int DIM>
__device__ __forceinline__ double pick(const double *x, int a)
{
    unsigned long long r = 0;
#pragma unroll
    for (int b = 0; b < DIM; ++b)
        r |= (unsigned long long)__double_as_longlong(x[b]) & (0ull - (unsigned long long)(a == b));
    return __longlong_as_double((long long)r);
}

// the ratio of specific heats and gamma - 1 (the latter a kernel argument, so that it
// stays in scalar registers instead of a vector register held across the kernel)
struct Gas {
    double g, gm1;
};

template <int DIM>
__device__ __forceinline__ double pressure(const double *u, const Gas &g)
{
    if (!(u[0] > 0.0)) return -INFINITY;
    double m2 = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) m2 += u[1 + a] * u[1 + a];
    return g.gm1 * (u[DIM + 1] - 0.5 * m2 / u[0]);
}

template <int DIM>
__device__ __forceinline__ bool permissible(const double *u, const Gas &g)
{
    if (!(u[0] > 0.0)) return false;
    return pressure<DIM>(u, g) > 0.0;
}

// interface-flux input admissibility relative to the data scales of the two
// elements sharing the face (largest mean density srho and |mean energy| sE):
// rho > 1e-12 srho and p > -1e-10 sE, so that the squeeze's binding point
// (rho or p = 1e-20 up to rounding) is decided the same way in every rounding order
template <int DIM>
__device__ __forceinline__ bool flux_admissible(const double *u, const Gas &g, double srho, double sE)
{
    if (!(u[0] > 1e-12 * srho)) return false;
    return pressure<DIM>(u, g) > -1e-10 * sE;
}

// the Euler flux along axis a from the reciprocal ir of the density and the pressure p
// (shared by the fluxes along every axis at one node)
template <int DIM>
__device__ __forceinline__ void euler_flux_ir(const double *u, double ir, double p, int a, double *f)
{
    const double ma = pick<DIM>(u + 1, a);
    const double va = ma * ir;
    f[0] = ma;
#pragma unroll
    for (int b = 0; b < DIM; ++b) f[1 + b] = u[1 + b] * va + (a == b ? p : 0.0);
    f[DIM + 1] = va * (u[DIM + 1] + p);
}

template <int DIM>
__device__ __forceinline__ void euler_flux(const double *u, int a, const Gas &g, double *f)
{
    double p = pressure<DIM>(u, g);
    const double ma = pick<DIM>(u + 1, a);
    double va = ma / u[0];
    f[0] = ma;
#pragma unroll
    for (int b = 0; b < DIM; ++b) f[1 + b] = u[1 + b] * va + (a == b ? p : 0.0);
    f[DIM + 1] = va * (u[DIM + 1] + p);
}

// HLL flux with Einfeldt's signal speeds (Roe averages), branch-free in the
// speeds: F* = (S_R+ f_L - S_L- f_R + S_L- S_R+ (u_R - u_L)) / (S_R+ - S_L-), S_L- =
// min(S_L, 0), S_R+ = max(S_R, 0).  One reciprocal per density and one for the Roe
// weights instead of a division per quotient.
template <int DIM>
__device__ void hlle(const double *uL, const double *uR, int a, const Gas &g, double *fs)
{
    constexpr int NV = DIM + 2;
    const double irL = 1.0 / uL[0], irR = 1.0 / uR[0];
    double m2L = 0.0, m2R = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        m2L += uL[1 + b] * uL[1 + b];
        m2R += uR[1 + b] * uR[1 + b];
    }
    const double pL = (uL[0] > 0.0) ? g.gm1 * (uL[DIM + 1] - 0.5 * m2L * irL) : -INFINITY;
    const double pR = (uR[0] > 0.0) ? g.gm1 * (uR[DIM + 1] - 0.5 * m2R * irR) : -INFINITY;
    const double mL = pick<DIM>(uL + 1, a), mR = pick<DIM>(uR + 1, a);
    const double vL = mL * irL, vR = mR * irR;
    double fL[NV], fR[NV];
    fL[0] = mL;
    fR[0] = mR;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        fL[1 + b] = uL[1 + b] * vL + (a == b ? pL : 0.0);
        fR[1 + b] = uR[1 + b] * vR + (a == b ? pR : 0.0);
    }
    fL[DIM + 1] = vL * (uL[DIM + 1] + pL);
    fR[DIM + 1] = vR * (uR[DIM + 1] + pR);
    const double cL = sqrt(fmax(g.g * pL * irL, 0.0)), cR = sqrt(fmax(g.g * pR * irR, 0.0));
    const double sqL = sqrt(uL[0]), sqR = sqrt(uR[0]);
    const double iS = 1.0 / (sqL + sqR);
    const double HL = (uL[DIM + 1] + pL) * irL, HR = (uR[DIM + 1] + pR) * irR;
    double vt2 = 0.0, vtn = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        const double vb = (sqL * (uL[1 + b] * irL) + sqR * (uR[1 + b] * irR)) * iS;
        vt2 += vb * vb;
        if (b == a) vtn = vb;
    }
    const double Ht = (sqL * HL + sqR * HR) * iS;
    const double ct = sqrt(fmax(g.gm1 * (Ht - 0.5 * vt2), 0.0));
    const double SL = fmin(vL - cL, vtn - ct);
    const double SR = fmax(vR + cR, vtn + ct);
    const double SLm = fmin(SL, 0.0), SRp = fmax(SR, 0.0);
    const double den = SRp - SLm;
    const double inv = den > 0.0 ? 1.0 / den : 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) fs[v] = (SRp * fL[v] - SLm * fR[v] + SLm * SRp * (uR[v] - uL[v])) * inv;
}

// ---------------------------------------------------------------------------
// reverse-mode building blocks of the adjoint (vector-Jacobian products)
// ---------------------------------------------------------------------------

// gu = (d f_a / d u)^T gf for the Euler flux of eqn. comp-euler-conservative
template <int DIM>
__device__ __forceinline__ void euler_flux_adj(const double *u, int a, const Gas &g, const double *gf, double *gu)
{
    constexpr int NV = DIM + 2;
    const double ir = 1.0 / u[0];
    double m2 = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) m2 += u[1 + b] * u[1 + b];
    const double p = g.gm1 * (u[DIM + 1] - 0.5 * m2 * ir);
    const double ma = pick<DIM>(u + 1, a);
    const double va = ma * ir;
    const double gp = pick<DIM>(gf + 1, a) + gf[NV - 1] * va;
    double gva = gf[NV - 1] * (u[DIM + 1] + p);
#pragma unroll
    for (int b = 0; b < DIM; ++b) gva += gf[1 + b] * u[1 + b];
    const double gE = gf[NV - 1] * va + g.gm1 * gp;
    const double gm2 = -0.5 * g.gm1 * ir * gp;
    const double gir = gva * ma - 0.5 * g.gm1 * m2 * gp;
    // f_0 = m_a, f_(1+b) = m_b va + delta_ab p, f_E = va (E + p); va = m_a / rho;
    // p = (g - 1)(E - m.m / (2 rho))
#pragma unroll
    for (int b = 0; b < DIM; ++b)
        gu[1 + b] = gf[1 + b] * va + 2.0 * u[1 + b] * gm2 + ((b == a) ? (gf[0] + gva * ir) : 0.0);
    gu[0] = -gir * ir * ir;
    gu[NV - 1] = gE;
}

// (guL, guR) = (d HLLE / d(uL, uR))^T gfs at (uL, uR), branches of every min/max
// taken as the forward evaluation takes them
template <int DIM>
__device__ void hlle_adj(const double *uL, const double *uR, int a, const Gas &g, const double *gfs, double *guL, double *guR)
{
    constexpr int NV = DIM + 2;
    double ir[2], m2[2], p[2], va[2], c[2], sq[2], H[2], q[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const double *w = s ? uR : uL;
        ir[s] = 1.0 / w[0];
        m2[s] = 0.0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) m2[s] += w[1 + b] * w[1 + b];
        p[s] = g.gm1 * (w[DIM + 1] - 0.5 * m2[s] * ir[s]);
        va[s] = pick<DIM>(w + 1, a) * ir[s];
        q[s] = g.g * p[s] * ir[s];
        c[s] = sqrt(fmax(q[s], 0.0));
        sq[s] = sqrt(w[0]);
        H[s] = (w[DIM + 1] + p[s]) * ir[s];
    }
    const double S = sq[0] + sq[1];
    double vt[DIM], vt2 = 0.0;
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        vt[b] = (sq[0] * (uL[1 + b] * ir[0]) + sq[1] * (uR[1 + b] * ir[1])) / S;
        vt2 += vt[b] * vt[b];
    }
    const double vta = pick<DIM>(vt, a);
    const double Ht = (sq[0] * H[0] + sq[1] * H[1]) / S;
    const double ct2 = g.gm1 * (Ht - 0.5 * vt2);
    const double ct = sqrt(fmax(ct2, 0.0));
    const double aL1 = va[0] - c[0], aL2 = vta - ct;
    const double aR1 = va[1] + c[1], aR2 = vta + ct;
    const bool selL2 = aL2 < aL1, selR2 = aR2 > aR1;
    const double SL = selL2 ? aL2 : aL1, SR = selR2 ? aR2 : aR1;
    const bool SLpos = 0.0 < SL, SRneg = 0.0 > SR;
    const double SLm = SLpos ? 0.0 : SL, SRp = SRneg ? 0.0 : SR;
    const double den = SRp - SLm;
    const double inv = den > 0.0 ? 1.0 / den : 0.0;
    // fs = (SRp fL - SLm fR + SLm SRp (uR - uL)) inv
    double gnum[NV], ginv = 0.0, gSRp = 0.0, gSLm = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double fl, fr;
        if (v == 0) { fl = pick<DIM>(uL + 1, a); fr = pick<DIM>(uR + 1, a); }
        else if (v == NV - 1) { fl = va[0] * (uL[DIM + 1] + p[0]); fr = va[1] * (uR[DIM + 1] + p[1]); }
        else {
            fl = uL[v] * va[0] + ((v - 1 == a) ? p[0] : 0.0);
            fr = uR[v] * va[1] + ((v - 1 == a) ? p[1] : 0.0);
        }
        const double du = uR[v] - uL[v];
        const double num = SRp * fl - SLm * fr + SLm * SRp * du;
        gnum[v] = gfs[v] * inv;
        ginv += gfs[v] * num;
        gSRp += gnum[v] * (fl + SLm * du);
        gSLm += gnum[v] * (-fr + SRp * du);
        guR[v] = gnum[v] * SLm * SRp;
        guL[v] = -gnum[v] * SLm * SRp;
    }
    const double gden = den > 0.0 ? -ginv * inv * inv : 0.0;
    gSRp += gden;
    gSLm -= gden;
    const double gSL = SLpos ? 0.0 : gSLm;
    const double gSR = SRneg ? 0.0 : gSRp;
    // wave-speed estimates: SL = min(vL - cL, vt_a - ct), SR = max(vR + cR, vt_a + ct)
    double gva[2], gc[2];
    gva[0] = selL2 ? 0.0 : gSL;
    gc[0] = selL2 ? 0.0 : -gSL;
    gva[1] = selR2 ? 0.0 : gSR;
    gc[1] = selR2 ? 0.0 : gSR;
    const double gvta = (selL2 ? gSL : 0.0) + (selR2 ? gSR : 0.0);
    const double gct = (selR2 ? gSR : 0.0) - (selL2 ? gSL : 0.0);
    // Roe averages
    const double gct2 = (ct > 0.0) ? gct / (2.0 * ct) : 0.0;
    const double gHt = g.gm1 * gct2;
    const double gvt2 = -0.5 * g.gm1 * gct2;
    double gsq[2], gS = -gHt * Ht / S, gH[2];
    gsq[0] = gHt / S * H[0];
    gsq[1] = gHt / S * H[1];
    gH[0] = gHt / S * sq[0];
    gH[1] = gHt / S * sq[1];
    double gvel[2][DIM];
#pragma unroll
    for (int b = 0; b < DIM; ++b) {
        const double gvtb = 2.0 * vt[b] * gvt2 + ((b == a) ? gvta : 0.0);
        const double gN = gvtb / S;
        const double v0 = uL[1 + b] * ir[0], v1 = uR[1 + b] * ir[1];
        gS -= gvtb * vt[b] / S;
        gsq[0] += gN * v0;
        gsq[1] += gN * v1;
        gvel[0][b] = gN * sq[0];
        gvel[1][b] = gN * sq[1];
    }
    gsq[0] += gS;
    gsq[1] += gS;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const double *w = s ? uR : uL;
        double *gw = s ? guR : guL;
        const double *gfs_ = gnum;   // flux adjoint of side s: SRp gnum (left), -SLm gnum (right)
        const double fsc = s ? -SLm : SRp;
        double gp = 0.0, gir = 0.0, gE = 0.0;
        // H = (E + p) ir
        gE += gH[s] * ir[s];
        gp += gH[s] * ir[s];
        gir += gH[s] * (w[DIM + 1] + p[s]);
        // sq = sqrt(rho)
        double grho = sq[s] > 0.0 ? gsq[s] / (2.0 * sq[s]) : 0.0;
        // c = sqrt(max(q, 0)), q = g p ir
        if (q[s] > 0.0 && c[s] > 0.0) {
            const double gq = gc[s] / (2.0 * c[s]);
            gp += gq * g.g * ir[s];
            gir += gq * g.g * p[s];
        }
        // flux f_a(w) with adjoint fsc * gnum
        const double gfE = fsc * gfs_[NV - 1];
        double gvas = gva[s] + gfE * (w[DIM + 1] + p[s]);
        gE += gfE * va[s];
        gp += gfE * va[s] + fsc * pick<DIM>(gfs_ + 1, a);
        double gm[DIM];
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const double gfb = fsc * gfs_[1 + b];
            gm[b] = gfb * va[s];
            gvas += gfb * w[1 + b];
        }
        // velocities vel_b = m_b ir (the normal one carries gvas, all carry the Roe parts)
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const double gvb = gvel[s][b] + ((b == a) ? gvas : 0.0);
            gm[b] += gvb * ir[s] + ((b == a) ? fsc * gfs_[0] : 0.0);
            gir += gvb * w[1 + b];
        }
        // p = (g-1)(E - 0.5 m2 ir)
        gE += g.gm1 * gp;
        const double gm2 = -0.5 * g.gm1 * ir[s] * gp;
        gir += -0.5 * g.gm1 * m2[s] * gp;
        grho += -gir * ir[s] * ir[s];
        gw[0] += grho;
#pragma unroll
        for (int b = 0; b < DIM; ++b) gw[1 + b] += gm[b] + 2.0 * w[1 + b] * gm2;
        gw[NV - 1] += gE;
    }
}

// ---------------------------------------------------------------------------
// element geometry helpers
// ---------------------------------------------------------------------------

template <int DIM, int K>
struct Geo {
    static constexpr int NV = DIM + 2;
    static constexpr int LOGK = (K == 2) ? 1 : (K == 4) ? 2 : 3;
    static constexpr int KD = (DIM == 2) ? K * K : K * K * K;
    static constexpr int KF = KD / K;
    __device__ static int coord(int c, int a) { return (c >> (a * LOGK)) & (K - 1); }
    __device__ static int stride(int a) { return 1 << (a * LOGK); }
    // index of c inside the face plane orthogonal to a (remaining axes, increasing order)
    __device__ static int trans(int c, int a)
    {
        if (DIM == 2) return coord(c, a == 0 ? 1 : 0);
        if (a == 0) return coord(c, 1) + K * coord(c, 2);
        if (a == 1) return coord(c, 0) + K * coord(c, 2);
        return coord(c, 0) + K * coord(c, 1);
    }
    // cell of face plane index t for axis a at position pos along a
    __device__ static int from_trans(int t, int a, int pos)
    {
        if (DIM == 2) return a == 0 ? (pos + K * t) : (t + K * pos);
        int t0 = t & (K - 1), t1 = t >> LOGK;
        if (a == 0) return pos + K * (t0 + K * t1);
        if (a == 1) return t0 + K * (pos + K * t1);
        return t0 + K * (t1 + K * pos);
    }
    __device__ static int subelem(int c, int n)
    {
        int ns = K / n;
        int s = coord(c, 0) / n + ns * (coord(c, 1) / n);
        if (DIM == 3) s += ns * ns * (coord(c, 2) / n);
        return s;
    }
};

__device__ __forceinline__ int ilog2i(int n) { return n == 8 ? 3 : n == 4 ? 2 : n == 2 ? 1 : 0; }

// Compile-time level hierarchy of a DGFV-TOP scheme on K^DIM subcells: DG levels
// n = TOP, TOP/2, ..., 2 (level index li = 0, 1, ...), their sub-element counts
// and offsets in the per-element blending-factor vector.
template <int DIM, int K, int TOP>
struct Lv {
    static constexpr int NLEV = (TOP == 8) ? 3 : (TOP == 4) ? 2 : 1;
    static constexpr int n(int li) { return TOP >> li; }
    static constexpr int per(int li)
    {
        int r = 1;
        for (int a = 0; a < DIM; ++a) r *= K / n(li);
        return r;
    }
    static constexpr int off(int li)
    {
        int o = 0;
        for (int j = 0; j < li; ++j) o += per(j);
        return o;
    }
    static constexpr int A = off(NLEV);
};

// Exact lane exchange v <- v[lane ^ mask] inside a wavefront, on the VALU (no LDS
// traffic).  Masks below 16 use DPP lane permutations (xor 1 / xor 2: quad permutes;
// xor 4: half-row mirror then quad reverse; xor 8: rotation by 8 inside a 16-lane
// row).  16 and 32 use the row swaps of gfx950: with both operands v, the first
// result holds the lower partner of every pair of 16- (32-) lane halves in both
// halves and the second the upper one, so a lane in the upper half takes the first.
__device__ __forceinline__ int lane_xor_i(int v, int mask)
{
    // every lane reads a valid source lane, so no prior destination value is kept
    // (mov_dpp instead of update_dpp with a zero, which costs a register clear each)
    switch (mask) {
    case 1: return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
    case 4: {
        int t = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);
        return __builtin_amdgcn_mov_dpp(t, 0x1B, 0xF, 0xF, false);
    }
    case 8: return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);
    case 16: {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (threadIdx.x & 16) ? (int)r[0] : (int)r[1];
    }
    case 32: {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (threadIdx.x & 32) ? (int)r[0] : (int)r[1];
    }
    default: return __shfl_xor(v, mask, 64);
    }
}

__device__ __forceinline__ int lane_xor(int v, int mask) { return lane_xor_i(v, mask); }

__device__ __forceinline__ double lane_xor(double v, int mask)
{
    int lo = lane_xor_i(__double2loint(v), mask);
    int hi = lane_xor_i(__double2hiint(v), mask);
    return __hiloint2double(hi, lo);
}

// One butterfly step of a reduction with a commutative operation: op(v, v[lane ^ mask]).
// Across 16- and 32-lane halves the row swap of v with itself leaves the lower half's
// values in one result and the upper half's in the other, in every lane, so op of the
// two results is the step's value without a select (and the same in both halves).
__device__ __forceinline__ void swap_halves(int v, int mask, int &lo, int &hi)
{
    if (mask == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        lo = (int)r[0];
        hi = (int)r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        lo = (int)r[0];
        hi = (int)r[1];
    }
}

template <class Op>
__device__ __forceinline__ int lane_step(int v, int mask, Op op)
{
    if (mask == 16 || mask == 32) {
        int lo, hi;
        swap_halves(v, mask, lo, hi);
        return op(lo, hi);
    }
    return op(v, lane_xor(v, mask));
}

template <class Op>
__device__ __forceinline__ double lane_step(double v, int mask, Op op)
{
    if (mask == 16 || mask == 32) {
        int l0, h0, l1, h1;
        swap_halves(__double2loint(v), mask, l0, h0);
        swap_halves(__double2hiint(v), mask, l1, h1);
        return op(__hiloint2double(l1, l0), __hiloint2double(h1, h0));
    }
    return op(v, lane_xor(v, mask));
}

// Sums of 8 values over the 64 lanes of a wavefront (one 2-D K = 8 element), every lane
// ending with all 8 sums in scalar registers.  A reduce-scatter: one row swap across the
// 32-lane halves pairs value j (kept by the lower lanes) with value j + 4 (kept by the
// upper ones), so each lane adds its partner's copy of the value it keeps; the same across
// 16-lane halves leaves 2 values per lane, an exchange across 8-lane halves 1, value
// (lane >> 3) & 7; a butterfly over the last three bits completes it, and lane 8q holds
// sum q.  17 exchanges instead of the 48 of eight butterflies.
__device__ __forceinline__ void wave_sum8(double *v)
{
    double w[4], x[2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const auto rl = __builtin_amdgcn_permlane32_swap(__double2loint(v[j]), __double2loint(v[4 + j]), false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(__double2hiint(v[j]), __double2hiint(v[4 + j]), false, false);
        w[j] = __hiloint2double((int)rh[0], (int)rl[0]) + __hiloint2double((int)rh[1], (int)rl[1]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const auto rl = __builtin_amdgcn_permlane16_swap(__double2loint(w[j]), __double2loint(w[2 + j]), false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap(__double2hiint(w[j]), __double2hiint(w[2 + j]), false, false);
        x[j] = __hiloint2double((int)rh[0], (int)rl[0]) + __hiloint2double((int)rh[1], (int)rl[1]);
    }
    const bool b3 = (threadIdx.x & 8) != 0;
    double y = (b3 ? x[1] : x[0]) + lane_xor(b3 ? x[0] : x[1], 8);
    y += lane_xor(y, 4);
    y += lane_xor(y, 2);
    y += lane_xor(y, 1);
    const int ylo = __double2loint(y), yhi = __double2hiint(y);
#pragma unroll
    for (int q = 0; q < 8; ++q)
        v[q] = __hiloint2double(__builtin_amdgcn_readlane(yhi, 8 * q), __builtin_amdgcn_readlane(ylo, 8 * q));
}

// OR of a predicate over the workgroup, ordered like a barrier.  A one-wavefront
// workgroup (every 2-D kernel) takes a wave vote after the barrier; the library's
// workgroup reduction behind __syncthreads_or keeps an LDS buffer of its own, which
// would cost the residual kernel one resident workgroup per CU.
template <int NT>
__device__ __forceinline__ bool block_or(bool pred)
{
    if constexpr (NT <= 64) {
        __syncthreads();
        return __any(pred ? 1 : 0) != 0;
    } else {
        return __syncthreads_or(pred ? 1 : 0) != 0;
    }
}

struct OpSum { __device__ double operator()(double a, double b) const { return a + b; } };
struct OpMin { __device__ double operator()(double a, double b) const { return fmin(a, b); } };
struct OpMax { __device__ double operator()(double a, double b) const { return fmax(a, b); } };
struct OpAnd { __device__ int operator()(int a, int b) const { return a & b; } };
struct OpOr { __device__ int operator()(int a, int b) const { return a | b; } };

// Maximum over the lanes that differ from this one in bits [B0, B1) of the lane index:
// one lane exchange per bit with a compile-time mask (maxima are exact in any order)
template <int B0, int B1>
__device__ __forceinline__ double lane_max_bits(double v)
{
    if constexpr (B0 < B1) return lane_max_bits<B0 + 1, B1>(lane_step(v, 1 << B0, OpMax()));
    else return v;
}

// the part of a sub-element reduction across the wavefronts of one element (3-D, K = 8):
// each wavefront holds the partials of its groups (the lanes of one sub-element in that
// wavefront: a whole z layer for the element, a quarter of it for a level-4 sub-element,
// a sixteenth for level 2), already reduced over the group's lanes.  One lane per group
// publishes them in LDS at a dense group index; s_x has 64 slots per wavefront, so one
// call exchanges at most 64 / (groups per wavefront) values: 64 for the element, 16
// for level-4 sub-elements, 4 for level 2 (callers reducing more values at level 2
// split them, see reduce_means).
template <int DIM, int K, int NQ, typename T, typename Op>
__device__ __forceinline__ void subreduce_xwave(T *v, int ln, T *s_x, Op op)
{
    constexpr int LOGK = Geo<DIM, K>::LOGK;
    constexpr int NB = DIM * LOGK;              // bits of the cell index
    if constexpr (NB > 6) {
        static_assert(NB == 9 && NQ <= 16, "at most 16 values per exchange at K = 8");
        constexpr int NW = 8;                   // wavefronts of one element (its z layers)
        if (ln <= 0) return;
        const int lnc = ln < 3 ? ln : 3;
        const int wmask = (1 << lnc) - 1;       // z bits inside the sub-element
        const int tid = threadIdx.x, WG = blockDim.x >> 6;
        const int w = (tid >> 6) & (NW - 1), wbase = (tid >> 6) & ~(NW - 1);
        // a wavefront is an 8 x 8 layer (x = lane bits 0-2, y = bits 3-5): the groups are
        // the (8 >> ln)^2 squares of side n; gi is this lane's square, packed
        const int lx = tid & 7, ly = (tid >> 3) & 7, low = (1 << lnc) - 1;
        const int gi = (lx >> lnc) + ((ly >> lnc) << (3 - lnc)), ng = 1 << (2 * (3 - lnc));
        if (((lx | ly) & low) == 0)             // the group's publishing lane
#pragma unroll
            for (int q = 0; q < NQ; ++q) s_x[(q * WG + (tid >> 6)) * ng + gi] = v[q];
        __syncthreads();
        const int g0 = w & ~wmask;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            T acc[NW];
#pragma unroll
            for (int i = 0; i < NW; ++i) acc[i] = s_x[(q * WG + wbase + i) * ng + gi];
#pragma unroll
            for (int m = 1; m < NW; m <<= 1) {
                if (!(wmask & m)) continue;
#pragma unroll
                for (int i = 0; i < NW; ++i)
                    if (!(i & m)) acc[i] = op(acc[i], acc[i | m]);
            }
            T r = acc[0];                       // acc[g0], by selects (no indexed registers)
#pragma unroll
            for (int i = 1; i < NW; ++i)
                if (i == g0) r = acc[i];
            v[q] = r;
        }
        __syncthreads();
    }
}

// xor-butterfly reduction of NQ values at once over the cells of one level-n
// sub-element (ln = log2 n; ln = LOGK gives the whole element); every lane ends with
// the values of its sub-element.  Bits inside a wavefront use lane exchanges.  Bits
// above them (3-D, K = 8: the bits of the z coordinate, one wavefront per z layer)
// go through LDS with one barrier pair for all NQ values: one lane per group and
// wavefront publishes the group's partials, and every lane combines those of the
// wavefronts of its sub-element pairwise in the butterfly's pairing (the operators are
// commutative, so this is the butterfly's result to the bit).  s_x holds 64 values per
// wavefront of the workgroup.
template <int DIM, int K, int NQ, typename T, typename Op>
__device__ __forceinline__ void subreduce_n(T *v, int ln, T *s_x, Op op)
{
    constexpr int LOGK = Geo<DIM, K>::LOGK;
    constexpr int NB = DIM * LOGK;              // bits of the cell index
#pragma unroll
    for (int bit = 0; bit < (NB < 6 ? NB : 6); ++bit) {
        if (bit % LOGK >= ln) continue;
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = lane_step(v[q], 1 << bit, op);
    }
    subreduce_xwave<DIM, K, NQ>(v, ln, s_x, op);
}

// AND (ALL) or OR of 0/1 votes over the same groups: inside a wavefront one ballot, each
// lane testing the bits of its group (the lanes that differ from it only in the varying
// bits of the cell index), then the cross-wavefront part of subreduce_n
template <int DIM, int K, int NQ, bool ALL>
__device__ __forceinline__ void subvote_n(int *v, int ln, int *s_x)
{
    constexpr int LOGK = Geo<DIM, K>::LOGK;
    constexpr int NB = DIM * LOGK;
    int vary = 0;                               // varying lane bits
#pragma unroll
    for (int bit = 0; bit < (NB < 6 ? NB : 6); ++bit)
        if (bit % LOGK < ln) vary |= 1 << bit;
    unsigned long long pat = 1;                 // lane offsets inside a group: subsets of vary
#pragma unroll
    for (int bit = 0; bit < 6; ++bit)
        if (vary & (1 << bit)) pat |= pat << (1 << bit);
    const unsigned long long gm = pat << ((threadIdx.x & 63) & ~vary);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const unsigned long long m = __ballot(v[q] != 0);
        v[q] = ALL ? ((m & gm) == gm ? 1 : 0) : ((m & gm) != 0 ? 1 : 0);
    }
    if constexpr (ALL) subreduce_xwave<DIM, K, NQ>(v, ln, s_x, OpAnd());
    else subreduce_xwave<DIM, K, NQ>(v, ln, s_x, OpOr());
}

template <int DIM, int K, bool ALL>
__device__ __forceinline__ int subvote(int v, int ln, int *s_x)
{
    subvote_n<DIM, K, 1, ALL>(&v, ln, s_x);
    return v;
}

template <int DIM, int K, typename T, typename Op>
__device__ __forceinline__ T subreduce(T v, int ln, T *s_x, Op op)
{
    subreduce_n<DIM, K, 1>(&v, ln, s_x, op);
    return v;
}

// sums of the NV conserved variables over each level-n sub-element; a 3-D K = 8
// level-2 sub-element takes them in two exchanges (4 + 1 values, see subreduce_xwave)
template <int DIM, int K, int NV>
__device__ __forceinline__ void reduce_means(double *mn, int ln, double *s_x)
{
    if constexpr (DIM * Geo<DIM, K>::LOGK > 6 && NV > 4) {
        if (ln <= 1) {
            subreduce_n<DIM, K, 4>(mn, ln, s_x, OpSum());
            subreduce_n<DIM, K, NV - 4>(mn + 4, ln, s_x, OpSum());
            return;
        }
    }
    subreduce_n<DIM, K, NV>(mn, ln, s_x, OpSum());
}

// blocked n-mode product: out = sum_m M[lo][m] * src[base + m*stride] along axis a
// for level n (lo = position of c inside its level-n sub-element along a)
template <int DIM, int K>
__device__ __forceinline__ double bapply(const double *src, int c, int a, int n, CDbl *M)
{
    typedef Geo<DIM, K> G;
    int st = G::stride(a);
    int lo = G::coord(c, a) & (n - 1);
    int base = c - lo * st;
    CDbl *row = M + lo * n;
    double acc = 0.0;
    for (int m = 0; m < n; ++m) acc += row[m] * src[base + m * st];
    return acc;
}

// weights theta of one cell from an element's alpha vector (eq. blending-weights)
template <class LV>
__device__ __forceinline__ void theta_from_alpha(const double *al, const int *sidx, double *th)
{
    double prod = 1.0;
#pragma unroll
    for (int li = 0; li < LV::NLEV; ++li) {
        double a = al[LV::off(li) + sidx[li]];
        th[1 + li] = a * prod;
        prod *= (1.0 - a);
    }
    th[0] = prod;
}

template <int DIM, int K, class LV>
__device__ __forceinline__ void subidx_all(int c, int *sidx)
{
#pragma unroll
    for (int li = 0; li < LV::NLEV; ++li) sidx[li] = Geo<DIM, K>::subelem(c, LV::n(li));
}

template <int DIM, int K>
__device__ __forceinline__ long long gindex(const KArgs &P, const int *e3, int c)
{
    typedef Geo<DIM, K> G;
    long long gx = (long long)e3[0] * K + G::coord(c, 0);
    long long gy = (long long)e3[1] * K + G::coord(c, 1);
    long long gz = DIM == 3 ? (long long)e3[2] * K + G::coord(c, 2) : 0;
    return gx + (long long)P.G[0] * (gy + (long long)P.G[1] * gz);
}

__device__ __forceinline__ void elem3(const KArgs &P, int e, int *e3)
{
    e3[0] = e % P.ne[0];
    int r = e / P.ne[0];
    e3[1] = r % P.ne[1];
    e3[2] = r / P.ne[1];
}

// neighbour element across face (axis a, side 0 = low, 1 = high); -1 at an outflow boundary
template <int DIM>
__device__ __forceinline__ int neighbour(const KArgs &P, const int *e3, int a, int side)
{
    int f[3] = {e3[0], e3[1], e3[2]};
    int d = side ? 1 : -1;
    f[a] += d;
    const int na = arg_ne(P, a);
    if (f[a] < 0 || f[a] >= na) {
        if (arg_bc(P, a) != SEDG_PERIODIC) return -1;
        f[a] = (f[a] + na) % na;
    }
    return f[0] + P.ne[0] * (f[1] + P.ne[1] * f[2]);
}

// face buffer slot: [elem][axis][side][var][face-plane index]
template <int DIM, int K>
__device__ __forceinline__ long long fb_index(int e, int a, int side, int v, int t)
{
    constexpr int NV = DIM + 2, KF = Geo<DIM, K>::KF;
    return ((((long long)e * DIM + a) * 2 + side) * NV + v) * KF + t;
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup i on XCD i mod 8),
// each XCD with its own L2.  The kernels that read their neighbours' face data
// remap workgroups so that every XCD works on one contiguous range of tiles: an
// element's x-neighbours are then on the same XCD and their face data in its L2.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n >> 3, r = n & 7, x = b & 7, i = b >> 3;
    return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// ---------------------------------------------------------------------------
// analyse kernel
// ---------------------------------------------------------------------------
//
// Levels are visited as the multi-level algorithm descends (all levels in
// EXTERNAL mode, the top level in FORCE_DG, none in FORCE_FV); the children's
// reconstruction needed by the indicator of level n is the reconstruction of
// level n/2, so every reconstruction is computed once.  Sub-element means and
// the minima of the check set are reduced only on levels where some
// sub-element fails the permissibility check (beta = 1 needs neither).

template <int DIM, int K, int TOP, int EPB>
struct AnalyseSmem {
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    double u[EPB][G::NV][G::KD];
    double r[EPB][2][G::NV][G::KD];         // reconstructions of the current level and of its children
    double t[EPB][G::NV][G::KD];            // temporary; primitive variables in the indicator
    double x[EPB * G::KD];                  // reduction exchange
    int ix[EPB * G::KD];
    double lam[EPB * G::KD / 64 + 1];
    double al[EPB][LV::A];                  // per sub-element: blending factor,
    double be[EPB][LV::A];                  //   squeezing parameter,
    double mean[EPB][G::NV][LV::A];         //   mean value
};

// unlimited reconstruction of level li of every variable into dst: u x_1 R x_2 R (x_3 R)
template <int DIM, int K, int TOP, int EPB>
__device__ __forceinline__ void recon_level(AnalyseSmem<DIM, K, TOP, EPB> &S, int le, int c, CTab &T, int n,
                                            double (*dst)[Geo<DIM, K>::KD])
{
    constexpr int NV = Geo<DIM, K>::NV;
    if (DIM == 2) {
        for (int v = 0; v < NV; ++v) S.t[le][v][c] = bapply<DIM, K>(S.u[le][v], c, 0, n, T.R);
        __syncthreads();
        for (int v = 0; v < NV; ++v) dst[v][c] = bapply<DIM, K>(S.t[le][v], c, 1, n, T.R);
    } else {
        for (int v = 0; v < NV; ++v) dst[v][c] = bapply<DIM, K>(S.u[le][v], c, 0, n, T.R);
        __syncthreads();
        for (int v = 0; v < NV; ++v) S.t[le][v][c] = bapply<DIM, K>(dst[v], c, 1, n, T.R);
        __syncthreads();
        for (int v = 0; v < NV; ++v) dst[v][c] = bapply<DIM, K>(S.t[le][v], c, 2, n, T.R);
    }
    __syncthreads();
}

// one tile (EPB elements) of the analyse kernel; every thread of the workgroup calls it
template <int DIM, int K, int TOP, int EPB>
__device__ __forceinline__ void analyse_body(const KArgs &P, int tile, AnalyseSmem<DIM, K, TOP, EPB> &S)
{
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    constexpr int NV = G::NV, KD = G::KD;
    const int tid = threadIdx.x;
    const int le = tid / KD, c = tid % KD;
    const int e = tile * EPB + le;
    const bool act = e < P.nel;
    const int ee = act ? e : P.nel - 1;
    int e3[3];
    elem3(P, ee, e3);
    const long long g = gindex<DIM, K>(P, e3, c);
    const Gas gam = {P.gamma, P.gm1};

    double ub[NV];
    for (int v = 0; v < NV; ++v) {
        ub[v] = P.u[v * P.dof + g];
        S.u[le][v][c] = ub[v];
    }
    // state check and CFL eigenvalue estimate of the mean values
    {
        bool fin = true;
        for (int v = 0; v < NV; ++v) fin = fin && isfinite(ub[v]);
        bool ok = fin && permissible<DIM>(ub, gam);
        if (act && !ok) atomicMin(P.err, P.err_base + e);
        if (P.lam_part) {
            double lam = 0.0;
            if (act && ok) {
                double cs = sqrt(gam.g * pressure<DIM>(ub, gam) / ub[0]);
                for (int a = 0; a < DIM; ++a) lam = fmax(lam, fabs(ub[1 + a] / ub[0]) + cs);
            }
            lam = lane_max_bits<0, 6>(lam);
            if ((tid & 63) == 0) S.lam[tid >> 6] = lam;
            __syncthreads();
            if (tid == 0) {
                double m = 0.0;
                for (int wv = 0; wv < (EPB * KD + 63) / 64; ++wv) m = fmax(m, S.lam[wv]);
                // non-negative doubles order like their bit patterns: an integer max is exact
                atomicMax((unsigned long long *)&P.lam_part[tile & P.lam_mask],
                          (unsigned long long)__double_as_longlong(m));
            }
        }
    }
    if constexpr (KD == 64) {
        // one element per wavefront: a row swap across the 32-lane halves leaves the lower
        // lanes the density maxima of both halves and the upper ones the energy maxima,
        // then a butterfly over the other five bits (maxima are exact in any order)
        const auto rl = __builtin_amdgcn_permlane32_swap(__double2loint(ub[0]), __double2loint(fabs(ub[NV - 1])),
                                                         false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(__double2hiint(ub[0]), __double2hiint(fabs(ub[NV - 1])),
                                                         false, false);
        double m = fmax(__hiloint2double((int)rh[0], (int)rl[0]), __hiloint2double((int)rh[1], (int)rl[1]));
        m = lane_max_bits<0, 5>(m);
        if (act && (c & 31) == 0) P.scale[2 * (long long)e + (c >> 5)] = m;
    } else {
        double sc[2] = {ub[0], fabs(ub[NV - 1])};
        subreduce_n<DIM, K, 2>(sc, G::LOGK, S.x, OpMax());
        if (act && c == 0) {
            P.scale[2 * (long long)e] = sc[0];
            P.scale[2 * (long long)e + 1] = sc[1];
        }
    }
    __syncthreads();

    const bool given = P.mode == SEDG_EXTERNAL || P.mode == SEDG_RANDOM;   // factors not from the indicator
    const long long draw = (P.mode == SEDG_RANDOM) ? *P.draw : 0;
    for (int q = c; q < LV::A; q += KD) {
        double a0 = 0.0;
        if (P.mode == SEDG_EXTERNAL) a0 = P.alpha_in[(long long)ee * LV::A + q];
        else if (P.mode == SEDG_RANDOM)
            a0 = splitmix_u01(P.seed, (unsigned long long)((draw * P.nel + ee) * LV::A + q));
        S.al[le][q] = a0;
        S.be[le][q] = 1.0;
        for (int v = 0; v < NV; ++v) S.mean[le][v][q] = 0.0;
    }
    __syncthreads();

    int broke = 0;
    int have_rec = -1;      // level index whose reconstruction sits in S.r[li & 1]
#pragma unroll
    for (int li = 0; li < LV::NLEV; ++li) {
        const int n = LV::n(li), ln = ilog2i(n);
        const bool enabled = (P.level_mask == 0) || ((P.level_mask >> ln) & 1u);
        bool visit;
        if (given) visit = true;
        else if (P.mode == SEDG_FORCE_DG) visit = (li == 0);
        else if (P.mode == SEDG_FORCE_FV) visit = false;
        else visit = enabled && !broke;
        if (!block_or<EPB * KD>(visit)) {
            if (P.mode != SEDG_ADAPTIVE || !block_or<EPB * KD>(!broke)) break;
            continue;
        }
        CTab &T = P.tabs[li];
        if (have_rec != li) {
            recon_level<DIM, K, TOP, EPB>(S, le, c, T, n, S.r[le][li & 1]);
            have_rec = li;
        }
        double (*R0)[KD] = S.r[le][li & 1];
        // ---- squeezing parameter (eq. calc-squeezing-parameter) ----
        double pt[NV];
        for (int v = 0; v < NV; ++v) pt[v] = R0[v][c];
        double pp = pressure<DIM>(pt, gam);
        int ok = (pt[0] > 0.0 && pp > 0.0) ? 1 : 0;
        double rmin = pt[0], pmin = pp;
        if (DIM == 2 && n >= 4) {
            // the sub-element's 4n face-node traces, one per cell of the sub-element: the
            // cell at local (lx, ly) with ly < 4 takes face ly (x low, x high, y low, y high)
            // at face node lx, so that one pass covers both axes and both sides, and every
            // trace lies in the sub-element whose reductions below take it
            const int lx = G::coord(c, 0) & (n - 1), ly = G::coord(c, 1) & (n - 1);
            if (KD == 64 && n == 8) {
                // the element's 32 traces over all 64 lanes: the lower half (ly < 4) forms
                // variables 0 and 1 of its trace, the lane 32 above it variables 2 and 3 of
                // the same trace, which a row swap then hands down (the same sums)
                const int lt = ly & 3, vb = (ly >> 2) * 2;
                const int a = lt >> 1;
                const bool hi = (lt & 1) != 0;
                const int b0 = c - lx - K * ly;     // low corner of the element (0)
                const int base = a == 0 ? b0 + K * lx : b0 + lx, st = a == 0 ? 1 : K;
                double h2[2];
                for (int j = 0; j < 2; ++j) {
                    double s = 0.0;
                    for (int m = 0; m < n; ++m) s += (hi ? T.bp[m] : T.bm[m]) * R0[vb + j][base + m * st];
                    h2[j] = s;
                }
                const double o0 = lane_xor(h2[0], 32), o1 = lane_xor(h2[1], 32);
                if (ly < 4) {
                    pt[0] = h2[0];
                    pt[1] = h2[1];
                    pt[2] = o0;
                    pt[3] = o1;
                    double q = pressure<DIM>(pt, gam);
                    if (!(pt[0] > 0.0 && q > 0.0)) ok = 0;
                    rmin = fmin(rmin, pt[0]);
                    pmin = fmin(pmin, q);
                }
            } else if (ly < 4) {
                const int a = ly >> 1;
                const bool hi = (ly & 1) != 0;
                const int b0 = c - lx - K * ly;     // low corner of the sub-element
                const int base = a == 0 ? b0 + K * lx : b0 + lx, st = a == 0 ? 1 : K;
                for (int v = 0; v < NV; ++v) {
                    double s = 0.0;
                    for (int m = 0; m < n; ++m) s += (hi ? T.bp[m] : T.bm[m]) * R0[v][base + m * st];
                    pt[v] = s;
                }
                double q = pressure<DIM>(pt, gam);
                if (!(pt[0] > 0.0 && q > 0.0)) ok = 0;
                rmin = fmin(rmin, pt[0]);
                pmin = fmin(pmin, q);
            }
        } else
        for (int a = 0; a < DIM; ++a) {
            // a lane on the low face of its sub-element takes the trace with b^-, one on
            // the high face the trace with b^+ (both sides in one pass; n >= 2)
            const int lo = G::coord(c, a) & (n - 1);
            const bool hi = (lo == n - 1);
            if (!(lo == 0 || hi)) continue;
            const int st = G::stride(a), base = c - lo * st;
            for (int v = 0; v < NV; ++v) {
                double s = 0.0;
                for (int m = 0; m < n; ++m) s += (hi ? T.bp[m] : T.bm[m]) * R0[v][base + m * st];
                pt[v] = s;
            }
            double q = pressure<DIM>(pt, gam);
            if (!(pt[0] > 0.0 && q > 0.0)) ok = 0;
            rmin = fmin(rmin, pt[0]);
            pmin = fmin(pmin, q);
        }
        ok = subvote<DIM, K, true>(ok, ln, S.ix);
        double b = 1.0;
        const int sub = G::subelem(c, n);
        const bool leader = ((G::coord(c, 0) | G::coord(c, 1) | (DIM == 3 ? G::coord(c, 2) : 0)) & (n - 1)) == 0;
        if (block_or<EPB * KD>(visit && !ok)) {
            double nd = (DIM == 2) ? n * n : n * n * n;
            double mn[NV], mm[2] = {rmin, pmin};
            for (int v = 0; v < NV; ++v) mn[v] = S.u[le][v][c];   // from LDS: ub need not stay live
            reduce_means<DIM, K, NV>(mn, ln, S.x);
            for (int v = 0; v < NV; ++v) mn[v] /= nd;
            subreduce_n<DIM, K, 2>(mm, ln, S.x, OpMin());
            rmin = mm[0];
            pmin = mm[1];
            if (!ok) {
                double rmean = mn[0], pmean = pressure<DIM>(mn, gam);
                double eps = fmin(1e-20, fmin(rmean, pmean));
                double br = (rmean - rmin > 0.0) ? (rmean - eps) / (rmean - rmin) : 1.0;
                double bq = (pmean - pmin > 0.0) ? (pmean - eps) / (pmean - pmin) : 1.0;
                b = fmin(fmin(br, bq), 1.0);
            }
            if (visit && leader)
                for (int v = 0; v < NV; ++v) S.mean[le][v][LV::off(li) + sub] = mn[v];
        }
        if (!visit) b = 1.0;
        if (leader) S.be[le][LV::off(li) + sub] = b;
        // children reconstruction = next level's reconstruction
        const bool need_next = (li + 1 < LV::NLEV) &&
                               (given || (P.mode == SEDG_ADAPTIVE && n >= 4));
        if (block_or<EPB * KD>(visit && need_next)) {
            recon_level<DIM, K, TOP, EPB>(S, le, c, P.tabs[li + 1], n / 2, S.r[le][(li + 1) & 1]);
            have_rec = li + 1;
        }
        if (P.mode != SEDG_ADAPTIVE) continue;
        // ---- blending factor (eq. calc-blending-factor) ----
        double a = 0.0;
        if (n == 2) {
            a = (b < P.beta_L) ? 0.0 : b;
        } else {
            CTab &H = P.tabs[li + 1];
            double (*R1)[KD] = S.r[le][(li + 1) & 1];
            const int h = n / 2;
            double wv[NV];
            for (int v = 0; v < NV; ++v) pt[v] = R0[v][c];
            int bad = (pt[0] > 0.0) ? 0 : 1;
            wv[0] = pt[0];
            for (int d = 0; d < DIM; ++d) wv[1 + d] = pt[1 + d] / pt[0];
            wv[DIM + 1] = pressure<DIM>(pt, gam);
            for (int v = 0; v < NV; ++v) S.t[le][v][c] = wv[v];
            __syncthreads();
            double sn[NV], sh[NV];
            {
                double wq = 1.0;
                for (int d = 0; d < DIM; ++d) wq *= T.w[G::coord(c, d) & (n - 1)];
                for (int v = 0; v < NV; ++v) {
                    double s = 0.0;
                    for (int d = 0; d < DIM; ++d) s += fabs(bapply<DIM, K>(S.t[le][v], c, d, n, T.Dcal));
                    sn[v] = wq * s;
                }
            }
            __syncthreads();
            for (int v = 0; v < NV; ++v) pt[v] = R1[v][c];
            bad |= (pt[0] > 0.0) ? 0 : 1;
            wv[0] = pt[0];
            for (int d = 0; d < DIM; ++d) wv[1 + d] = pt[1 + d] / pt[0];
            wv[DIM + 1] = pressure<DIM>(pt, gam);
            for (int v = 0; v < NV; ++v) S.t[le][v][c] = wv[v];
            __syncthreads();
            {
                double wq = (DIM == 2) ? 0.5 : 0.25;   // child measure in parent coordinates
                for (int d = 0; d < DIM; ++d) wq *= H.w[G::coord(c, d) & (h - 1)];
                for (int v = 0; v < NV; ++v) {
                    double s = 0.0;
                    for (int d = 0; d < DIM; ++d) s += fabs(bapply<DIM, K>(S.t[le][v], c, d, h, H.Dcal));
                    sh[v] = wq * s;
                }
            }
            __syncthreads();
            if constexpr (DIM == 2 && K == 8) {
                if (ln == G::LOGK) {
                    // the whole element (one wavefront): reduce-scatter of the 8 sums
                    double snh[2 * NV];
                    for (int v = 0; v < NV; ++v) {
                        snh[v] = sn[v];
                        snh[NV + v] = sh[v];
                    }
                    wave_sum8(snh);
                    for (int v = 0; v < NV; ++v) {
                        sn[v] = snh[v];
                        sh[v] = snh[NV + v];
                    }
                } else {
                    for (int v = 0; v < NV; ++v) {
                        sn[v] = subreduce<DIM, K>(sn[v], ln, S.x, OpSum());
                        sh[v] = subreduce<DIM, K>(sh[v], ln, S.x, OpSum());
                    }
                }
            } else if constexpr (G::KD <= 64) {
                for (int v = 0; v < NV; ++v) {
                    sn[v] = subreduce<DIM, K>(sn[v], ln, S.x, OpSum());
                    sh[v] = subreduce<DIM, K>(sh[v], ln, S.x, OpSum());
                }
            } else {
                double snh[2 * NV];
                for (int v = 0; v < NV; ++v) {
                    snh[v] = sn[v];
                    snh[NV + v] = sh[v];
                }
                subreduce_n<DIM, K, 2 * NV>(snh, ln, S.x, OpSum());   // n >= 4: one exchange
                for (int v = 0; v < NV; ++v) {
                    sn[v] = snh[v];
                    sh[v] = snh[NV + v];
                }
            }
            bad = subvote<DIM, K, false>(bad, ln, S.ix);
            double amin = 1.0;
            int nonfin = 0;
            for (int v = 0; v < NV; ++v) {
                double den = fmax(fmax(sh[v], sn[v]), P.sigma_floor);
                const double d = fabs(sn[v] - sh[v]);
                // below 0.99 tau_S den the rounded quotient lies below tau_S for certain (the
                // bound's and the quotient's rounding are some 1e-16 relative), so the ramp
                // clamps to 0 and 1 - 0 leaves amin as it is: the division is skipped
                if (d < P.ind_quick * den) continue;
                double r = d / den;
                double x = P.tau_A * (r - P.tau_S);
                if (!isfinite(x)) nonfin = 1;
                double cut = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
                amin = fmin(amin, 1.0 - cut);
            }
            a = (bad || nonfin) ? 0.0 : amin;
            if (b < P.beta_L) a = 0.0;
        }
        if (!visit) a = 0.0;
        // level decision over the whole element (strict comparisons)
        int hl[2] = {(a > P.alpha_H) ? 1 : 0, (a < P.alpha_L) ? 1 : 0};
        if constexpr (G::KD <= 64) {
            hl[0] = subvote<DIM, K, true>(hl[0], G::LOGK, S.ix);
            hl[1] = subvote<DIM, K, true>(hl[1], G::LOGK, S.ix);
        } else {
            subvote_n<DIM, K, 2, true>(hl, G::LOGK, S.ix);
        }
        const int hi = hl[0], lo = hl[1];
        if (visit) {
            if (hi) { a = 1.0; broke = 1; }
            else if (lo) a = 0.0;
            if (leader) S.al[le][LV::off(li) + sub] = a;
        }
    }
    if (P.mode == SEDG_FORCE_DG)
        for (int q = c; q < LV::off(1 < LV::NLEV ? 1 : 0) + (LV::NLEV > 1 ? 0 : LV::A); q += KD) S.al[le][q] = 1.0;
    __syncthreads();
    // publish alpha, beta and the sub-element means (coalesced); a mean enters the
    // blends only as (1 - beta) <u>_s, so it is stored only for a squeezed sub-element
    // (beta < 1), and its readers take 0 elsewhere
    if (act)
        for (int q = c; q < LV::A; q += KD) {
            const double bq = S.be[le][q];
            P.alpha[(long long)e * LV::A + q] = S.al[le][q];
            P.beta[(long long)e * LV::A + q] = bq;
            if (bq < 1.0)
                for (int v = 0; v < NV; ++v) P.mean[((long long)e * NV + v) * LV::A + q] = S.mean[le][v][q];
        }
    // blended interface states on the element faces: theta_FV * mean + sum_n theta_n *
    // ((1 - beta) <u>_s + beta * (u_s x_a E^{+-})) (cascade of Sec. 2.6, App. eq. 3D-prolongation).
    // One task per (element, face, face cell), spread over the workgroup's lanes, rather
    // than each boundary lane looping over the faces its cell touches; with at least
    // twice as many lanes as tasks (2-D, K = 8) the variables of a task are split over
    // two lanes.
    {
        constexpr int NF = 2 * DIM, KF = G::KF, NT = EPB * NF * KF;
        constexpr int VS = (EPB * KD >= 2 * NT) ? 2 : 1, VPL = (NV + VS - 1) / VS;
        for (int w = tid; w < NT * VS; w += EPB * KD) {
            const int tsk = w % NT, v0 = (w / NT) * VPL;
            const int tle = tsk / (NF * KF), rem = tsk - tle * (NF * KF), f = rem / KF, t = rem - f * KF;
            const int a = f >> 1, sd = f & 1;
            const int cc = G::from_trans(t, a, sd ? K - 1 : 0);
            const int te = tile * EPB + tle;
            int sidx[MAXLEV];
            subidx_all<DIM, K, LV>(cc, sidx);
            double th[MAXLEV + 1];
            theta_from_alpha<LV>(S.al[tle], sidx, th);
            double st[VPL];
            for (int j = 0; j < VPL; ++j) st[j] = (v0 + j < NV) ? th[0] * S.u[tle][v0 + j][cc] : 0.0;
#pragma unroll
            for (int li = 0; li < LV::NLEV; ++li) {
                if (th[1 + li] == 0.0) continue;
                CTab &T = P.tabs[li];
                int n = LV::n(li);
                CDbl *E = sd ? T.Ep : T.Em;
                const int q = LV::off(li) + sidx[li];
                double b = S.be[tle][q];
                for (int j = 0; j < VPL; ++j) {
                    if (v0 + j >= NV) break;
                    double tr = bapply<DIM, K>(S.u[tle][v0 + j], cc, a, n, E);
                    st[j] += th[1 + li] * ((1.0 - b) * S.mean[tle][v0 + j][q] + b * tr);
                }
            }
            if (te < P.nel)
                for (int j = 0; j < VPL; ++j)
                    if (v0 + j < NV) P.fbuf[fb_index<DIM, K>(te, a, sd, v0 + j, t)] = st[j];
        }
    }
}

template <int DIM, int K, int TOP, int EPB>
__global__ void __launch_bounds__((EPB * Geo<DIM, K>::KD))
__attribute__((amdgpu_waves_per_eu(DIM == 2 ? 4 : 2, 8))) analyse_kernel(KArgs P)
{
    __shared__ AnalyseSmem<DIM, K, TOP, EPB> S;
    // XCD-contiguous tiles: horizontally adjacent elements share the 128-B lines of the
    // state, and an XCD's L2 then serves the second element its half
    analyse_body<DIM, K, TOP, EPB>(P, xcd_tile(blockIdx.x, gridDim.x), S);
}

// ---------------------------------------------------------------------------
// residual kernel
// ---------------------------------------------------------------------------
//
// Per element: (1) weights of every cell from the element's alpha; (2) unique
// common fluxes on the faces some level uses - the element faces always, an
// interior subcell face only when the FV level or a DG level whose sub-element
// boundary contains it is active - processed K faces per round, one lane per
// face subcell; (3) the FV part, then for each active DG level the squeezed
// reconstruction, nodal fluxes, Dhat along the flux axis, P along the others
// and the Bhat surface term; (4) blend and store (SSP-RK3 stage fused).
// In 3-D the flux buffer holds one axis at a time (LDS budget): the element is
// processed in one pass per axis, the squeezed nodal values of each level are
// reconstructed in the first pass and kept for the others; in 2-D all axes are held.

template <int DIM, int K, int TOP, int EPB>
struct ResidualSmem {
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    static constexpr bool AXO = (DIM == 3);
    static constexpr int NAX = AXO ? 1 : DIM;
    double u[EPB][G::NV][G::KD];
    double F[EPB][NAX][G::NV][(K + 1) * G::KF];
    // temporary of the contraction passes; between them (active-level vote, face
    // fluxes) its first two variables serve as the lane exchange buffers
    double tmp[EPB][G::NV][G::KD];
    // 3-D: the reconstruction's first pass and the nodal fluxes (2-D stages both in tmp)
    double nod[AXO ? EPB : 1][AXO ? G::NV : 1][AXO ? G::KD : 1];
    double al[EPB][LV::A];
    double mean[EPB][G::NV][LV::A];
    double be[EPB][LV::A];
    int act[EPB][MAXLEV + 1];
    // 3-D: the squeezed nodal values of every level, reconstructed in the first axis pass
    // and reused by the other two
    double nodc[AXO ? EPB : 1][AXO ? LV::NLEV : 1][AXO ? G::NV : 1][AXO ? G::KD : 1];
};

// theta of the cell across an element face, from the neighbour's alpha
template <int DIM, int K, class LV>
__device__ __forceinline__ void theta_cell_of(const double *al, int cell, double *th)
{
    int sidx[MAXLEV];
    subidx_all<DIM, K, LV>(cell, sidx);
    theta_from_alpha<LV>(al, sidx, th);
}

// The two sides of an element face for the lane at transverse position t: the
// element's own face state and weights, the neighbour's (nb < 0: a domain boundary,
// where the exterior state is the boundary cell's mean and the exterior weights mirror
// the own side), the data scales of the pair and the
// cells whose means replace a non-admissible FV input (element -1: own element).
// The face-buffer and scale loads of both sides are issued together, unconditionally
// (a boundary lane reads its own element), so that one memory latency covers them.
template <int DIM, int K, class LV>
__device__ __forceinline__ void element_face_sides(const KArgs &P, int ee, int fa, int t, bool high, int nb,
                                                   const double *al_own, const double *al_nb, double own_sr,
                                                   double own_se, double *uL, double *uR, double *thL, double *thR,
                                                   int &mLe, int &mLc, int &mRe, int &mRc, double &srho, double &sE)
{
    constexpr int NV = DIM + 2;
    typedef Geo<DIM, K> G;
    const int sdo = high ? 1 : 0;
    const int nbc = nb >= 0 ? nb : ee;
    double uo[NV], un[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        uo[v] = P.fbuf[fb_index<DIM, K>(ee, fa, sdo, v, t)];
        un[v] = P.fbuf[fb_index<DIM, K>(nbc, fa, 1 - sdo, v, t)];
    }
    const double nsr = P.scale[2 * (long long)nbc], nse = P.scale[2 * (long long)nbc + 1];
    const int co = G::from_trans(t, fa, high ? K - 1 : 0), cn = G::from_trans(t, fa, high ? 0 : K - 1);
    double tho[MAXLEV + 1], thn[MAXLEV + 1];
    theta_cell_of<DIM, K, LV>(al_own, co, tho);
    if (nb >= 0) {
        theta_cell_of<DIM, K, LV>(al_nb, cn, thn);
        srho = fmax(nsr, own_sr);
        sE = fmax(nse, own_se);
    } else {
        // outflow boundary (zero gradient of the subcell means): the exterior state is the
        // mean of the element's boundary cell, the exterior weights mirror its own
        for (int l = 0; l <= LV::NLEV; ++l) thn[l] = tho[l];
        int e3o[3];
        elem3(P, ee, e3o);
        const long long gco = gindex<DIM, K>(P, e3o, co);
#pragma unroll
        for (int v = 0; v < NV; ++v) un[v] = P.u[v * P.dof + gco];
    }
    const int me = nb >= 0 ? nb : -1, mc = nb >= 0 ? cn : co;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        uL[v] = high ? uo[v] : un[v];
        uR[v] = high ? un[v] : uo[v];
    }
    for (int l = 0; l <= LV::NLEV; ++l) {
        thL[l] = high ? tho[l] : thn[l];
        thR[l] = high ? thn[l] : tho[l];
    }
    mLe = high ? -1 : me;
    mLc = high ? co : mc;
    mRe = high ? me : -1;
    mRc = high ? mc : co;
}

// Stage an element's state (and, for the adjoint, its adjoint state), blending
// factors, squeezing parameters and sub-element means in LDS.  Every global load is
// issued before the first LDS store, so that one memory latency covers them all (each
// lane holds at most one entry of the per-element vectors: A <= K^d).  The means are
// read only for squeezed sub-elements (beta < 1; only (1 - beta) <u>_s enters the
// blends, and the analysis stores no others): 0 elsewhere.
template <int DIM, int K, class LV, bool LAM, class SM>
__device__ __forceinline__ void preload_element(const KArgs &P, SM &S, int le, int c, int ee, long long g)
{
    constexpr int NV = DIM + 2;
    static_assert(LV::A <= Geo<DIM, K>::KD, "one factor per lane");
    double uv[NV], lv[NV], mv[NV], ao = 0.0, bo = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        uv[v] = P.u[v * P.dof + g];
        if constexpr (LAM) lv[v] = P.lam[v * P.dof + g];
    }
    const bool hq = c < LV::A;
    for (int v = 0; v < NV; ++v) mv[v] = 0.0;
    if (hq) {
        ao = P.alpha[(long long)ee * LV::A + c];
        bo = P.beta[(long long)ee * LV::A + c];
        if (bo < 1.0)
#pragma unroll
            for (int v = 0; v < NV; ++v) mv[v] = P.mean[((long long)ee * NV + v) * LV::A + c];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        S.u[le][v][c] = uv[v];
        if constexpr (LAM) S.lam[le][v][c] = lv[v];
    }
    if (hq) {
        S.al[le][c] = ao;
        S.be[le][c] = bo;
#pragma unroll
        for (int v = 0; v < NV; ++v) S.mean[le][v][c] = mv[v];
    }
}

// The needed faces of na axes starting at a0: first the two element faces of each
// axis, then the interior faces at multiples of 'step' (1 when the FV level is
// active, else the smallest active DG level; K leaves none).
template <int K>
__device__ __forceinline__ int face_count(int na, int step, bool skip_elem = false)
{
    return na * ((skip_elem ? 0 : 2) + K / step - 1);
}

template <int K>
__device__ __forceinline__ void face_at(int a0, int na, int step, int fidx, int *fa, int *fk, bool skip_elem = false)
{
    if (!skip_elem && fidx < 2 * na) {
        *fa = a0 + (fidx >> 1);
        *fk = (fidx & 1) * K;
    } else {
        int j = fidx - (skip_elem ? 0 : 2 * na), cnt = K / step - 1;
        *fa = a0 + j / cnt;
        *fk = step * (1 + j % cnt);
    }
}

// The common flux F* at the face subcells of one face per group of KF lanes (the
// lane's face node t; the group's face cells start at sbase in the exchange buffers):
// the DG candidates of every level whose sub-element boundary contains the face, then
// the FV candidate with the remaining weight (R4, R17).  uL, uR, thL, thR: the blended
// interface states and weights on both sides; srho, sE: the data scales of the two
// elements; (mLe, mLc), (mRe, mRc): the cells whose means replace a non-admissible FV
// input (element -1: own element ee, read from uown in LDS when given, else from
// global memory).  wsL, wsR: LDS exchange buffers of the element's lanes (lane c);
// every lane of the workgroup (NT threads) calls it with the same face count.
template <int DIM, int K, class LV, int NT, bool WIDE = false>
__device__ __forceinline__ void common_flux(const KArgs &P, double *wsL, double *wsR, int c, int sbase, int t, bool has,
                                            int fa, int k, const double *uL, const double *uR, const double *thL,
                                            const double *thR, double srho, double sE, int mLe, int mLc, int mRe,
                                            int mRc, const double *uown, int ee, double *F)
{
    typedef Geo<DIM, K> G;
    constexpr int NV = G::NV, KD = G::KD;
    const Gas gam = {P.gamma, P.gm1};
    // DG candidates level by level: R along the face, HLLE at the face nodes, P back
    double thFV = 1.0;
    for (int v = 0; v < NV; ++v) F[v] = 0.0;
#pragma unroll
    for (int li = 0; li < LV::NLEV; ++li) {
        // uniform skip: no element of the block has this level active on a needed face
        if (!block_or<NT>(has && (k % LV::n(li) == 0) && (thL[1 + li] != 0.0 || thR[1 + li] != 0.0)))
            continue;
        CTab &T = P.tabs[li];
        const int n = LV::n(li), ln = ilog2i(n);
        const double tb = 0.5 * (thL[1 + li] + thR[1 + li]);
        const bool need = has && (k % n == 0) && (tb != 0.0);
        double nl[NV], nr[NV];
        int lo0, lo1 = 0, tb0, tb1 = 0;
        if (DIM == 2) { lo0 = t & (n - 1); tb0 = t - lo0; }
        else {
            int t0 = t & (K - 1), t1 = t >> G::LOGK;
            lo0 = t0 & (n - 1); tb0 = t0 - lo0;
            lo1 = t1 & (n - 1); tb1 = t1 - lo1;
        }
        const int t0 = t - K * (t >> G::LOGK), t1 = t >> G::LOGK;   // 3-D face coordinates
        if constexpr (WIDE) {
            // every variable through the exchange buffers at once (NV x NT doubles each):
            // one LDS round trip per pass instead of one per variable
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                wsL[v * NT + c] = uL[v];
                wsR[v * NT + c] = uR[v];
            }
            __syncthreads();
            if (DIM == 2) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double sl = 0.0, sr = 0.0;
                    if (need)
                        for (int m = 0; m < n; ++m) {
                            double Rm = T.R[lo0 * n + m];
                            sl += Rm * wsL[v * NT + sbase + tb0 + m];
                            sr += Rm * wsR[v * NT + sbase + tb0 + m];
                        }
                    nl[v] = sl;
                    nr[v] = sr;
                }
            } else {
                double al0[NV], ar0[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    al0[v] = 0.0;
                    ar0[v] = 0.0;
                    if (need)
                        for (int m0 = 0; m0 < n; ++m0) {
                            double Rm = T.R[lo0 * n + m0];
                            int q = v * NT + sbase + (tb0 + m0) + K * t1;
                            al0[v] += Rm * wsL[q];
                            ar0[v] += Rm * wsR[q];
                        }
                }
                __syncthreads();
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    wsL[v * NT + c] = al0[v];
                    wsR[v * NT + c] = ar0[v];
                }
                __syncthreads();
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double sl = 0.0, sr = 0.0;
                    if (need)
                        for (int m1 = 0; m1 < n; ++m1) {
                            double Rm1 = T.R[lo1 * n + m1];
                            int q = v * NT + sbase + t0 + K * (tb1 + m1);
                            sl += Rm1 * wsL[q];
                            sr += Rm1 * wsR[q];
                        }
                    nl[v] = sl;
                    nr[v] = sr;
                }
            }
            __syncthreads();
        } else
        for (int v = 0; v < NV; ++v) {
            wsL[c] = uL[v];
            wsR[c] = uR[v];
            __syncthreads();
            double sl = 0.0, sr = 0.0;
            if (DIM == 2) {
                if (need)
                    for (int m = 0; m < n; ++m) {
                        double Rm = T.R[lo0 * n + m];
                        sl += Rm * wsL[sbase + tb0 + m];
                        sr += Rm * wsR[sbase + tb0 + m];
                    }
            } else {
                // separable: along t0 for the lane's own row, through LDS, then along t1
                // (the row sums the lane (t0, tb1 + m1) leaves are exactly the inner sums
                // of R x R; need is uniform over a level-n segment)
                double al0 = 0.0, ar0 = 0.0;
                if (need)
                    for (int m0 = 0; m0 < n; ++m0) {
                        double Rm = T.R[lo0 * n + m0];
                        int q = sbase + (tb0 + m0) + K * t1;
                        al0 += Rm * wsL[q];
                        ar0 += Rm * wsR[q];
                    }
                __syncthreads();
                wsL[c] = al0;
                wsR[c] = ar0;
                __syncthreads();
                if (need)
                    for (int m1 = 0; m1 < n; ++m1) {
                        double Rm1 = T.R[lo1 * n + m1];
                        int q = sbase + t0 + K * (tb1 + m1);
                        sl += Rm1 * wsL[q];
                        sr += Rm1 * wsR[q];
                    }
            }
            nl[v] = sl;
            nr[v] = sr;
            __syncthreads();
        }
        int okf = need ? ((flux_admissible<DIM>(nl, gam, srho, sE) && flux_admissible<DIM>(nr, gam, srho, sE)) ? 1 : 0) : 1;
        // segment-wide admissibility (transverse bits of the level-n block of this face)
        for (int q = 0; q < DIM - 1; ++q)
            for (int bb = 0; bb < ln; ++bb) {
                int bit = q * G::LOGK + bb;
                int mask = 1 << bit;
                if (bit < 6) okf = lane_step(okf, mask, OpAnd());
                else {
                    ((int *)wsL)[c] = okf;
                    __syncthreads();
                    okf &= ((int *)wsL)[c ^ mask];
                    __syncthreads();
                }
            }
        if (P.fbc && need && !okf) atomicAdd(P.fbc, 1);
        double fnod[NV];
        if (need && okf) hlle<DIM>(nl, nr, fa, gam, fnod);
        else for (int v = 0; v < NV; ++v) fnod[v] = 0.0;
        if constexpr (WIDE) {
#pragma unroll
            for (int v = 0; v < NV; ++v) wsL[v * NT + c] = fnod[v];
            __syncthreads();
            if (DIM == 2) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double sacc = 0.0;
                    if (need && okf)
                        for (int m = 0; m < n; ++m) sacc += T.P[lo0 * n + m] * wsL[v * NT + sbase + tb0 + m];
                    if (need && okf) F[v] += tb * sacc;
                }
            } else {
                double a0s[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    a0s[v] = 0.0;
                    if (need && okf)
                        for (int m0 = 0; m0 < n; ++m0)
                            a0s[v] += T.P[lo0 * n + m0] * wsL[v * NT + sbase + (tb0 + m0) + K * t1];
                }
                __syncthreads();
#pragma unroll
                for (int v = 0; v < NV; ++v) wsL[v * NT + c] = a0s[v];
                __syncthreads();
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double sacc = 0.0;
                    if (need && okf)
                        for (int m1 = 0; m1 < n; ++m1)
                            sacc += T.P[lo1 * n + m1] * wsL[v * NT + sbase + t0 + K * (tb1 + m1)];
                    if (need && okf) F[v] += tb * sacc;
                }
            }
            __syncthreads();
        } else
        for (int v = 0; v < NV; ++v) {
            wsL[c] = fnod[v];
            __syncthreads();
            double sacc = 0.0;
            if (DIM == 2) {
                if (need && okf)
                    for (int m = 0; m < n; ++m) sacc += T.P[lo0 * n + m] * wsL[sbase + tb0 + m];
            } else {
                // separable, as for R above (okf is uniform over a level-n segment too)
                double a0s = 0.0;
                if (need && okf)
                    for (int m0 = 0; m0 < n; ++m0)
                        a0s += T.P[lo0 * n + m0] * wsL[sbase + (tb0 + m0) + K * t1];
                __syncthreads();
                wsL[c] = a0s;
                __syncthreads();
                if (need && okf)
                    for (int m1 = 0; m1 < n; ++m1)
                        sacc += T.P[lo1 * n + m1] * wsL[sbase + t0 + K * (tb1 + m1)];
            }
            if (need && okf) F[v] += tb * sacc;
            __syncthreads();
        }
        if (need && okf) thFV -= tb;
    }
    if (has) {
        if (thFV != 0.0) {
            double aL[NV], aR[NV], fs[NV];
            for (int v = 0; v < NV; ++v) { aL[v] = uL[v]; aR[v] = uR[v]; }
            if (!flux_admissible<DIM>(aL, gam, srho, sE)) {
                if (P.fbc) atomicAdd(P.fbc, 1);
                if (mLe < 0 && uown) for (int v = 0; v < NV; ++v) aL[v] = uown[v * KD + mLc];
                else {
                    int n3[3];
                    elem3(P, mLe < 0 ? ee : mLe, n3);
                    long long gn = gindex<DIM, K>(P, n3, mLc);
                    for (int v = 0; v < NV; ++v) aL[v] = P.u[v * P.dof + gn];
                }
            }
            if (!flux_admissible<DIM>(aR, gam, srho, sE)) {
                if (P.fbc) atomicAdd(P.fbc, 1);
                if (mRe < 0 && uown) for (int v = 0; v < NV; ++v) aR[v] = uown[v * KD + mRc];
                else {
                    int n3[3];
                    elem3(P, mRe < 0 ? ee : mRe, n3);
                    long long gn = gindex<DIM, K>(P, n3, mRc);
                    for (int v = 0; v < NV; ++v) aR[v] = P.u[v * P.dof + gn];
                }
            }
            hlle<DIM>(aL, aR, fa, gam, fs);
            for (int v = 0; v < NV; ++v) F[v] += thFV * fs[v];
        }
    }
}

// one tile (EPB elements) of the residual kernel; every thread of the workgroup calls it.
// The common fluxes on the element faces come precomputed in P.ef (eface_kernel).
template <int DIM, int K, int TOP, int EPB>
__device__ __forceinline__ void residual_body(const KArgs &P, int tile, ResidualSmem<DIM, K, TOP, EPB> &S)
{
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    typedef ResidualSmem<DIM, K, TOP, EPB> SM;
    constexpr int NV = G::NV, KD = G::KD, KF = G::KF;
    const int tid = threadIdx.x;
    const int le = tid / KD, c = tid % KD;
    const int e = tile * EPB + le;
    const bool act = e < P.nel;
    const int ee = act ? e : P.nel - 1;
    int e3[3];
    elem3(P, ee, e3);
    const long long g = gindex<DIM, K>(P, e3, c);
    const Gas gam = {P.gamma, P.gm1};

    preload_element<DIM, K, LV, false, SM>(P, S, le, c, ee, g);
    int sidx[MAXLEV];
    subidx_all<DIM, K, LV>(c, sidx);
    double th[MAXLEV + 1];
    theta_from_alpha<LV>(P.alpha + (long long)ee * LV::A, sidx, th);
    // active levels of the element (any cell with a nonzero weight)
    int actv[MAXLEV + 1];
    if constexpr (KD == 64) {
        // one element per wavefront: one ballot per level, no LDS round trip
#pragma unroll
        for (int l = 0; l <= MAXLEV; ++l) actv[l] = (l <= LV::NLEV && __ballot(th[l] != 0.0) != 0) ? 1 : 0;
    } else {
        int flags = 0;
        for (int l = 0; l <= LV::NLEV; ++l) flags |= (th[l] != 0.0) ? (1 << l) : 0;
        flags = subreduce<DIM, K>(flags, G::LOGK, (int *)&S.tmp[0][0][0], OpOr());
        if (c == 0)
            for (int l = 0; l <= MAXLEV; ++l) S.act[le][l] = (flags >> l) & 1;
    }
    const double own_sr = P.scale[2 * (long long)ee], own_se = P.scale[2 * (long long)ee + 1];
    __syncthreads();
    if constexpr (KD != 64)
        for (int l = 0; l <= MAXLEV; ++l) actv[l] = S.act[le][l];
    // lane exchange buffers of the face fluxes (the temporary is free then)
    double *const wsx = &S.tmp[0][0][0];
    double *const wsL = &S.tmp[le][0][0], *const wsR = &S.tmp[le][1][0];
    // staging of the nodal fluxes: its own array in 3-D (the temporary holds the
    // transverse passes), the temporary in 2-D
    double *const fst = SM::AXO ? &S.nod[SM::AXO ? le : 0][0][0] : &S.tmp[le][0][0];

    double out[NV];
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
    constexpr int NPASS = SM::AXO ? DIM : 1;
    for (int pass = 0; pass < NPASS; ++pass) {
        // each pass adds its axes' FV part, then its levels' parts from the top (blend of
        // eq. blending-weights, summed axis pass by axis pass in 3-D)
        double rfv[NV];
        for (int v = 0; v < NV; ++v) rfv[v] = 0.0;
        const int a0 = SM::AXO ? pass : 0, a1 = SM::AXO ? pass + 1 : DIM;
        // ---------------- common fluxes on the needed faces of axes [a0, a1) ----------------
        int step = K;
#pragma unroll
        for (int li = 0; li < LV::NLEV; ++li)
            if (actv[1 + li]) step = min(step, LV::n(li));
        if (actv[0]) step = 1;
        // the element-face fluxes come precomputed (once per face), only interior faces
        // are left to this kernel: copy the element faces' rows of the flux buffer first
        {
            // an element of one wavefront with at least twice as many lanes as rows: the
            // variables of a row are split over two lanes
            constexpr int NTR = (SM::AXO ? 1 : DIM) * 2 * KF;
            constexpr int VS = (KD == 64 && KD >= 2 * NTR) ? 2 : 1, VPL = (NV + VS - 1) / VS;
            for (int w = c; w < (a1 - a0) * 2 * KF * VS; w += KD) {
                const int nrow = (a1 - a0) * 2 * KF;
                const int q = w % nrow, v0 = (w / nrow) * VPL;
                const int fa = a0 + q / (2 * KF), sd = (q / KF) & 1, tt = q % KF;
                const int nb = sd ? neighbour<DIM>(P, e3, fa, 1) : -1;
                const int src = nb >= 0 ? nb : ee, ssd = nb >= 0 ? 0 : sd;
                double fv[VPL];
                for (int j = 0; j < VPL; ++j)
                    if (v0 + j < NV) fv[j] = P.ef[fb_index<DIM, K>(src, fa, ssd, v0 + j, tt)];
                for (int j = 0; j < VPL; ++j)
                    if (v0 + j < NV) S.F[le][SM::AXO ? 0 : fa][v0 + j][(sd ? K : 0) * KF + tt] = fv[j];
            }
        }
        const int nfaces = face_count<K>(a1 - a0, step, true);
        int nfmax = nfaces;
        if (EPB > 1) {
            wsx[tid] = (double)nfaces;
            __syncthreads();
            for (int q = 0; q < EPB; ++q) nfmax = max(nfmax, (int)wsx[q * KD]);
            __syncthreads();
        }
        const int slot = c / KF, t = c % KF;
        for (int r0 = 0; r0 < nfmax; r0 += K) {
            const int fidx = r0 + slot;
            // an idle lane takes face 1 of the first axis, so that every cell it reads lies
            // in the element
            int fa = a0, k = 1;
            const bool has = fidx < nfaces;
            if (has) face_at<K>(a0, a1 - a0, step, fidx, &fa, &k, true);
            double uL[NV], uR[NV], thL[MAXLEV + 1], thR[MAXLEV + 1];
            // interior face: blended interface states of the two adjacent cells; a cell
            // whose mean replaces a non-admissible FV input is the cell itself
            const int cl = G::from_trans(t, fa, k - 1), cr = G::from_trans(t, fa, k);
            theta_cell_of<DIM, K, LV>(S.al[le], cl, thL);
            theta_cell_of<DIM, K, LV>(S.al[le], cr, thR);
            for (int v = 0; v < NV; ++v) {
                uL[v] = thL[0] * S.u[le][v][cl];
                uR[v] = thR[0] * S.u[le][v][cr];
            }
#pragma unroll
            for (int li = 0; li < LV::NLEV; ++li) {
                CTab &T = P.tabs[li];
                int n = LV::n(li);
                if (thL[1 + li] != 0.0) {
                    int s = G::subelem(cl, n);
                    double b = S.be[le][LV::off(li) + s];
                    for (int v = 0; v < NV; ++v) {
                        double tr = bapply<DIM, K>(S.u[le][v], cl, fa, n, T.Ep);
                        uL[v] += thL[1 + li] * ((1.0 - b) * S.mean[le][v][LV::off(li) + s] + b * tr);
                    }
                }
                if (thR[1 + li] != 0.0) {
                    int s = G::subelem(cr, n);
                    double b = S.be[le][LV::off(li) + s];
                    for (int v = 0; v < NV; ++v) {
                        double tr = bapply<DIM, K>(S.u[le][v], cr, fa, n, T.Em);
                        uR[v] += thR[1 + li] * ((1.0 - b) * S.mean[le][v][LV::off(li) + s] + b * tr);
                    }
                }
            }
            double F[NV];
            common_flux<DIM, K, LV, EPB * KD>(P, wsL, wsR, c, slot * KF, t, has, fa, k, uL, uR,
                                             thL, thR, own_sr, own_se, -1, cl, -1, cr, &S.u[le][0][0], ee, F);
            if (has) {
                const int axs = SM::AXO ? 0 : fa;
                for (int v = 0; v < NV; ++v) S.F[le][axs][v][k * KF + t] = F[v];
            }
        }
        __syncthreads();

        // ---------------- FV part: -(K/dx_a) (F_{i+1/2} - F_{i-1/2}) ----------------
        if (th[0] != 0.0) {
            for (int a = a0; a < a1; ++a) {
                const int axs = SM::AXO ? 0 : a;
                const int pos = G::coord(c, a), tr = G::trans(c, a);
                double sc = K / arg_dx(P, a);
                for (int v = 0; v < NV; ++v)
                    rfv[v] -= sc * (S.F[le][axs][v][(pos + 1) * KF + tr] - S.F[le][axs][v][pos * KF + tr]);
            }
            for (int v = 0; v < NV; ++v) out[v] += th[0] * rfv[v];
        }

        // ---------------- DG levels: (K/(n dx_a)) (f~_a x_a Dhat x_perp P - F*_a x_a Bhat) ----------------
#pragma unroll
        for (int li = 0; li < LV::NLEV; ++li) {
            if (!block_or<EPB * KD>(actv[1 + li])) continue;
            CTab &T = P.tabs[li];
            const int n = LV::n(li);
            const bool on = th[1 + li] != 0.0;
            // squeezed reconstruction at this cell's node
            double nodal[NV];
            if (DIM == 2) {
                for (int v = 0; v < NV; ++v) S.tmp[le][v][c] = bapply<DIM, K>(S.u[le][v], c, 0, n, T.R);
                __syncthreads();
                for (int v = 0; v < NV; ++v) nodal[v] = bapply<DIM, K>(S.tmp[le][v], c, 1, n, T.R);
            } else if (pass == 0) {
                for (int v = 0; v < NV; ++v) fst[v * KD + c] = bapply<DIM, K>(S.u[le][v], c, 0, n, T.R);
                __syncthreads();
                for (int v = 0; v < NV; ++v) S.tmp[le][v][c] = bapply<DIM, K>(fst + v * KD, c, 1, n, T.R);
                __syncthreads();
                for (int v = 0; v < NV; ++v) nodal[v] = bapply<DIM, K>(S.tmp[le][v], c, 2, n, T.R);
            } else {
                for (int v = 0; v < NV; ++v) nodal[v] = S.nodc[SM::AXO ? le : 0][SM::AXO ? li : 0][SM::AXO ? v : 0][SM::AXO ? c : 0];
            }
            if (!SM::AXO || pass == 0) {
                int s = sidx[li];
                double b = S.be[le][LV::off(li) + s];
                for (int v = 0; v < NV; ++v) nodal[v] = (1.0 - b) * S.mean[le][v][LV::off(li) + s] + b * nodal[v];
                if (SM::AXO)
                    for (int v = 0; v < NV; ++v)
                        S.nodc[SM::AXO ? le : 0][SM::AXO ? li : 0][SM::AXO ? v : 0][SM::AXO ? c : 0] = nodal[v];
            }
            double lrl[NV];
            for (int v = 0; v < NV; ++v) lrl[v] = 0.0;
            const double nir = 1.0 / nodal[0];
            double nm2 = 0.0;
            for (int d = 0; d < DIM; ++d) nm2 += nodal[1 + d] * nodal[1 + d];
            const double npr = (nodal[0] > 0.0) ? gam.gm1 * (nodal[DIM + 1] - 0.5 * nm2 * nir) : -INFINITY;
            for (int a = a0; a < a1; ++a) {
                const int axs = SM::AXO ? 0 : a;
                double f[NV];
                euler_flux_ir<DIM>(nodal, nir, npr, a, f);
                __syncthreads();
                for (int v = 0; v < NV; ++v) fst[v * KD + c] = f[v];
                __syncthreads();
                double vol[NV];
                for (int v = 0; v < NV; ++v) vol[v] = bapply<DIM, K>(fst + v * KD, c, a, n, T.Dhat);
                for (int bax = 0; bax < DIM; ++bax) {
                    if (bax == a) continue;
                    __syncthreads();
                    for (int v = 0; v < NV; ++v) S.tmp[le][v][c] = vol[v];
                    __syncthreads();
                    for (int v = 0; v < NV; ++v) vol[v] = bapply<DIM, K>(S.tmp[le][v], c, bax, n, T.P);
                }
                if (on) {
                    const int pos = G::coord(c, a), tr = G::trans(c, a);
                    const int lo = pos & (n - 1);
                    const int kl = pos - lo, kr = kl + n;
                    const double sc = K / (n * arg_dx(P, a));
                    for (int v = 0; v < NV; ++v) {
                        double surf = T.Bhl[lo] * S.F[le][axs][v][kl * KF + tr] + T.Bhr[lo] * S.F[le][axs][v][kr * KF + tr];
                        lrl[v] += sc * (vol[v] - surf);
                    }
                }
            }
            if (on)
                for (int v = 0; v < NV; ++v) out[v] += th[1 + li] * lrl[v];
            __syncthreads();
        }
    }

    if (!act) return;
    if (P.stage == 0) {
        for (int v = 0; v < NV; ++v) P.out[v * P.dof + g] = out[v];
    } else if (P.stage == 5) {
        // one stage of a Shu-Osher form with up to two earlier states (SSP-RK(5,4));
        // every load before the first store
        const double dt = *P.dt;
        double ub[NV], a0[NV], a1[NV], b0[NV];
        for (int v = 0; v < NV; ++v) {
            const long long i = v * P.dof + g;
            ub[v] = S.u[le][v][c];
            a0[v] = P.u0 ? P.u0[i] : 0.0;
            a1[v] = P.x1 ? P.x1[i] : 0.0;
            b0[v] = P.yout ? P.y0[i] : 0.0;
        }
        for (int v = 0; v < NV; ++v) {
            const long long i = v * P.dof + g;
            const double dl = dt * out[v];
            if (P.yout) P.yout[i] = P.rk[4] * b0[v] + P.rk[5] * ub[v] + P.rk[6] * dl;
            P.out[i] = P.rk[0] * a0[v] + P.rk[1] * ub[v] + P.rk[2] * dl + P.rk[3] * a1[v];
        }
    } else {
        double dt = *P.dt;
        double ub[NV], u0[NV];
        for (int v = 0; v < NV; ++v) ub[v] = S.u[le][v][c];
        // all loads of u^n before the first store (the output may alias nothing, but
        // the compiler cannot know it, and would otherwise wait once per variable)
        if (P.stage != 1)
            for (int v = 0; v < NV; ++v) u0[v] = P.u0[v * P.dof + g];
        for (int v = 0; v < NV; ++v) {
            long long i = v * P.dof + g;
            double r;
            if (P.stage == 1) r = ub[v] + dt * out[v];
            else if (P.stage == 2) r = 0.75 * u0[v] + 0.25 * (ub[v] + dt * out[v]);
            else r = (1.0 / 3.0) * u0[v] + (2.0 / 3.0) * (ub[v] + dt * out[v]);
            P.out[i] = r;
        }
    }
}

// Common fluxes on the element faces, once per face (the residual kernel would otherwise
// evaluate each on both sides): a workgroup of 64 lanes takes 64 / K^{d-1} (element,
// axis) tasks, each the element's low face along the axis (the element is the right
// side, its low neighbour the left), plus the high face of an element at an outflow
// boundary, which no neighbour takes.  F* goes to P.ef in the face-buffer layout.
template <int DIM, int K, int TOP>
__device__ __forceinline__ void eface_body(const KArgs &P, int tile, double *wsL, double *wsR)
{
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    constexpr int NV = G::NV, KF = G::KF, NS = 64 / KF;
    const int c = threadIdx.x, slot = c / KF, t = c % KF;
    const long long task = (long long)tile * NS + slot;
    const bool valid = task < (long long)P.nel * DIM;
    const int e = valid ? (int)(task / DIM) : 0, a = valid ? (int)(task % DIM) : 0;
    int e3[3];
    elem3(P, e, e3);
    const double own_sr = P.scale[2 * (long long)e], own_se = P.scale[2 * (long long)e + 1];
    for (int sd = 0; sd < 2; ++sd) {
        const int nb = neighbour<DIM>(P, e3, a, sd);
        const bool has = valid && (sd == 0 || nb < 0);
        if (!block_or<64>(has)) continue;
        double uL[NV], uR[NV], thL[MAXLEV + 1], thR[MAXLEV + 1], srho = own_sr, sE = own_se;
        int mLe = -1, mLc = 0, mRe = -1, mRc = 0;
        element_face_sides<DIM, K, LV>(P, e, a, t, sd == 1, nb, P.alpha + (long long)e * LV::A,
                                       P.alpha + (long long)(nb >= 0 ? nb : e) * LV::A, own_sr, own_se, uL, uR,
                                       thL, thR, mLe, mLc, mRe, mRc, srho, sE);
        double F[NV];
        common_flux<DIM, K, LV, 64, true>(P, wsL, wsR, c, slot * KF, t, has, a, sd ? K : 0, uL, uR, thL, thR, srho, sE, mLe,
                                    mLc, mRe, mRc, nullptr, e, F);
        if (has)
            for (int v = 0; v < NV; ++v) P.ef[fb_index<DIM, K>(e, a, sd, v, t)] = F[v];
    }
}

template <int DIM, int K, int TOP>
__global__ void __launch_bounds__(64) eface_kernel(KArgs P)
{
    __shared__ double wsL[(DIM + 2) * 64], wsR[(DIM + 2) * 64];
    eface_body<DIM, K, TOP>(P, xcd_tile(blockIdx.x, gridDim.x), wsL, wsR);
    if (P.fin_lam && blockIdx.x == 0) {
        // the step size of the stage's residual (launched after this kernel): one launch
        // less per step than a kernel of its own; maxima are exact in any order
        const int l = threadIdx.x;
        double m = 0.0;
#pragma unroll
        for (int k = 0; k < LAM_SLOTS / 64; ++k) {
            m = fmax(m, P.fin_lam[l + 64 * k]);
            P.fin_lam[l + 64 * k] = 0.0;
        }
        m = lane_max_bits<0, 6>(m);
        if (l == 0) {
            const double d = P.fin_num / m;
            P.fin_dt[0] = d;
            if (P.fin_dt_log) P.fin_dt_log[P.fin_ctr[0]] = d;
        }
    }
}

template <int DIM, int K, int TOP, int EPB>
__global__ void __launch_bounds__((EPB * Geo<DIM, K>::KD))
__attribute__((amdgpu_waves_per_eu(DIM == 3 ? 2 : 3, 8))) residual_kernel(KArgs P)
{
    __shared__ ResidualSmem<DIM, K, TOP, EPB> S;
    residual_body<DIM, K, TOP, EPB>(P, xcd_tile(blockIdx.x, gridDim.x), S);
}

// ---------------------------------------------------------------------------
// frozen blending factors: preparation kernel
// ---------------------------------------------------------------------------
//
// With alpha and beta given (the frozen map of the adjoint), the residual needs
// the sub-element means of every level, the element data scales and the face
// buffer.  For the adjoint the same launch also publishes each element's own
// share of the flux adjoints on its element faces (the part its neighbour cannot
// form from its own data).

// Flux-adjoint contributions of one element's subcells to face k (0..K) along axis a
// at face-plane index t, for the adjoint state lam: the FV part gives
// -(K/dx_a) theta_FV lam on the cell left of the face and +(K/dx_a) theta_FV lam on
// the cell right of it; the level-n surface term gives -(K/(n dx_a)) theta_n Bhat lam
// over the sub-element rows ending (Bhr) or starting (Bhl) at the face.  Cells left
// (right) of the face exist for k > 0 (k < K).
template <int DIM, int K, class LV>
__device__ void own_face_adjoint(const KArgs &P, const double *al, const double (*lam)[Geo<DIM, K>::KD], int a, int k,
                                 int t, double *gf)
{
    typedef Geo<DIM, K> G;
    constexpr int NV = G::NV;
    for (int v = 0; v < NV; ++v) gf[v] = 0.0;
    const double sc = K / arg_dx(P, a);
    const int st = G::stride(a);
    double th[MAXLEV + 1];
    if (k > 0) {
        const int cl = G::from_trans(t, a, k - 1);
        theta_cell_of<DIM, K, LV>(al, cl, th);
        if (th[0] != 0.0)
            for (int v = 0; v < NV; ++v) gf[v] -= sc * th[0] * lam[v][cl];
#pragma unroll
        for (int li = 0; li < LV::NLEV; ++li) {
            const int n = LV::n(li);
            if (k % n != 0 || th[1 + li] == 0.0) continue;
            CTab &T = P.tabs[li];
            const double w = (K / (n * arg_dx(P, a))) * th[1 + li];
            for (int lo = 0; lo < n; ++lo) {
                const int cell = cl - (n - 1 - lo) * st;
                for (int v = 0; v < NV; ++v) gf[v] -= w * T.Bhr[lo] * lam[v][cell];
            }
        }
    }
    if (k < K) {
        const int cr = G::from_trans(t, a, k);
        theta_cell_of<DIM, K, LV>(al, cr, th);
        if (th[0] != 0.0)
            for (int v = 0; v < NV; ++v) gf[v] += sc * th[0] * lam[v][cr];
#pragma unroll
        for (int li = 0; li < LV::NLEV; ++li) {
            const int n = LV::n(li);
            if (k % n != 0 || th[1 + li] == 0.0) continue;
            CTab &T = P.tabs[li];
            const double w = (K / (n * arg_dx(P, a))) * th[1 + li];
            for (int lo = 0; lo < n; ++lo) {
                const int cell = cr + lo * st;
                for (int v = 0; v < NV; ++v) gf[v] -= w * T.Bhl[lo] * lam[v][cell];
            }
        }
    }
}

// out(t) = sum over the level-n face segment holding face-plane index t of
// M[lo][m] src(m) (2-D), or M[lo0][m0] M[lo1][m1] src(m0, m1) (3-D); src is a
// face-plane array of K^(DIM-1) values
template <int DIM, int K>
__device__ __forceinline__ double seg_apply(const double *src, int t, int n, CDbl *M)
{
    if (DIM == 2) {
        const int lo0 = t & (n - 1), tb0 = t - lo0;
        double s = 0.0;
        for (int m = 0; m < n; ++m) s += M[lo0 * n + m] * src[tb0 + m];
        return s;
    }
    const int t0 = t & (K - 1), t1 = t >> Geo<DIM, K>::LOGK;
    const int lo0 = t0 & (n - 1), tb0 = t0 - lo0, lo1 = t1 & (n - 1), tb1 = t1 - lo1;
    double s = 0.0;
    for (int m1 = 0; m1 < n; ++m1) {
        double a0 = 0.0;
        for (int m0 = 0; m0 < n; ++m0) a0 += M[lo0 * n + m0] * src[(tb0 + m0) + K * (tb1 + m1)];
        s += M[lo1 * n + m1] * a0;
    }
    return s;
}

template <int DIM, int K, int TOP, int EPB>
struct PrepSmem {
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    double u[EPB][G::NV][G::KD];
    double lam[EPB][G::NV][G::KD];
    double x[EPB * G::KD];
    double al[EPB][LV::A];
    double be[EPB][LV::A];
    double mean[EPB][G::NV][LV::A];
};

template <int DIM, int K, int TOP, int EPB>
__global__ void __launch_bounds__((EPB * Geo<DIM, K>::KD)) frozen_prep_kernel(KArgs P)
{
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    constexpr int NV = G::NV, KD = G::KD;
    __shared__ PrepSmem<DIM, K, TOP, EPB> S;
    const int tid = threadIdx.x;
    const int le = tid / KD, c = tid % KD;
    const int e = blockIdx.x * EPB + le;
    const bool act = e < P.nel;
    const int ee = act ? e : P.nel - 1;
    int e3[3];
    elem3(P, ee, e3);
    const long long g = gindex<DIM, K>(P, e3, c);
    const Gas gam = {P.gamma, P.gm1};
    const bool adj = P.lam != nullptr;

    double ub[NV];
    bool fin = true;
    for (int v = 0; v < NV; ++v) {
        ub[v] = P.u[v * P.dof + g];
        S.u[le][v][c] = ub[v];
        fin = fin && isfinite(ub[v]);
        if (adj) S.lam[le][v][c] = P.lam[v * P.dof + g];
    }
    if (act && !(fin && permissible<DIM>(ub, gam))) atomicMin(P.err, P.err_base + e);
    {
        double sc[2] = {ub[0], fabs(ub[NV - 1])};
        subreduce_n<DIM, K, 2>(sc, G::LOGK, S.x, OpMax());
        if (act && c == 0) {
            P.scale[2 * (long long)e] = sc[0];
            P.scale[2 * (long long)e + 1] = sc[1];
        }
    }
    for (int q = c; q < LV::A; q += KD) {
        S.al[le][q] = P.alpha[(long long)ee * LV::A + q];
        S.be[le][q] = P.beta[(long long)ee * LV::A + q];
    }
    // sub-element means of every level (the same reduction as the analyse kernel)
#pragma unroll
    for (int li = 0; li < LV::NLEV; ++li) {
        const int n = LV::n(li), ln = ilog2i(n);
        double nd = (DIM == 2) ? n * n : n * n * n;
        double mn[NV];
        for (int v = 0; v < NV; ++v) mn[v] = ub[v];
        reduce_means<DIM, K, NV>(mn, ln, S.x);
        for (int v = 0; v < NV; ++v) mn[v] /= nd;
        const bool leader = ((G::coord(c, 0) | G::coord(c, 1) | (DIM == 3 ? G::coord(c, 2) : 0)) & (n - 1)) == 0;
        if (leader)
            for (int v = 0; v < NV; ++v) S.mean[le][v][LV::off(li) + G::subelem(c, n)] = mn[v];
    }
    __syncthreads();
    if (act)
        for (int q = c; q < LV::A; q += KD)
            for (int v = 0; v < NV; ++v) P.mean[((long long)e * NV + v) * LV::A + q] = S.mean[le][v][q];
    int sidx[MAXLEV];
    subidx_all<DIM, K, LV>(c, sidx);
    double th[MAXLEV + 1];
    theta_from_alpha<LV>(S.al[le], sidx, th);
    // blended interface states on the element faces (as in the analyse kernel)
    for (int a = 0; a < DIM; ++a) {
        int pos = G::coord(c, a);
        for (int sd = 0; sd < 2; ++sd) {
            if (pos != (sd ? K - 1 : 0)) continue;
            double st[NV];
            for (int v = 0; v < NV; ++v) st[v] = th[0] * ub[v];
#pragma unroll
            for (int li = 0; li < LV::NLEV; ++li) {
                if (th[1 + li] == 0.0) continue;
                CTab &T = P.tabs[li];
                int n = LV::n(li);
                CDbl *E = sd ? T.Ep : T.Em;
                const int q = LV::off(li) + sidx[li];
                double b = S.be[le][q];
                for (int v = 0; v < NV; ++v) {
                    double tr = bapply<DIM, K>(S.u[le][v], c, a, n, E);
                    st[v] += th[1 + li] * ((1.0 - b) * S.mean[le][v][q] + b * tr);
                }
            }
            if (act)
                for (int v = 0; v < NV; ++v) P.fbuf[fb_index<DIM, K>(e, a, sd, v, G::trans(c, a))] = st[v];
            if (adj) {
                double gf[NV];
                own_face_adjoint<DIM, K, LV>(P, S.al[le], S.lam[le], a, sd ? K : 0, G::trans(c, a), gf);
                if (act)
                    for (int v = 0; v < NV; ++v) P.gfb[fb_index<DIM, K>(e, a, sd, v, G::trans(c, a))] = gf[v];
            }
        }
    }
}

// Each element's own share of the flux adjoints on its element faces, alone: for the
// transposed RK stages, whose face states, means and scales were recorded on the
// tape by the analysis that produced the stage.
template <int DIM, int K, int TOP, int EPB>
__global__ void __launch_bounds__((EPB * Geo<DIM, K>::KD)) face_adjoint_kernel(KArgs P)
{
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    constexpr int NV = G::NV, KD = G::KD;
    __shared__ double s_lam[EPB][NV][KD];
    __shared__ double s_al[EPB][LV::A];
    const int tid = threadIdx.x;
    const int le = tid / KD, c = tid % KD;
    const int e = blockIdx.x * EPB + le;
    const bool act = e < P.nel;
    const int ee = act ? e : P.nel - 1;
    int e3[3];
    elem3(P, ee, e3);
    const long long g = gindex<DIM, K>(P, e3, c);
    for (int v = 0; v < NV; ++v) s_lam[le][v][c] = P.lam[v * P.dof + g];
    for (int q = c; q < LV::A; q += KD) s_al[le][q] = P.alpha[(long long)ee * LV::A + q];
    __syncthreads();
    // one task per (element, face, face cell) over the workgroup's lanes
    constexpr int NF = 2 * DIM, KF = G::KF;
    for (int tsk = tid; tsk < EPB * NF * KF; tsk += EPB * KD) {
        const int tle = tsk / (NF * KF), rem = tsk - tle * (NF * KF), f = rem / KF, t = rem - f * KF;
        const int te = blockIdx.x * EPB + tle;
        if (te >= P.nel) continue;
        const int a = f >> 1, sd = f & 1;
        double gf[NV];
        own_face_adjoint<DIM, K, LV>(P, s_al[tle], s_lam[tle], a, sd ? K : 0, t, gf);
        for (int v = 0; v < NV; ++v) P.gfb[fb_index<DIM, K>(te, a, sd, v, t)] = gf[v];
    }
}

// Reverse of common_flux on one face per group of KF lanes: from the flux adjoint on
// the face (the group's KF face values of variable v at gseg[v * gstride + 0 .. KF - 1])
// to the adjoints of the blended interface states (guL, guR) and of the subcell states
// whose means replaced a non-admissible FV input (gdL, gdR).  The other arguments are
// those of common_flux; every lane of the workgroup (NT threads) calls it with the same
// face count.
template <int DIM, int K, class LV, int NT>
__device__ __forceinline__ void common_flux_adj(const KArgs &P, double *wsL, double *wsR, int c, int sbase, int t,
                                                bool has, int fa, int k, const double *uL, const double *uR,
                                                const double *thL, const double *thR, double srho, double sE, int mLe,
                                                int mLc, int mRe, int mRc, const double *uown, int ee,
                                                const double *gseg, int gstride, double *guL, double *guR, double *gdL,
                                                double *gdR)
{
    typedef Geo<DIM, K> G;
    constexpr int NV = G::NV, KD = G::KD;
    const Gas gam = {P.gamma, P.gm1};
    double gFv[NV];
    for (int v = 0; v < NV; ++v) gFv[v] = gseg[v * gstride + t];
    for (int v = 0; v < NV; ++v) { guL[v] = 0.0; guR[v] = 0.0; gdL[v] = 0.0; gdR[v] = 0.0; }
    double thFV = 1.0;
#pragma unroll
    for (int li = 0; li < LV::NLEV; ++li) {
        if (!block_or<NT>(has && (k % LV::n(li) == 0) && (thL[1 + li] != 0.0 || thR[1 + li] != 0.0)))
            continue;
        CTab &T = P.tabs[li];
        const int n = LV::n(li), ln = ilog2i(n);
        const double tb = 0.5 * (thL[1 + li] + thR[1 + li]);
        const bool need = has && (k % n == 0) && (tb != 0.0);
        // nodal face states R_perp uL, R_perp uR
        double nl[NV], nr[NV];
        for (int v = 0; v < NV; ++v) {
            wsL[c] = uL[v];
            wsR[c] = uR[v];
            __syncthreads();
            nl[v] = need ? seg_apply<DIM, K>(&wsL[sbase], t, n, T.R) : 0.0;
            nr[v] = need ? seg_apply<DIM, K>(&wsR[sbase], t, n, T.R) : 0.0;
            __syncthreads();
        }
        int okf = need ? ((flux_admissible<DIM>(nl, gam, srho, sE) && flux_admissible<DIM>(nr, gam, srho, sE)) ? 1 : 0) : 1;
        for (int q = 0; q < DIM - 1; ++q)
            for (int bb = 0; bb < ln; ++bb) {
                int bit = q * G::LOGK + bb;
                int mask = 1 << bit;
                if (bit < 6) okf = lane_step(okf, mask, OpAnd());
                else {
                    ((int *)wsL)[c] = okf;
                    __syncthreads();
                    okf &= ((int *)wsL)[c ^ mask];
                    __syncthreads();
                }
            }
        const bool use = need && okf;
        // face-node flux adjoints tb * P_perp^T gF, then the HLLE Jacobian^T
        double gnl[NV], gnr[NV];
        for (int v = 0; v < NV; ++v) { gnl[v] = 0.0; gnr[v] = 0.0; }
        if (use) {
            double gh[NV];
            for (int v = 0; v < NV; ++v) gh[v] = tb * seg_apply<DIM, K>(&gseg[v * gstride], t, n, T.PT);
            hlle_adj<DIM>(nl, nr, fa, gam, gh, gnl, gnr);
        }
        // back to face means: R_perp^T
        for (int v = 0; v < NV; ++v) {
            wsL[c] = gnl[v];
            wsR[c] = gnr[v];
            __syncthreads();
            if (use) {
                guL[v] += seg_apply<DIM, K>(&wsL[sbase], t, n, T.RT);
                guR[v] += seg_apply<DIM, K>(&wsR[sbase], t, n, T.RT);
            }
            __syncthreads();
        }
        if (use) thFV -= tb;
    }
    if (has && thFV != 0.0) {
        double aL[NV], aR[NV];
        for (int v = 0; v < NV; ++v) { aL[v] = uL[v]; aR[v] = uR[v]; }
        const bool fbL = !flux_admissible<DIM>(aL, gam, srho, sE);
        const bool fbR = !flux_admissible<DIM>(aR, gam, srho, sE);
        if (fbL) {
            if (mLe < 0 && uown) for (int v = 0; v < NV; ++v) aL[v] = uown[v * KD + mLc];
            else {
                int n3[3];
                elem3(P, mLe < 0 ? ee : mLe, n3);
                long long gn = gindex<DIM, K>(P, n3, mLc);
                for (int v = 0; v < NV; ++v) aL[v] = P.u[v * P.dof + gn];
            }
        }
        if (fbR) {
            if (mRe < 0 && uown) for (int v = 0; v < NV; ++v) aR[v] = uown[v * KD + mRc];
            else {
                int n3[3];
                elem3(P, mRe < 0 ? ee : mRe, n3);
                long long gn = gindex<DIM, K>(P, n3, mRc);
                for (int v = 0; v < NV; ++v) aR[v] = P.u[v * P.dof + gn];
            }
        }
        double gfs[NV], gaL[NV], gaR[NV];
        for (int v = 0; v < NV; ++v) { gfs[v] = thFV * gFv[v]; gaL[v] = 0.0; gaR[v] = 0.0; }
        hlle_adj<DIM>(aL, aR, fa, gam, gfs, gaL, gaR);
        for (int v = 0; v < NV; ++v) {
            if (fbL) gdL[v] += gaL[v]; else guL[v] += gaL[v];
            if (fbR) gdR[v] += gaR[v]; else guR[v] += gaR[v];
        }
    }
}

// ---------------------------------------------------------------------------
// adjoint kernel: lam_out = (dL/du)^T lam of the frozen right-hand side
// ---------------------------------------------------------------------------
//
// Reverse of the residual kernel, one element per EPB slot, every element writing
// only its own cells.  First the DG volume terms of every level (P^T across,
// Dhat^T along each axis, Euler-flux Jacobian^T at the squeezed nodal values),
// taken back through the squeezed reconstruction (R^T on every axis plus the
// sub-element mean).  Then, axis by axis:
//   (1) flux adjoints gF at the interior faces of the axis, from the element's own
//       adjoint state;
//   (2) reverse of the common fluxes on the interior faces the forward evaluated:
//       the FV candidate and the level DG candidates (P_perp^T, HLLE Jacobian^T,
//       R_perp^T), giving adjoints of the blended interface states (GS) and of
//       subcell means that replaced a flux input (GD); those of the element faces
//       come from the element-face adjoint kernel (eface_adjoint_kernel);
//   (3) interface-state adjoints -> state adjoints: theta_FV directly, the level-n
//       traces through E^T along the axis and the squeeze mean.
// Only the state adjoint stays live across the face loop.  The RK variants fuse
// the transposed SSP-RK3 combinations into the store.

template <int DIM, int K, int TOP, int EPB>
struct AdjointSmem {
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    double u[EPB][G::NV][G::KD];
    double lam[EPB][G::NV][G::KD];
    double gF[EPB][G::NV][(K + 1) * G::KF];
    double GS[EPB][2][G::NV][G::KD];
    double GD[EPB][2][G::NV][G::KD];
    double tmp[EPB][G::NV][G::KD];
    double al[EPB][LV::A];
    double be[EPB][LV::A];
    double mean[EPB][G::NV][LV::A];
    double wsL[EPB * G::KD], wsR[EPB * G::KD];
    int act[EPB][MAXLEV + 1];
};

template <int DIM, int K, int TOP, int EPB>
__global__ void __launch_bounds__((EPB * Geo<DIM, K>::KD))
__attribute__((amdgpu_waves_per_eu(2, 8))) adjoint_kernel(KArgs P)
{
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    constexpr int NV = G::NV, KD = G::KD, KF = G::KF;
    __shared__ AdjointSmem<DIM, K, TOP, EPB> S;
    const int tid = threadIdx.x;
    const int le = tid / KD, c = tid % KD;
    const int e = xcd_tile(blockIdx.x, gridDim.x) * EPB + le;
    const bool act = e < P.nel;
    const int ee = act ? e : P.nel - 1;
    int e3[3];
    elem3(P, ee, e3);
    const long long g = gindex<DIM, K>(P, e3, c);
    const Gas gam = {P.gamma, P.gm1};

    preload_element<DIM, K, LV, true, AdjointSmem<DIM, K, TOP, EPB>>(P, S, le, c, ee, g);
    int sidx[MAXLEV];
    subidx_all<DIM, K, LV>(c, sidx);
    double th[MAXLEV + 1];
    theta_from_alpha<LV>(P.alpha + (long long)ee * LV::A, sidx, th);
    int actv[MAXLEV + 1];
    if constexpr (KD == 64) {
        // one element per wavefront: one ballot per level, no LDS round trip
#pragma unroll
        for (int l = 0; l <= MAXLEV; ++l) actv[l] = (l <= LV::NLEV && __ballot(th[l] != 0.0) != 0) ? 1 : 0;
    } else {
        int flags = 0;
        for (int l = 0; l <= LV::NLEV; ++l) flags |= (th[l] != 0.0) ? (1 << l) : 0;
        flags = subreduce<DIM, K>(flags, G::LOGK, (int *)S.wsL, OpOr());
        if (c == 0)
            for (int l = 0; l <= MAXLEV; ++l) S.act[le][l] = (flags >> l) & 1;
    }
    const double own_sr = P.scale[2 * (long long)ee], own_se = P.scale[2 * (long long)ee + 1];
    __syncthreads();
    if constexpr (KD != 64)
        for (int l = 0; l <= MAXLEV; ++l) actv[l] = S.act[le][l];

    double gu[NV];
    for (int v = 0; v < NV; ++v) gu[v] = 0.0;

    // ---------------- DG volume terms of every level, reversed through the squeeze ----------------
    // per level: squeezed nodal values ut; over the axes gut += J_a(ut)^T (sc theta_n lam x_perp P^T
    // x_a Dhat^T); then gu += b (gut x_all R^T) + (1 - b) / n^DIM * (sum of gut over the sub-element)
#pragma unroll
    for (int li = 0; li < LV::NLEV; ++li) {
        if (!block_or<EPB * KD>(actv[1 + li])) continue;
        CTab &T = P.tabs[li];
        const int n = LV::n(li), ln = ilog2i(n);
        const double thn = th[1 + li];
        const double b = S.be[le][LV::off(li) + sidx[li]];
        double ut[NV];
        if (DIM == 2) {
            for (int v = 0; v < NV; ++v) S.tmp[le][v][c] = bapply<DIM, K>(S.u[le][v], c, 0, n, T.R);
            __syncthreads();
            for (int v = 0; v < NV; ++v) ut[v] = bapply<DIM, K>(S.tmp[le][v], c, 1, n, T.R);
        } else {
            for (int v = 0; v < NV; ++v) S.GS[le][0][v][c] = bapply<DIM, K>(S.u[le][v], c, 0, n, T.R);
            __syncthreads();
            for (int v = 0; v < NV; ++v) S.tmp[le][v][c] = bapply<DIM, K>(S.GS[le][0][v], c, 1, n, T.R);
            __syncthreads();
            for (int v = 0; v < NV; ++v) ut[v] = bapply<DIM, K>(S.tmp[le][v], c, 2, n, T.R);
        }
        for (int v = 0; v < NV; ++v) ut[v] = (1.0 - b) * S.mean[le][v][LV::off(li) + sidx[li]] + b * ut[v];
        double gut[NV];
        for (int v = 0; v < NV; ++v) gut[v] = 0.0;
        for (int a = 0; a < DIM; ++a) {
            const double sc = K / (n * arg_dx(P, a));
            double gv[NV];
            for (int v = 0; v < NV; ++v) gv[v] = sc * thn * S.lam[le][v][c];
            for (int bax = 0; bax < DIM; ++bax) {
                if (bax == a) continue;
                __syncthreads();
                for (int v = 0; v < NV; ++v) S.tmp[le][v][c] = gv[v];
                __syncthreads();
                for (int v = 0; v < NV; ++v) gv[v] = bapply<DIM, K>(S.tmp[le][v], c, bax, n, T.PT);
            }
            __syncthreads();
            for (int v = 0; v < NV; ++v) S.tmp[le][v][c] = gv[v];
            __syncthreads();
            double gfl[NV], gj[NV];
            for (int v = 0; v < NV; ++v) gfl[v] = bapply<DIM, K>(S.tmp[le][v], c, a, n, T.DhatT);
            if (thn != 0.0) {
                euler_flux_adj<DIM>(ut, a, gam, gfl, gj);
                for (int v = 0; v < NV; ++v) gut[v] += gj[v];
            }
        }
        double y[NV];
        for (int v = 0; v < NV; ++v) y[v] = gut[v];
        for (int ax = DIM - 1; ax >= 0; --ax) {
            __syncthreads();
            for (int v = 0; v < NV; ++v) S.tmp[le][v][c] = y[v];
            __syncthreads();
            for (int v = 0; v < NV; ++v) y[v] = bapply<DIM, K>(S.tmp[le][v], c, ax, n, T.RT);
        }
        const double nd = (DIM == 2) ? n * n : n * n * n;
        double ms[NV];
        for (int v = 0; v < NV; ++v) ms[v] = gut[v];
        reduce_means<DIM, K, NV>(ms, ln, S.wsL);
        if (thn != 0.0)
            for (int v = 0; v < NV; ++v) gu[v] += b * y[v] + (1.0 - b) * ms[v] / nd;
        __syncthreads();
    }

    for (int a = 0; a < DIM; ++a) {
        // the faces the forward evaluated: every face when the FV level is active, else
        // the multiples of the smallest active DG level (the element faces at least;
        // their reverse comes precomputed from the element-face adjoint kernel)
        int step = K;
#pragma unroll
        for (int li = 0; li < LV::NLEV; ++li)
            if (actv[1 + li]) step = min(step, LV::n(li));
        if (actv[0]) step = 1;
        // ---------------- (1) flux adjoints on the interior faces of axis a ----------------
        // only the faces at multiples of step are read: one lane per (such face, face cell)
        const int nki = K / step - 1;
        for (int j = c; j < nki * KF; j += KD) {
            const int k = (j / KF + 1) * step, t = j % KF, q = k * KF + t;
            double gf[NV];
            own_face_adjoint<DIM, K, LV>(P, S.al[le], S.lam[le], a, k, t, gf);
            for (int v = 0; v < NV; ++v) S.gF[le][v][q] = gf[v];
        }
        // the element faces' interface-state and mean adjoints of the element's own cells
        {
            const int pos = G::coord(c, a), tt = G::trans(c, a);
            double gs0[NV], gs1[NV], gd0[NV], gd1[NV];
            for (int v = 0; v < NV; ++v) {
                gs0[v] = gs1[v] = gd0[v] = gd1[v] = 0.0;
                if (act && pos == 0) {
                    gs0[v] = P.gsb[fb_index<DIM, K>(ee, a, 0, v, tt)];
                    gd0[v] = P.gdb[fb_index<DIM, K>(ee, a, 0, v, tt)];
                }
                if (act && pos == K - 1) {
                    gs1[v] = P.gsb[fb_index<DIM, K>(ee, a, 1, v, tt)];
                    gd1[v] = P.gdb[fb_index<DIM, K>(ee, a, 1, v, tt)];
                }
            }
            for (int v = 0; v < NV; ++v) {
                S.GS[le][0][v][c] = gs0[v];
                S.GS[le][1][v][c] = gs1[v];
                S.GD[le][0][v][c] = gd0[v];
                S.GD[le][1][v][c] = gd1[v];
            }
        }
        __syncthreads();

        // ---------------- (2) reverse of the common fluxes on the interior faces ----------------
        const int nfaces = face_count<K>(1, step, true);
        int nfmax = nfaces;
        if (EPB > 1) {
            S.wsL[tid] = (double)nfaces;
            __syncthreads();
            for (int q = 0; q < EPB; ++q) nfmax = max(nfmax, (int)S.wsL[q * KD]);
            __syncthreads();
        }
        const int slot = c / KF, t = c % KF;
        for (int r0 = 0; r0 < nfmax; r0 += K) {
            const int fidx = r0 + slot;
            // an idle lane takes face 1, so that every cell it reads lies in the element
            int fa = a, k = 1;
            const bool has = fidx < nfaces;
            if (has) face_at<K>(a, 1, step, fidx, &fa, &k, true);
            double uL[NV], uR[NV], thL[MAXLEV + 1], thR[MAXLEV + 1];
            const int cl = G::from_trans(t, fa, k - 1), cr = G::from_trans(t, fa, k);
            theta_cell_of<DIM, K, LV>(S.al[le], cl, thL);
            theta_cell_of<DIM, K, LV>(S.al[le], cr, thR);
            for (int v = 0; v < NV; ++v) {
                uL[v] = thL[0] * S.u[le][v][cl];
                uR[v] = thR[0] * S.u[le][v][cr];
            }
#pragma unroll
            for (int li = 0; li < LV::NLEV; ++li) {
                CTab &T = P.tabs[li];
                int n = LV::n(li);
                if (thL[1 + li] != 0.0) {
                    int s = G::subelem(cl, n);
                    double b = S.be[le][LV::off(li) + s];
                    for (int v = 0; v < NV; ++v) {
                        double tr = bapply<DIM, K>(S.u[le][v], cl, fa, n, T.Ep);
                        uL[v] += thL[1 + li] * ((1.0 - b) * S.mean[le][v][LV::off(li) + s] + b * tr);
                    }
                }
                if (thR[1 + li] != 0.0) {
                    int s = G::subelem(cr, n);
                    double b = S.be[le][LV::off(li) + s];
                    for (int v = 0; v < NV; ++v) {
                        double tr = bapply<DIM, K>(S.u[le][v], cr, fa, n, T.Em);
                        uR[v] += thR[1 + li] * ((1.0 - b) * S.mean[le][v][LV::off(li) + s] + b * tr);
                    }
                }
            }
            double guL[NV], guR[NV], gdL[NV], gdR[NV];
            common_flux_adj<DIM, K, LV, EPB * KD>(P, &S.wsL[le * KD], &S.wsR[le * KD], c, slot * KF, t, has, fa, k, uL,
                                                  uR, thL, thR, own_sr, own_se, -1, cl, -1, cr, &S.u[le][0][0], ee,
                                                  &S.gF[le][0][k * KF], (K + 1) * KF, guL, guR, gdL, gdR);
            if (has)
                for (int v = 0; v < NV; ++v) {
                    S.GS[le][1][v][cl] = guL[v];
                    S.GS[le][0][v][cr] = guR[v];
                    S.GD[le][1][v][cl] = gdL[v];
                    S.GD[le][0][v][cr] = gdR[v];
                }
        }
        __syncthreads();

        // ---------------- (3) interface-state adjoints -> state adjoints ----------------
        {
            double gs[NV];
            for (int v = 0; v < NV; ++v) {
                gs[v] = S.GS[le][0][v][c] + S.GS[le][1][v][c];
                gu[v] += th[0] * gs[v] + S.GD[le][0][v][c] + S.GD[le][1][v][c];
            }
#pragma unroll
            for (int li = 0; li < LV::NLEV; ++li) {
                // a level the element does not use contributes nothing (the flag is uniform
                // over the element's lanes, and the reduction stays inside the element)
                if (!actv[1 + li]) continue;
                const double thn = th[1 + li];
                CTab &T = P.tabs[li];
                const int n = LV::n(li), ln = ilog2i(n);
                const double b = S.be[le][LV::off(li) + sidx[li]];
                const double nd = (DIM == 2) ? n * n : n * n * n;
                for (int v = 0; v < NV; ++v) {
                    // the trace part through E^T along a; the squeeze-mean part summed over the sub-element
                    const double ms = subreduce<DIM, K>(thn * gs[v], ln, S.wsL, OpSum());
                    if (thn != 0.0) {
                        const double tr = bapply<DIM, K>(S.GS[le][0][v], c, a, n, T.EmT) +
                                          bapply<DIM, K>(S.GS[le][1][v], c, a, n, T.EpT);
                        gu[v] += thn * b * tr + (1.0 - b) * ms / nd;
                    }
                }
            }
        }
        __syncthreads();
    }

    if (!act) return;
    if (P.stage == 0) {
        for (int v = 0; v < NV; ++v) P.out[v * P.dof + g] = gu[v];
        return;
    }
    // transposed SSP-RK3 stages (stage codes 13, 12, 11 reverse stages 3, 2, 1)
    const double dt = *P.dt;
    double ac[NV];
    if (P.stage != 13)
        for (int v = 0; v < NV; ++v) ac[v] = P.acc[v * P.dof + g];
    for (int v = 0; v < NV; ++v) {
        const long long i = v * P.dof + g;
        const double l = S.lam[le][v][c];
        if (P.stage == 13) {
            P.out[i] = (2.0 / 3.0) * (l + dt * gu[v]);
            P.acc[i] = (1.0 / 3.0) * l;
        } else if (P.stage == 12) {
            P.out[i] = 0.25 * (l + dt * gu[v]);
            P.acc[i] = ac[v] + 0.75 * l;
        } else {
            P.out[i] = ac[v] + l + dt * gu[v];
        }
    }
}

// Reverse of the common fluxes on the element faces, once per face (the transpose of
// eface_kernel): face tasks (element, axis) of KF lanes, 64 / KF per workgroup, each
// the element's low face along the axis plus its high face at an outflow boundary.
// The flux adjoint on a face is the sum of the two elements' shares (P.gfb); the
// interface-state adjoints (P.gsb) and mean-fallback adjoints (P.gdb) of each side go
// to the element owning that side, in the face-buffer layout (at an outflow boundary
// the mirrored side adds to the own one).
template <int DIM, int K, int TOP>
__global__ void __launch_bounds__(64) eface_adjoint_kernel(KArgs P)
{
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    constexpr int NV = G::NV, KF = G::KF, NS = 64 / KF;
    __shared__ double wsL[64], wsR[64], wsG[NV * 64];
    const int c = threadIdx.x, slot = c / KF, t = c % KF;
    const long long task = (long long)xcd_tile(blockIdx.x, gridDim.x) * NS + slot;
    const bool valid = task < (long long)P.nel * DIM;
    const int e = valid ? (int)(task / DIM) : 0, a = valid ? (int)(task % DIM) : 0;
    int e3[3];
    elem3(P, e, e3);
    const double own_sr = P.scale[2 * (long long)e], own_se = P.scale[2 * (long long)e + 1];
    for (int sd = 0; sd < 2; ++sd) {
        const int nb = neighbour<DIM>(P, e3, a, sd);
        const bool has = valid && (sd == 0 || nb < 0);
        if (!block_or<64>(has)) continue;
        const int nbc = nb >= 0 ? nb : e;
        double uL[NV], uR[NV], thL[MAXLEV + 1], thR[MAXLEV + 1], srho = own_sr, sE = own_se;
        int mLe = -1, mLc = 0, mRe = -1, mRc = 0;
        double go[NV], gn[NV];
        for (int v = 0; v < NV; ++v) {
            go[v] = P.gfb[fb_index<DIM, K>(e, a, sd, v, t)];
            gn[v] = P.gfb[fb_index<DIM, K>(nbc, a, 1 - sd, v, t)];
        }
        element_face_sides<DIM, K, LV>(P, e, a, t, sd == 1, nb, P.alpha + (long long)e * LV::A,
                                       P.alpha + (long long)nbc * LV::A, own_sr, own_se, uL, uR, thL, thR, mLe, mLc,
                                       mRe, mRc, srho, sE);
        for (int v = 0; v < NV; ++v) wsG[v * 64 + c] = go[v] + (nb >= 0 ? gn[v] : 0.0);
        __syncthreads();
        double guL[NV], guR[NV], gdL[NV], gdR[NV];
        common_flux_adj<DIM, K, LV, 64>(P, wsL, wsR, c, slot * KF, t, has, a, sd ? K : 0, uL, uR, thL, thR, srho, sE,
                                        mLe, mLc, mRe, mRc, nullptr, e, wsG + slot * KF, 64, guL, guR, gdL, gdR);
        if (has) {
            if (sd == 0) {
                // own side: the right one; the left belongs to the low neighbour's high face,
                // or at an outflow boundary is the own boundary cell's mean
                for (int v = 0; v < NV; ++v) {
                    P.gsb[fb_index<DIM, K>(e, a, 0, v, t)] = guR[v];
                    P.gdb[fb_index<DIM, K>(e, a, 0, v, t)] = gdR[v] + (nb < 0 ? gdL[v] + guL[v] : 0.0);
                }
                if (nb >= 0)
                    for (int v = 0; v < NV; ++v) {
                        P.gsb[fb_index<DIM, K>(nb, a, 1, v, t)] = guL[v];
                        P.gdb[fb_index<DIM, K>(nb, a, 1, v, t)] = gdL[v];
                    }
            } else {
                // an outflow high face: own side left, the exterior (right) the own cell's mean
                for (int v = 0; v < NV; ++v) {
                    P.gsb[fb_index<DIM, K>(e, a, 1, v, t)] = guL[v];
                    P.gdb[fb_index<DIM, K>(e, a, 1, v, t)] = gdL[v] + gdR[v] + guR[v];
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// batched ensembles of independent 2-D problems
// ---------------------------------------------------------------------------
//
// The problems of an ensemble share the scheme parameters but not the mesh:
// each has its own element counts, boundary conditions, spacing, K (4 or 8) and
// step size.  Their states, blending factors, face buffers and scales sit back to
// back in ensemble-wide arrays; a tile is EPB consecutive elements of one problem
// and the tiles of all problems are numbered consecutively.  One launch of the
// analyse kernel and one of the residual kernel per RK stage cover the whole
// ensemble: each workgroup takes a range of tiles, reads its problem's
// descriptor and runs the K = 4 or K = 8 body (a workgroup-uniform branch; both
// bodies use the same workgroup size and share one LDS allocation).

#define BATCH_SLOTS 16      // CFL slots per problem

struct ProbDesc {
    long long state_off;    // doubles before the problem's state (nvar * dof each)
    long long alpha_off;    // doubles before its blending factors (nel * A each)
    long long fbuf_off;     // doubles before its face buffer
    long long elem_off;     // elements before it
    long long dof;
    int nel, K, tile_off, ntiles;
    int ftile_off;          // element-face tiles before it
    int ne[2], G[2], bc[2];
    double dx[2];
    double cfl_num;         // numerator of its CFL step
};

// Workgroup-uniform values loaded from memory: readfirstlane tells the compiler they
// are uniform, so they and everything derived from them stay in scalar registers.
__device__ __forceinline__ int wg_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long wg_uniform(long long v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wg_uniform(double v) { return __longlong_as_double(wg_uniform(__double_as_longlong(v))); }

// the kernel arguments of one problem of the ensemble (D read with uniform loads)
__device__ __forceinline__ KArgs problem_args(const KArgs &P, const ProbDesc &Dm, int p)
{
    ProbDesc D;
    D.state_off = wg_uniform(Dm.state_off);
    D.alpha_off = wg_uniform(Dm.alpha_off);
    D.fbuf_off = wg_uniform(Dm.fbuf_off);
    D.elem_off = wg_uniform(Dm.elem_off);
    D.dof = wg_uniform(Dm.dof);
    D.nel = wg_uniform(Dm.nel);
    D.K = wg_uniform(Dm.K);
    for (int a = 0; a < 2; ++a) {
        D.ne[a] = wg_uniform(Dm.ne[a]);
        D.G[a] = wg_uniform(Dm.G[a]);
        D.bc[a] = wg_uniform(Dm.bc[a]);
        D.dx[a] = wg_uniform(Dm.dx[a]);
    }
    KArgs Q = P;
    Q.u = P.u + D.state_off;
    Q.u0 = P.u0 ? P.u0 + D.state_off : nullptr;
    Q.x1 = P.x1 ? P.x1 + D.state_off : nullptr;
    Q.y0 = P.y0 ? P.y0 + D.state_off : nullptr;
    Q.yout = P.yout ? P.yout + D.state_off : nullptr;
    Q.out = P.out + D.state_off;
    Q.alpha = P.alpha + D.alpha_off;
    Q.beta = P.beta + D.alpha_off;
    Q.mean = P.mean + 4 * D.alpha_off;      // nvar = 4 in 2-D
    Q.fbuf = P.fbuf + D.fbuf_off;
    Q.ef = P.ef ? P.ef + D.fbuf_off : nullptr;
    Q.scale = P.scale + 2 * D.elem_off;
    Q.lam_part = P.lam_part ? P.lam_part + (long long)p * BATCH_SLOTS : nullptr;
    Q.dt = P.dt ? P.dt + p : nullptr;
    Q.tabs = (D.K == 4) ? P.tabs + 1 : P.tabs;   // level tables 8, 4, 2: K = 4 starts at 4
    Q.err_base = (int)D.elem_off;
    Q.lam_mask = BATCH_SLOTS - 1;
    Q.dof = D.dof;
    Q.nel = D.nel;
    Q.ne[0] = D.ne[0]; Q.ne[1] = D.ne[1]; Q.ne[2] = 1;
    Q.G[0] = D.G[0]; Q.G[1] = D.G[1]; Q.G[2] = 1;
    Q.bc[0] = D.bc[0]; Q.bc[1] = D.bc[1]; Q.bc[2] = SEDG_PERIODIC;
    Q.dx[0] = D.dx[0]; Q.dx[1] = D.dx[1]; Q.dx[2] = 1.0;
    return Q;
}

// WA: waves per SIMD the register allocation of the analyse kernel is asked to leave
// room for (a tuning dimension: more waves hide more latency, fewer registers may spill)
template <int EPB4, int EPB8, bool PERSIST, int WA>
__global__ void __launch_bounds__(64 * EPB8)
__attribute__((amdgpu_waves_per_eu(WA, 8))) analyse_batch_kernel(KArgs P)
{
    static_assert(16 * EPB4 == 64 * EPB8, "one workgroup size for both K");
    __shared__ union {
        AnalyseSmem<2, 4, 4, EPB4> k4;
        AnalyseSmem<2, 8, 8, EPB8> k8;
    } U;
    const int L = P.xcd_map ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int t0 = PERSIST ? L * P.chunk : L;
    const int t1 = PERSIST ? min(P.ntiles, (L + 1) * P.chunk) : L + 1;
    for (int t = t0; t < t1; ++t) {
        const int p = wg_uniform(P.tile_prob[t]);
        const ProbDesc &D = P.probs[p];
        const KArgs Q = problem_args(P, D, p);
        const int tl = t - wg_uniform(D.tile_off);
        if (wg_uniform(D.K) == 4) analyse_body<2, 4, 4, EPB4>(Q, tl, U.k4);
        else analyse_body<2, 8, 8, EPB8>(Q, tl, U.k8);
        __syncthreads();
    }
}

// the analysis of the problems of one K: one workgroup per tile of the range
// [tile_base, tile_base + grid) (which holds that K's tiles only)
template <int K, int EPB, int WA>
__global__ void __launch_bounds__((EPB * Geo<2, K>::KD))
__attribute__((amdgpu_waves_per_eu(WA, 8))) analyse_batch_one_kernel(KArgs P)
{
    __shared__ AnalyseSmem<2, K, K, EPB> S;
    const int t = P.tile_base + (P.xcd_map ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x);
    const int p = wg_uniform(P.tile_prob[t]);
    const ProbDesc &D = P.probs[p];
    const KArgs Q = problem_args(P, D, p);
    analyse_body<2, K, K, EPB>(Q, t - wg_uniform(D.tile_off), S);
}

template <int EPB4, int EPB8, bool PERSIST>
__global__ void __launch_bounds__(64 * EPB8)
__attribute__((amdgpu_waves_per_eu(3, 8))) residual_batch_kernel(KArgs P)
{
    static_assert(16 * EPB4 == 64 * EPB8, "one workgroup size for both K");
    __shared__ union {
        ResidualSmem<2, 4, 4, EPB4> k4;
        ResidualSmem<2, 8, 8, EPB8> k8;
    } U;
    const int L = P.xcd_map ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int t0 = PERSIST ? L * P.chunk : L;
    const int t1 = PERSIST ? min(P.ntiles, (L + 1) * P.chunk) : L + 1;
    for (int t = t0; t < t1; ++t) {
        const int p = wg_uniform(P.tile_prob[t]);
        const ProbDesc &D = P.probs[p];
        const KArgs Q = problem_args(P, D, p);
        const int tl = t - wg_uniform(D.tile_off);
        if (wg_uniform(D.K) == 4) residual_body<2, 4, 4, EPB4>(Q, tl, U.k4);
        else residual_body<2, 8, 8, EPB8>(Q, tl, U.k8);
        __syncthreads();
    }
}

// element-face fluxes of the ensemble: every face tile (64 / K face tasks of one problem)
// is one workgroup of 64 lanes
__global__ void __launch_bounds__(64) eface_batch_kernel(KArgs P)
{
    __shared__ double wsL[4 * 64], wsR[4 * 64];
    const int L = P.xcd_map ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int p = wg_uniform(P.ftile_prob[L]);
    const ProbDesc &D = P.probs[p];
    const KArgs Q = problem_args(P, D, p);
    const int tl = L - wg_uniform(D.ftile_off);
    if (wg_uniform(D.K) == 4) eface_body<2, 4, 4>(Q, tl, wsL, wsR);
    else eface_body<2, 8, 8>(Q, tl, wsL, wsR);
}

// per-problem CFL steps: one workgroup of BATCH_SLOTS threads per problem, which
// also clears the problem's slots for the next step
__global__ void __launch_bounds__(BATCH_SLOTS) finalize_batch_kernel(double *lam_part, const ProbDesc *probs, int nprob,
                                                                     double *dt, double *dt_log, const int *step_ctr)
{
    __shared__ double s[BATCH_SLOTS];
    const int p = blockIdx.x, i = threadIdx.x;
    s[i] = lam_part[(long long)p * BATCH_SLOTS + i];
    lam_part[(long long)p * BATCH_SLOTS + i] = 0.0;
    __syncthreads();
    for (int w = BATCH_SLOTS / 2; w > 0; w >>= 1) {
        if (i < w) s[i] = fmax(s[i], s[i + w]);
        __syncthreads();
    }
    if (i == 0) {
        const double d = probs[p].cfl_num / s[0];
        dt[p] = d;
        if (dt_log) dt_log[(long long)step_ctr[0] * nprob + p] = d;
    }
}

__global__ void fill_kernel(double *x, int n, double v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ void count_step_kernel(int *ctr)
{
    if (threadIdx.x == 0) ctr[0] += 1;
}

// CFL step from the eigenvalue maxima folded into LAM_SLOTS slots (eq. cfl-condition);
// one block of LAM_SLOTS threads, which also clears the slots for the next step.
__global__ void __launch_bounds__(LAM_SLOTS) finalize_dt_kernel(double *lam_part, int nparts, double num, double *dt,
                                                               double *dt_log, int *step_ctr)
{
    __shared__ double s[LAM_SLOTS];
    (void)nparts;
    s[threadIdx.x] = lam_part[threadIdx.x];
    lam_part[threadIdx.x] = 0.0;
    __syncthreads();
    for (int w = LAM_SLOTS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double d = num / s[0];
        dt[0] = d;
        if (dt_log) dt_log[step_ctr[0]] = d;
    }
}

// RANDOM mode: the next right-hand side draws new factors
__global__ void draw_advance_kernel(long long *draw)
{
    if (threadIdx.x == 0) draw[0] += 1;
}

// step-size log of a fixed-step run: dt_log[step] = dt
__global__ void log_dt_kernel(const double *dt, double *dt_log, const int *step_ctr)
{
    if (threadIdx.x == 0) dt_log[step_ctr[0]] = dt[0];
}

// factor log: the factors of stage `stage` of step step_ctr go to
// log[(nstages * step + stage) * n ...]
__global__ void log_alpha_kernel(const double *alpha, double *log, const int *step_ctr, int stage, long long n,
                                 int nstages)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) log[((long long)nstages * step_ctr[0] + stage) * n + i] = alpha[i];
}

// state check of sedg_init_state: the smallest element index holding a mean value that
// is not finite or not permissible
template <int DIM>
__global__ void check_state_kernel(const double *u, long long dof, int G0, int G1, int K, int ne0, int ne1, int *err,
                                   double gam)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dof) return;
    constexpr int NV = DIM + 2;
    double ub[NV];
    bool fin = true;
    for (int v = 0; v < NV; ++v) {
        ub[v] = u[v * dof + i];
        fin = fin && isfinite(ub[v]);
    }
    const Gas gs = {gam, gam - 1.0};
    if (fin && permissible<DIM>(ub, gs)) return;
    const long long gx = i % G0, r = i / G0, gy = r % G1, gz = r / G1;
    const int e = (int)(gx / K + (long long)ne0 * (gy / K + (long long)ne1 * (gz / K)));
    atomicMin(err, e);
}

// Diagnostics of one right-hand side, one thread per element: the element's share of
// the change of bulk (eq. change-of-bulk, with |Omega_q| as a weight) and of its
// absolute value, the weighted blending factor of every subcell (eq. order-estimate,
// its nested form: start at 1 (FV) and take levels from the lowest up,
// abar = abar (1 - alpha_n) + n alpha_n), the lowest order carrying weight in the
// element, and its squeezed and rejected sub-elements.  Record per element:
// [bulk x NV | |bulk| x NV | abar min, sum, max | lowest order | squeezed | rejected].
struct DiagGeo {
    int dim, K, nv, nlev, A;
    int lev_n[MAXLEV], lev_off[MAXLEV];
    int ne[3];
    int G[3];
    long long dof;
    int nel;
    double vol;            // |Omega_q| / K^dim: the weight of one subcell mean
    double beta_L;
};

__global__ void diag_kernel(DiagGeo D, const double *dudt, const double *alpha, const double *beta, double *abar_out,
                            double *rec)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= D.nel) return;
    const int R = 2 * D.nv + 6;
    double *r = rec + (long long)e * R;
    const int ex = e % D.ne[0], ey = (e / D.ne[0]) % D.ne[1], ez = e / (D.ne[0] * D.ne[1]);
    const int ky = D.dim > 1 ? D.K : 1, kz = D.dim > 2 ? D.K : 1;
    double bulk[5] = {0, 0, 0, 0, 0}, babs[5] = {0, 0, 0, 0, 0};
    double amin = 1e300, asum = 0.0, amax = -1e300;
    bool fv = false;
    bool lvl[MAXLEV] = {false, false, false};
    const double *al = alpha + (long long)e * D.A;
    for (int k = 0; k < kz; ++k)
        for (int j = 0; j < ky; ++j)
            for (int i = 0; i < D.K; ++i) {
                const long long g = (long long)ex * D.K + i +
                                    (long long)D.G[0] * (((long long)ey * D.K + j) + (long long)D.G[1] * ((long long)ez * D.K + k));
                for (int v = 0; v < D.nv; ++v) {
                    const double x = dudt[v * D.dof + g];
                    bulk[v] += D.vol * x;
                    babs[v] += D.vol * fabs(x);
                }
                double a[MAXLEV], prod = 1.0;
                for (int li = 0; li < D.nlev; ++li) {
                    const int n = D.lev_n[li], ns = D.K / n;
                    const int sx = i / n, sy = D.dim > 1 ? j / n : 0, sz = D.dim > 2 ? k / n : 0;
                    a[li] = al[D.lev_off[li] + sx + ns * (sy + ns * sz)];
                    if (a[li] * prod != 0.0) lvl[li] = true;
                    prod *= 1.0 - a[li];
                }
                if (prod != 0.0) fv = true;
                double ab = 1.0;
                for (int li = D.nlev - 1; li >= 0; --li) ab = ab * (1.0 - a[li]) + D.lev_n[li] * a[li];
                amin = fmin(amin, ab);
                amax = fmax(amax, ab);
                asum += ab;
                if (abar_out) abar_out[g] = ab;
            }
    int low = 0;
    if (fv) low = 1;
    else
        for (int li = 0; li < D.nlev; ++li)
            if (lvl[li]) low = D.lev_n[li];
    int sq = 0, rej = 0;
    for (int q = 0; q < D.A; ++q) {
        const double b = beta[(long long)e * D.A + q];
        sq += b < 1.0 ? 1 : 0;
        rej += b < D.beta_L ? 1 : 0;
    }
    for (int v = 0; v < D.nv; ++v) { r[v] = bulk[v]; r[D.nv + v] = babs[v]; }
    r[2 * D.nv] = amin;
    r[2 * D.nv + 1] = asum;
    r[2 * D.nv + 2] = amax;
    r[2 * D.nv + 3] = low;
    r[2 * D.nv + 4] = sq;
    r[2 * D.nv + 5] = rej;
}

__global__ void set_int_kernel(int *x, int v)
{
    if (threadIdx.x == 0) x[0] = v;
}

__global__ void set_scalars_kernel(double *dt, double val, int *step_ctr)
{
    if (threadIdx.x == 0) {
        if (dt) dt[0] = val;
        if (step_ctr) step_ctr[0] = 0;
    }
}

// ---------------------------------------------------------------------------
// blended refinement and coarsening (App., non-conforming interfaces)
// ---------------------------------------------------------------------------
// Refinement of a parent element (eq. 3D-refinement), written for the multi-level
// weights: every fine subcell takes theta_FV of its parent cell times the parent cell's
// mean (the expansion E = I (x) 1_2) plus, for each DG level n, theta^(n) times the mean
// over the fine subcell of the level-n sub-element's nodal polynomial (Z = P^(n -> 2n)
// along every axis).  Coarsening (eq. 3D-coarsening) compresses each child separately:
// theta_FV times the mean of the 2^d fine cells (C = 1/2 I (x) 1_2^T) plus theta^(n) times
// the means over the coarse subcells of the child's level-n polynomials (Q = P^(n -> n/2)),
// and glues the 2^d children.  With the single-level weights (levels {1, K}) these are the
// paper's formulas; both conserve every element's total for any factors.

typedef const __attribute__((address_space(4))) sedg_nc_tab CNc;

struct RcArgs {
    const double *in;       // refine: coarse state; coarsen: fine state
    const double *alpha;    // factors of the input mesh's elements (A per element)
    double *out;            // refine: fine state; coarsen: coarse state
    CTab *tabs;
    CNc *nc;
    long long dof_c, dof_f; // subcells of the coarse and the fine mesh
    int ne[3];              // coarse elements per axis (1 on unused axes)
    int Gc[3], Gf[3];       // coarse and fine subcell extents
};

// out = in x_a M within blocks along axis a: the extents of in are ext, those of out ext
// with ext[a] replaced by ext[a] / n * ro; M is ro x n (row-major), applied to the n
// inputs of each block of n along a.  Work spread over the workgroup.
__device__ __forceinline__ void rc_pass(const double *in, double *out, const int *ext, int a, int ro, int n,
                                        CDbl *M, int tid, int nthr)
{
    int eo[3] = {ext[0], ext[1], ext[2]};
    eo[a] = ext[a] / n * ro;
    const int total = eo[0] * eo[1] * eo[2];
    for (int o = tid; o < total; o += nthr) {
        int oc[3] = {o % eo[0], (o / eo[0]) % eo[1], o / (eo[0] * eo[1])};
        const int oa = (a == 0) ? oc[0] : (a == 1) ? oc[1] : oc[2];
        const int b = oa / ro, r = oa - b * ro;
        const int st = (a == 0) ? 1 : (a == 1) ? ext[0] : ext[0] * ext[1];
        int ic[3] = {oc[0], oc[1], oc[2]};
        if (a == 0) ic[0] = b * n; else if (a == 1) ic[1] = b * n; else ic[2] = b * n;
        const int base = ic[0] + ext[0] * (ic[1] + ext[1] * ic[2]);
        double acc = 0.0;
        for (int m = 0; m < n; ++m) acc += M[r * n + m] * in[base + m * st];
        out[o] = acc;
    }
}

template <int DIM, int K, int TOP>
__global__ void __launch_bounds__((Geo<DIM, K>::KD)) refine_kernel(RcArgs A)
{
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    constexpr int KD = G::KD, NV = G::NV, ND = 1 << DIM, FD = KD * ND, F = 2 * K;
    __shared__ double s_al[LV::A];
    __shared__ double s_u[KD], s_a[FD], s_b[FD];
    const int e = blockIdx.x, c = threadIdx.x;
    int e3[3] = {e % A.ne[0], (e / A.ne[0]) % A.ne[1], e / (A.ne[0] * A.ne[1])};
    const int cx = G::coord(c, 0), cy = G::coord(c, 1), cz = DIM == 3 ? G::coord(c, 2) : 0;
    const long long gx = (long long)e3[0] * K + cx, gy = (long long)e3[1] * K + cy,
                    gz = DIM == 3 ? (long long)e3[2] * K + cz : 0;
    const long long g = gx + A.Gc[0] * (gy + (long long)A.Gc[1] * gz);
    for (int q = c; q < LV::A; q += KD) s_al[q] = A.alpha[(long long)e * LV::A + q];
    __syncthreads();
    int sidx[MAXLEV];
    subidx_all<DIM, K, LV>(c, sidx);
    double th[MAXLEV + 1];
    theta_from_alpha<LV>(s_al, sidx, th);
    // the parent cell's 2^d fine cells: index inside the element's (2K)^d block and in the fine grid
    int fl[ND];
    long long fg[ND];
    for (int k = 0; k < ND; ++k) {
        const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
        fl[k] = (2 * cx + dx) + F * ((2 * cy + dy) + F * (DIM == 3 ? 2 * cz + dz : 0));
        fg[k] = (2 * gx + dx) + A.Gf[0] * ((2 * gy + dy) + (long long)A.Gf[1] * (DIM == 3 ? 2 * gz + dz : 0));
    }
    const int ek[3] = {K, K, DIM == 3 ? K : 1};
    for (int v = 0; v < NV; ++v) {
        const double ub = A.in[v * A.dof_c + g];
        double acc[ND];
        for (int k = 0; k < ND; ++k) acc[k] = th[0] * ub;
        s_u[c] = ub;
        __syncthreads();
#pragma unroll
        for (int li = 0; li < LV::NLEV; ++li) {
            if (!block_or<KD>(th[1 + li] != 0.0)) continue;
            const int n = LV::n(li);
            CTab &T = A.tabs[li];
            // nodal polynomial of every level-n sub-element: R along every axis
            double *src = s_u, *dst = s_a;
            for (int ax = 0; ax < DIM; ++ax) {
                rc_pass(src, dst, ek, ax, n, n, T.R, c, KD);
                __syncthreads();
                src = dst;
                dst = (dst == s_a) ? s_b : s_a;
            }
            // means over the fine subcells: Z along every axis (extents grow to 2K)
            int ex[3] = {K, K, DIM == 3 ? K : 1};
            for (int ax = 0; ax < DIM; ++ax) {
                rc_pass(src, dst, ex, ax, 2 * n, n, A.nc[li].Z, c, KD);
                __syncthreads();
                ex[ax] = F;
                src = dst;
                dst = (dst == s_a) ? s_b : s_a;
            }
            for (int k = 0; k < ND; ++k) acc[k] += th[1 + li] * src[fl[k]];
            __syncthreads();
        }
        for (int k = 0; k < ND; ++k) A.out[v * A.dof_f + fg[k]] = acc[k];
        __syncthreads();
    }
}

template <int DIM, int K, int TOP>
__global__ void __launch_bounds__((Geo<DIM, K>::KD)) coarsen_kernel(RcArgs A)
{
    typedef Geo<DIM, K> G;
    typedef Lv<DIM, K, TOP> LV;
    constexpr int KD = G::KD, NV = G::NV, ND = 1 << DIM, H = K / 2;
    constexpr int HD = (DIM == 2) ? H * H : H * H * H;
    __shared__ double s_al[LV::A];
    __shared__ double s_u[KD], s_a[KD], s_b[KD], s_o[KD];
    const int e = blockIdx.x, c = threadIdx.x;
    int e3[3] = {e % A.ne[0], (e / A.ne[0]) % A.ne[1], e / (A.ne[0] * A.ne[1])};
    const int fne0 = 2 * A.ne[0], fne1 = 2 * A.ne[1];
    const int ek[3] = {K, K, DIM == 3 ? K : 1};
    for (int v = 0; v < NV; ++v) {
        for (int r = 0; r < ND; ++r) {
            const int rx = r & 1, ry = (r >> 1) & 1, rz = (r >> 2) & 1;
            const int f3[3] = {2 * e3[0] + rx, 2 * e3[1] + ry, DIM == 3 ? 2 * e3[2] + rz : 0};
            const long long fe = f3[0] + (long long)fne0 * (f3[1] + (long long)fne1 * f3[2]);
            // the child's cell c and factors
            const long long fgx = (long long)f3[0] * K + G::coord(c, 0), fgy = (long long)f3[1] * K + G::coord(c, 1),
                            fgz = DIM == 3 ? (long long)f3[2] * K + G::coord(c, 2) : 0;
            s_u[c] = A.in[v * A.dof_f + fgx + A.Gf[0] * (fgy + (long long)A.Gf[1] * fgz)];
            for (int q = c; q < LV::A; q += KD) s_al[q] = A.alpha[fe * LV::A + q];
            __syncthreads();
            // this thread's coarse output inside the child, if any: child position p, whose
            // fine cells start at 2p (their weights are those of the fine cell 2p)
            const bool has = c < HD;
            const int p0 = c % H, p1 = (c / H) % H, p2 = DIM == 3 ? c / (H * H) : 0;
            const int fc = (2 * p0) + K * ((2 * p1) + K * (DIM == 3 ? 2 * p2 : 0));
            double th[MAXLEV + 1];
            {
                int sidx[MAXLEV];
                subidx_all<DIM, K, LV>(has ? fc : 0, sidx);
                theta_from_alpha<LV>(s_al, sidx, th);
            }
            double acc = 0.0;
            if (has) {
                double m = 0.0;
                for (int k = 0; k < ND; ++k) {
                    const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
                    m += s_u[fc + dx + K * (dy + K * dz)];
                }
                acc = th[0] * (m / ND);
            }
#pragma unroll
            for (int li = 0; li < LV::NLEV; ++li) {
                if (!block_or<KD>(has && th[1 + li] != 0.0)) continue;
                const int n = LV::n(li);
                CTab &T = A.tabs[li];
                double *src = s_u, *dst = s_a;
                for (int ax = 0; ax < DIM; ++ax) {
                    rc_pass(src, dst, ek, ax, n, n, T.R, c, KD);
                    __syncthreads();
                    src = dst;
                    dst = (dst == s_a) ? s_b : s_a;
                }
                int ex[3] = {K, K, DIM == 3 ? K : 1};
                for (int ax = 0; ax < DIM; ++ax) {
                    rc_pass(src, dst, ex, ax, n / 2, n, A.nc[li].Q, c, KD);
                    __syncthreads();
                    ex[ax] = H;
                    src = dst;
                    dst = (dst == s_a) ? s_b : s_a;
                }
                if (has) acc += th[1 + li] * src[c];
                __syncthreads();
            }
            // the coarse cell of the parent element this output fills
            if (has) s_o[(rx * H + p0) + K * ((ry * H + p1) + K * (DIM == 3 ? rz * H + p2 : 0))] = acc;
            __syncthreads();
        }
        const long long gx = (long long)e3[0] * K + G::coord(c, 0), gy = (long long)e3[1] * K + G::coord(c, 1),
                        gz = DIM == 3 ? (long long)e3[2] * K + G::coord(c, 2) : 0;
        A.out[v * A.dof_c + gx + A.Gc[0] * (gy + (long long)A.Gc[1] * gz)] = s_o[c];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct sedg_ctx {
    sedg_mesh mesh;
    sedg_params params;
    int nv, nel, A, nlev;
    int lev_n[MAXLEV], lev_off[MAXLEV];
    long long dof;
    int G[3];
    double dx[3];
    sedg_level_tab *d_tabs;
    double *d_alpha, *d_beta, *d_fbuf, *d_lam, *d_dt, *d_u0, *d_u1, *d_u2, *d_scale, *d_mean;
    double *d_ef;                          // element-face common fluxes
    double *d_u3;                          // fourth stage buffer of SSP-RK(5,4) (first use)
    sedg_nc_tab *d_nc;                     // refinement / coarsening tables (first use)
    double *d_gfb, *d_l1, *d_l2, *d_acc;   // adjoint (allocated on first use)
    double *d_gsb, *d_gdb;
    int *d_err, *d_ctr;
    long long *d_draw;                     // RANDOM mode: right-hand sides drawn so far
    int *d_fbc;                            // diagnostics: interface-safety fallback counter
    double *d_diag;                        // diagnostics: per-element records (first use)
    int nblocks;
    hipStream_t last;
    std::map<std::tuple<double *, double *, double *, int>, hipGraphExec_t> graphs;
    // event timing (benchmark mode)
    bool prof;
    std::vector<hipEvent_t> pool;
    size_t pool_used;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
    hipEvent_t prev;        // the event closing the last timed launch of the current call
};

namespace {

int epb_for(int dim, int K)
{
    if (dim == 2) return K == 4 ? 4 : 1;
    return 1;
}

bool supported(int dim, int K) { return (dim == 2 || dim == 3) && (K == 4 || K == 8); }

// element and subcell counts stay within the int arithmetic of the launches and the
// per-element indexing: at most SEDG_MAX_ELEMENTS elements (far beyond any mesh whose
// state fits in device memory) and at most INT_MAX subcells along an axis; counted in
// 64 bits, so that an oversized request is rejected rather than wrapped
static bool mesh_extent_ok(int dim, int K, const int *nelem)
{
    long long nel = 1;
    for (int a = 0; a < dim; ++a) {
        if (nelem[a] < 1 || (long long)nelem[a] * K > INT_MAX) return false;
        nel *= nelem[a];
        if (nel > SEDG_MAX_ELEMENTS) return false;
    }
    return true;
}

template <int DIM, int K, int TOP>
void launch_kernel(int which, const KArgs &P, int nblocks, hipStream_t s)
{
    constexpr int EPBv = (DIM == 2 && K == 4) ? 4 : 1;
    constexpr int threads = EPBv * Geo<DIM, K>::KD;
    if (which == 0) hipLaunchKernelGGL((analyse_kernel<DIM, K, TOP, EPBv>), dim3(nblocks), dim3(threads), 0, s, P);
    else if (which == 1) hipLaunchKernelGGL((residual_kernel<DIM, K, TOP, EPBv>), dim3(nblocks), dim3(threads), 0, s, P);
    else if (which == 2) hipLaunchKernelGGL((frozen_prep_kernel<DIM, K, TOP, EPBv>), dim3(nblocks), dim3(threads), 0, s, P);
    else if (which == 5) hipLaunchKernelGGL((face_adjoint_kernel<DIM, K, TOP, EPBv>), dim3(nblocks), dim3(threads), 0, s, P);
    else if (which == 6) {
        constexpr int NS = 64 / Geo<DIM, K>::KF;   // face tasks per workgroup
        const long long tasks = (long long)P.nel * DIM;
        hipLaunchKernelGGL((eface_kernel<DIM, K, TOP>), dim3((unsigned)((tasks + NS - 1) / NS)), dim3(64), 0, s, P);
    }
    else if constexpr (!(DIM == 3 && K == 8)) {  // one element's adjoint data exceed the LDS at 3-D K = 8
        if (which == 7) {
            constexpr int NS = 64 / Geo<DIM, K>::KF;
            const long long tasks = (long long)P.nel * DIM;
            hipLaunchKernelGGL((eface_adjoint_kernel<DIM, K, TOP>), dim3((unsigned)((tasks + NS - 1) / NS)), dim3(64), 0,
                               s, P);
        } else {
            hipLaunchKernelGGL((adjoint_kernel<DIM, K, TOP, EPBv>), dim3(nblocks), dim3(threads), 0, s, P);
        }
    }
}

template <int DIM, int K>
void launch_top(int which, int top, const KArgs &P, int nblocks, hipStream_t s)
{
    if (top == 2) launch_kernel<DIM, K, 2>(which, P, nblocks, s);
    else if (top == 4) launch_kernel<DIM, K, 4>(which, P, nblocks, s);
    else launch_kernel<DIM, K, (K >= 8 ? 8 : 4)>(which, P, nblocks, s);
}

void launch_shape(int which, int d, int K, int top, int nblocks, const KArgs &P, hipStream_t s)
{
    if (d == 2 && K == 4) launch_top<2, 4>(which, top, P, nblocks, s);
    else if (d == 2 && K == 8) launch_top<2, 8>(which, top, P, nblocks, s);
    else if (d == 3 && K == 4) launch_top<3, 4>(which, top, P, nblocks, s);
    else launch_top<3, 8>(which, top, P, nblocks, s);
}

void launch_any(int which, const sedg_ctx *C, const KArgs &P, hipStream_t s)
{
    launch_shape(which, C->mesh.dim, C->mesh.K, C->lev_n[0], C->nblocks, P, s);
}

void launch_analyse_any(const sedg_ctx *C, const KArgs &P, hipStream_t s) { launch_any(0, C, P, s); }
// the residual kernel reads the element-face fluxes of the face kernel launched before it
void launch_faces_any(const sedg_ctx *C, const KArgs &P, hipStream_t s) { launch_any(6, C, P, s); }
void launch_residual_only_any(const sedg_ctx *C, const KArgs &P, hipStream_t s) { launch_any(1, C, P, s); }
void launch_residual_any(const sedg_ctx *C, const KArgs &P, hipStream_t s)
{
    launch_faces_any(C, P, s);
    launch_residual_only_any(C, P, s);
}
void launch_prep_any(const sedg_ctx *C, const KArgs &P, hipStream_t s) { launch_any(2, C, P, s); }
void launch_adjoint_any(const sedg_ctx *C, const KArgs &P, hipStream_t s) { launch_any(3, C, P, s); }
void launch_face_adjoint_any(const sedg_ctx *C, const KArgs &P, hipStream_t s) { launch_any(5, C, P, s); }
// the adjoint kernel reads the element-face reverse of the kernel launched before it
void launch_eface_adjoint_any(const sedg_ctx *C, const KArgs &P, hipStream_t s) { launch_any(7, C, P, s); }

bool adjoint_supported(const sedg_ctx *C) { return !(C->mesh.dim == 3 && C->mesh.K == 8); }

// adjoint work buffers, allocated on first use
int ensure_adjoint_buffers(sedg_ctx *C)
{
    if (C->d_gfb) return SEDG_OK;
    size_t kf = 1;
    for (int a = 1; a < C->mesh.dim; ++a) kf *= C->mesh.K;
    size_t nst = (size_t)C->nv * C->dof;
    const size_t nfb = (size_t)C->nel * C->mesh.dim * 2 * C->nv * kf;
    bool ok = hipMalloc(&C->d_gfb, sizeof(double) * nfb) == hipSuccess;
    ok = ok && hipMalloc(&C->d_gsb, sizeof(double) * nfb) == hipSuccess;
    ok = ok && hipMalloc(&C->d_gdb, sizeof(double) * nfb) == hipSuccess;
    ok = ok && hipMalloc(&C->d_l1, sizeof(double) * nst) == hipSuccess;
    ok = ok && hipMalloc(&C->d_l2, sizeof(double) * nst) == hipSuccess;
    ok = ok && hipMalloc(&C->d_acc, sizeof(double) * nst) == hipSuccess;
    if (!ok) {
        void *ptrs[] = {C->d_gfb, C->d_gsb, C->d_gdb, C->d_l1, C->d_l2, C->d_acc};
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
        C->d_gfb = C->d_gsb = C->d_gdb = C->d_l1 = C->d_l2 = C->d_acc = nullptr;
        return SEDG_ENOMEM;
    }
    return SEDG_OK;
}

// the indicator's quick bound (see KArgs::ind_quick)
static double ind_quick(const sedg_params &p)
{
    return (p.tau_A >= 0.0 && p.tau_A <= DBL_MAX && p.tau_S > 0.0) ? 0.99 * p.tau_S : 0.0;
}

KArgs base_args(const sedg_ctx *C)
{
    KArgs P;
    std::memset(&P, 0, sizeof(P));
    P.alpha = C->d_alpha;
    P.beta = C->d_beta;
    P.fbuf = C->d_fbuf;
    P.ef = C->d_ef;
    P.scale = C->d_scale;
    P.mean = C->d_mean;
    P.tabs = (CTab *)C->d_tabs;
    P.err = C->d_err;
    P.lam_mask = LAM_SLOTS - 1;
    P.dof = C->dof;
    P.nel = C->nel;
    for (int a = 0; a < 3; ++a) {
        P.ne[a] = a < C->mesh.dim ? C->mesh.nelem[a] : 1;
        P.G[a] = C->G[a];
        P.bc[a] = C->mesh.bc[a];
        P.dx[a] = C->dx[a];
    }
    P.nlev = C->nlev;
    for (int li = 0; li < MAXLEV; ++li) { P.lev_n[li] = C->lev_n[li]; P.lev_off[li] = C->lev_off[li]; }
    P.A = C->A;
    P.mode = C->params.mode;
    P.level_mask = C->params.level_mask;
    P.gamma = C->mesh.gamma;
    P.gm1 = C->mesh.gamma - 1.0;
    P.tau_A = C->params.tau_A;
    P.tau_S = C->params.tau_S;
    P.alpha_H = C->params.alpha_H;
    P.alpha_L = C->params.alpha_L;
    P.beta_L = C->params.beta_L;
    P.sigma_floor = C->params.sigma_floor > 0.0 ? C->params.sigma_floor : 1.0;
    P.ind_quick = ind_quick(C->params);
    P.seed = C->params.seed;
    P.draw = C->d_draw;
    return P;
}

// after an analysis in RANDOM mode, the next one draws new factors
void advance_draw(const sedg_ctx *C, hipStream_t s)
{
    if (C->params.mode == SEDG_RANDOM) hipLaunchKernelGGL(draw_advance_kernel, dim3(1), dim3(64), 0, s, C->d_draw);
}

double cfl_numerator(const sedg_ctx *C)
{
    double dxm = C->dx[0];
    for (int a = 1; a < C->mesh.dim; ++a) dxm = dxm < C->dx[a] ? dxm : C->dx[a];
    return C->params.cfl * dxm / ((double)(1 << (C->mesh.dim - 1)) * (2.0 * C->mesh.K - 1.0));
}

int set_levels(sedg_ctx *C, const sedg_params *p)
{
    int K = C->mesh.K;
    int top = p->top_level > 0 ? p->top_level : K;
    if (top < 2 || top > K || (top & (top - 1))) return SEDG_EINVAL;
    if (p->mode < 0 || p->mode > SEDG_RANDOM) return SEDG_EINVAL;
    if (p->integrator != SEDG_SSPRK3 && p->integrator != SEDG_SSPRK54) return SEDG_EINVAL;
    C->params = *p;
    if (hipMemset(C->d_draw, 0, sizeof(long long)) != hipSuccess) return SEDG_EHIP;
    C->nlev = 0;
    int off = 0;
    for (int n = top; n >= 2; n /= 2) {
        int li = C->nlev++;
        C->lev_n[li] = n;
        C->lev_off[li] = off;
        int per = 1;
        for (int a = 0; a < C->mesh.dim; ++a) per *= K / n;
        off += per;
    }
    for (int li = C->nlev; li < MAXLEV; ++li) { C->lev_n[li] = 2; C->lev_off[li] = 0; }
    C->A = off;
    sedg_level_tab h[MAXLEV];
    std::memset(h, 0, sizeof(h));
    for (int li = 0; li < C->nlev; ++li)
        if (sedg_build_level(C->lev_n[li], C->mesh.family, &h[li])) return SEDG_EINVAL;
    if (hipMemcpy(C->d_tabs, h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return SEDG_EHIP;
    if (C->d_nc) {
        sedg_nc_tab hn[MAXLEV];
        std::memset(hn, 0, sizeof(hn));
        for (int li = 0; li < C->nlev; ++li)
            if (sedg_build_nc(C->lev_n[li], C->mesh.family, &hn[li])) return SEDG_EINVAL;
        if (hipMemcpy(C->d_nc, hn, sizeof(hn), hipMemcpyHostToDevice) != hipSuccess) return SEDG_EHIP;
    }
    for (auto &kv : C->graphs) (void)hipGraphExecDestroy(kv.second);
    C->graphs.clear();
    return SEDG_OK;
}

}  // namespace

extern "C" {

const char *sedg_strerror(int code)
{
    switch (code) {
    case SEDG_OK: return "ok";
    case SEDG_EINVAL: return "invalid argument";
    case SEDG_EHIP: return "HIP runtime error";
    case SEDG_ENOMEM: return "device allocation failed";
    case SEDG_ESTATE: return "non-permissible or non-finite mean value";
    case SEDG_EUNSUPPORTED: return "unsupported configuration";
    case SEDG_ESCRATCH: return "problem larger than the static work space of sedg_rhs_noalloc";
    default: return "unknown error";
    }
}

int sedg_create(const sedg_mesh *mesh, const sedg_params *params, sedg_ctx **out)
{
    if (!mesh || !params || !out) return SEDG_EINVAL;
    *out = nullptr;
    if (!supported(mesh->dim, mesh->K)) return SEDG_EUNSUPPORTED;
    if (!(mesh->gamma > 1.0)) return SEDG_EINVAL;
    if (mesh->family != SEDG_GAUSS && mesh->family != SEDG_LGL) return SEDG_EINVAL;
    if (!mesh_extent_ok(mesh->dim, mesh->K, mesh->nelem)) return SEDG_EINVAL;
    sedg_ctx *C = new sedg_ctx();
    C->mesh = *mesh;
    C->nv = mesh->dim + 2;
    C->nel = 1;
    C->dof = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < mesh->dim) {
            if (mesh->nelem[a] < 1 || !(mesh->hi[a] > mesh->lo[a])) { delete C; return SEDG_EINVAL; }
            if (mesh->bc[a] != SEDG_PERIODIC && mesh->bc[a] != SEDG_OUTFLOW) { delete C; return SEDG_EINVAL; }
            C->G[a] = mesh->nelem[a] * mesh->K;
            C->nel *= mesh->nelem[a];
            C->dx[a] = (mesh->hi[a] - mesh->lo[a]) / mesh->nelem[a];
        } else {
            C->G[a] = 1;
            C->dx[a] = 1.0;
            C->mesh.nelem[a] = 1;
        }
        C->dof *= C->G[a];
    }
    int epb = epb_for(mesh->dim, mesh->K);
    C->nblocks = (C->nel + epb - 1) / epb;
    int maxA = 0;
    for (int n = mesh->K; n >= 2; n /= 2) {
        int per = 1;
        for (int a = 0; a < mesh->dim; ++a) per *= mesh->K / n;
        maxA += per;
    }
    size_t kf = 1;
    for (int a = 1; a < mesh->dim; ++a) kf *= mesh->K;
    size_t nst = (size_t)C->nv * C->dof;
    bool ok = true;
    ok = ok && hipMalloc(&C->d_tabs, sizeof(sedg_level_tab) * MAXLEV) == hipSuccess;
    ok = ok && hipMalloc(&C->d_alpha, sizeof(double) * (size_t)C->nel * maxA) == hipSuccess;
    ok = ok && hipMalloc(&C->d_beta, sizeof(double) * (size_t)C->nel * maxA) == hipSuccess;
    ok = ok && hipMalloc(&C->d_fbuf, sizeof(double) * (size_t)C->nel * mesh->dim * 2 * C->nv * kf) == hipSuccess;
    ok = ok && hipMalloc(&C->d_lam, sizeof(double) * LAM_SLOTS) == hipSuccess;
    ok = ok && hipMalloc(&C->d_scale, sizeof(double) * 2 * (size_t)C->nel) == hipSuccess;
    ok = ok && hipMalloc(&C->d_ef, sizeof(double) * (size_t)C->nel * mesh->dim * 2 * C->nv * kf) == hipSuccess;
    ok = ok && hipMalloc(&C->d_mean, sizeof(double) * (size_t)C->nel * C->nv * maxA) == hipSuccess;
    ok = ok && hipMalloc(&C->d_dt, sizeof(double) * 2) == hipSuccess;
    ok = ok && hipMalloc(&C->d_u1, sizeof(double) * nst) == hipSuccess;
    ok = ok && hipMalloc(&C->d_u2, sizeof(double) * nst) == hipSuccess;
    ok = ok && hipMalloc(&C->d_err, sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc(&C->d_ctr, sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc(&C->d_draw, sizeof(long long)) == hipSuccess;
    ok = ok && hipMalloc(&C->d_fbc, sizeof(int)) == hipSuccess;
    if (!ok) { sedg_destroy(C); return SEDG_ENOMEM; }
    int big = INT_MAX;
    if (hipMemcpy(C->d_err, &big, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) { sedg_destroy(C); return SEDG_EHIP; }
    if (hipMemset(C->d_lam, 0, sizeof(double) * LAM_SLOTS) != hipSuccess) { sedg_destroy(C); return SEDG_EHIP; }
    int rc = set_levels(C, params);
    if (rc) { sedg_destroy(C); return rc; }
    C->last = nullptr;
    C->prof = false;
    C->pool_used = 0;
    *out = C;
    return SEDG_OK;
}

int sedg_destroy(sedg_ctx *C)
{
    if (!C) return SEDG_OK;
    (void)hipDeviceSynchronize();
    for (auto &kv : C->graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipEvent_t e : C->pool) (void)hipEventDestroy(e);
    void *ptrs[] = {C->d_tabs, C->d_alpha, C->d_beta, C->d_fbuf, C->d_lam, C->d_dt, C->d_u1, C->d_u2, C->d_err, C->d_ctr,
                    C->d_scale, C->d_mean, C->d_ef, C->d_gfb, C->d_gsb, C->d_gdb, C->d_l1, C->d_l2, C->d_acc,
                    C->d_draw, C->d_fbc, C->d_diag, C->d_u3, C->d_nc};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete C;
    return SEDG_OK;
}

long sedg_state_len(const sedg_ctx *C) { return C ? (long)(C->nv * C->dof) : SEDG_EINVAL; }
long sedg_alpha_len(const sedg_ctx *C) { return C ? (long)C->A * C->nel : SEDG_EINVAL; }

int sedg_set_params(sedg_ctx *C, const sedg_params *p)
{
    if (!C || !p) return SEDG_EINVAL;
    (void)hipDeviceSynchronize();
    return set_levels(C, p);
}

int sedg_rhs(sedg_ctx *C, const double *u, double *dudt, double *alpha_out, double *beta_out,
             const double *alpha_in, void *stream)
{
    if (!C || !u || !dudt || u == dudt) return SEDG_EINVAL;
    if (C->params.mode == SEDG_EXTERNAL && !alpha_in) return SEDG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    KArgs P = base_args(C);
    P.u = u;
    P.out = dudt;
    P.alpha_in = alpha_in;
    P.stage = 0;
    launch_analyse_any(C, P, s);
    advance_draw(C, s);
    launch_residual_any(C, P, s);
    size_t na = sizeof(double) * (size_t)C->A * C->nel;
    if (alpha_out && hipMemcpyAsync(alpha_out, C->d_alpha, na, hipMemcpyDeviceToDevice, s) != hipSuccess) return SEDG_EHIP;
    if (beta_out && hipMemcpyAsync(beta_out, C->d_beta, na, hipMemcpyDeviceToDevice, s) != hipSuccess) return SEDG_EHIP;
    C->last = s;
    return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
}

int sedg_max_dt(sedg_ctx *C, const double *u, double *dt_dev, void *stream)
{
    if (!C || !u || !dt_dev) return SEDG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    KArgs P = base_args(C);
    P.u = u;
    P.lam_part = C->d_lam;
    // the analyse pass also produces alpha/beta/face data (harmless side effect)
    P.mode = SEDG_FORCE_FV;
    launch_analyse_any(C, P, s);
    hipLaunchKernelGGL(finalize_dt_kernel, dim3(1), dim3(LAM_SLOTS), 0, s, C->d_lam, C->nblocks,
                       cfl_numerator(C), dt_dev, (double *)nullptr, (int *)nullptr);
    C->last = s;
    return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
}

}  // extern "C"

static hipEvent_t prof_event(sedg_ctx *C)
{
    if (C->pool_used == C->pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        C->pool.push_back(e);
    }
    return C->pool[C->pool_used++];
}

// launch f() on s and, when profiling, time it as kind 'kind': one event at every
// boundary between timed launches (the event closing one launch opens the next), so
// that the stream carries one marker per launch rather than two
template <typename F>
static void timed(sedg_ctx *C, int kind, hipStream_t s, F f)
{
    if (!C->prof) { f(); return; }
    hipEvent_t a = C->prev;
    if (!a) {
        a = prof_event(C);
        if (a) (void)hipEventRecord(a, s);
    }
    f();
    hipEvent_t b = prof_event(C);
    if (b) (void)hipEventRecord(b, s);
    if (a && b) C->marks.push_back({kind, {a, b}});
    C->prev = b;
}

static void enqueue_step(sedg_ctx *C, double *u, double dt_fixed, double *dt_log, double *alpha_log, hipStream_t s)
{
    KArgs P = base_args(C);
    P.dt = C->d_dt;
    const long long na = (long long)C->A * C->nel;
    auto log_alpha = [&](int stage) {
        if (alpha_log)
            hipLaunchKernelGGL(log_alpha_kernel, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, s, C->d_alpha,
                               alpha_log, C->d_ctr, stage, na, 3);
    };
    // stage 1: u1 = u + dt L(u)
    P.u = u;
    P.out = C->d_u1;
    P.stage = 1;
    P.lam_part = dt_fixed > 0.0 ? nullptr : C->d_lam;
    timed(C, 0, s, [&] { launch_analyse_any(C, P, s); });
    advance_draw(C, s);
    log_alpha(0);
    if (!(dt_fixed > 0.0)) {
        // the step size is formed inside the element-face launch that follows
        P.fin_lam = C->d_lam;
        P.fin_num = cfl_numerator(C);
        P.fin_dt = C->d_dt;
        P.fin_dt_log = dt_log;
        P.fin_ctr = C->d_ctr;
    } else if (dt_log)
        hipLaunchKernelGGL(log_dt_kernel, dim3(1), dim3(64), 0, s, (const double *)C->d_dt, dt_log, (const int *)C->d_ctr);
    timed(C, 3, s, [&] { launch_faces_any(C, P, s); });
    P.fin_lam = nullptr;
    timed(C, 1, s, [&] { launch_residual_only_any(C, P, s); });
    // stage 2: u2 = 3/4 u + 1/4 (u1 + dt L(u1))
    P.lam_part = nullptr;
    P.u = C->d_u1;
    P.u0 = u;
    P.out = C->d_u2;
    P.stage = 2;
    timed(C, 0, s, [&] { launch_analyse_any(C, P, s); });
    advance_draw(C, s);
    log_alpha(1);
    timed(C, 3, s, [&] { launch_faces_any(C, P, s); });
    timed(C, 1, s, [&] { launch_residual_only_any(C, P, s); });
    // stage 3: u = 1/3 u + 2/3 (u2 + dt L(u2))
    P.u = C->d_u2;
    P.u0 = u;
    P.out = u;
    P.stage = 3;
    timed(C, 0, s, [&] { launch_analyse_any(C, P, s); });
    advance_draw(C, s);
    log_alpha(2);
    timed(C, 3, s, [&] { launch_faces_any(C, P, s); });
    timed(C, 1, s, [&] { launch_residual_only_any(C, P, s); });
    if (dt_log || alpha_log) hipLaunchKernelGGL(count_step_kernel, dim3(1), dim3(64), 0, s, C->d_ctr);
}

// SSP-RK(5,4) of Spiteri & Ruuth (SIAM J. Numer. Anal. 40, 2002) in Shu-Osher form:
//   u1 = u + c10 dt L(u)
//   u2 = a20 u + a21 u1 + c21 dt L(u1)
//   u3 = a30 u + a32 u2 + c32 dt L(u2)
//   u4 = a40 u + a43 u3 + c43 dt L(u3)
//   u' = a52 u2 + a53 u3 + c53 dt L(u3) + a54 u4 + c54 dt L(u4)
// Buffers: u1 and then u3 in d_u1; u2 in d_u2, overwritten in place by stage 4 with
// a52 u2 + a53 u3 + c53 dt L(u3); u4 in d_u3.
namespace {
const double RK54_C10 = 0.391752226571890;
const double RK54_A20 = 0.444370493651235, RK54_A21 = 0.555629506348765, RK54_C21 = 0.368410593050371;
const double RK54_A30 = 0.620101851488403, RK54_A32 = 0.379898148511597, RK54_C32 = 0.251891774271694;
const double RK54_A40 = 0.178079954393132, RK54_A43 = 0.821920045606868, RK54_C43 = 0.544974750228521;
const double RK54_A52 = 0.517231671970585, RK54_A53 = 0.096059710526147, RK54_C53 = 0.063692468666290;
const double RK54_A54 = 0.386708617503269, RK54_C54 = 0.226007483236906;
}  // namespace

static void enqueue_step_rk54(sedg_ctx *C, double *u, double dt_fixed, double *dt_log, double *alpha_log,
                              hipStream_t s)
{
    KArgs P = base_args(C);
    P.dt = C->d_dt;
    const long long na = (long long)C->A * C->nel;
    auto log_alpha = [&](int stage) {
        if (alpha_log)
            hipLaunchKernelGGL(log_alpha_kernel, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, s, C->d_alpha,
                               alpha_log, C->d_ctr, stage, na, 5);
    };
    auto set = [&](double r0, double r1, double r2, double r3, double r4, double r5, double r6) {
        P.rk[0] = r0; P.rk[1] = r1; P.rk[2] = r2; P.rk[3] = r3; P.rk[4] = r4; P.rk[5] = r5; P.rk[6] = r6;
    };
    P.stage = 5;
    // stage 1
    P.u = u; P.u0 = nullptr; P.x1 = nullptr; P.y0 = nullptr; P.yout = nullptr; P.out = C->d_u1;
    set(0.0, 1.0, RK54_C10, 0.0, 0.0, 0.0, 0.0);
    P.lam_part = dt_fixed > 0.0 ? nullptr : C->d_lam;
    timed(C, 0, s, [&] { launch_analyse_any(C, P, s); });
    advance_draw(C, s);
    log_alpha(0);
    if (!(dt_fixed > 0.0)) {
        // the step size is formed inside the element-face launch that follows
        P.fin_lam = C->d_lam;
        P.fin_num = cfl_numerator(C);
        P.fin_dt = C->d_dt;
        P.fin_dt_log = dt_log;
        P.fin_ctr = C->d_ctr;
    } else if (dt_log)
        hipLaunchKernelGGL(log_dt_kernel, dim3(1), dim3(64), 0, s, (const double *)C->d_dt, dt_log, (const int *)C->d_ctr);
    timed(C, 3, s, [&] { launch_faces_any(C, P, s); });
    P.fin_lam = nullptr;
    timed(C, 1, s, [&] { launch_residual_only_any(C, P, s); });
    P.lam_part = nullptr;
    // stages 2 .. 5
    struct { double *in, *out; const double *u0, *x1, *y0; double *yout; double r[7]; } st[4] = {
        {C->d_u1, C->d_u2, u, nullptr, nullptr, nullptr, {RK54_A20, RK54_A21, RK54_C21, 0, 0, 0, 0}},
        {C->d_u2, C->d_u1, u, nullptr, nullptr, nullptr, {RK54_A30, RK54_A32, RK54_C32, 0, 0, 0, 0}},
        {C->d_u1, C->d_u3, u, nullptr, C->d_u2, C->d_u2, {RK54_A40, RK54_A43, RK54_C43, 0, RK54_A52, RK54_A53, RK54_C53}},
        {C->d_u3, u, nullptr, C->d_u2, nullptr, nullptr, {0, RK54_A54, RK54_C54, 1.0, 0, 0, 0}},
    };
    for (int k = 0; k < 4; ++k) {
        P.u = st[k].in;
        P.out = st[k].out;
        P.u0 = st[k].u0;
        P.x1 = st[k].x1;
        P.y0 = st[k].y0;
        P.yout = st[k].yout;
        set(st[k].r[0], st[k].r[1], st[k].r[2], st[k].r[3], st[k].r[4], st[k].r[5], st[k].r[6]);
        timed(C, 0, s, [&] { launch_analyse_any(C, P, s); });
        advance_draw(C, s);
        log_alpha(k + 1);
        timed(C, 3, s, [&] { launch_faces_any(C, P, s); });
        timed(C, 1, s, [&] { launch_residual_only_any(C, P, s); });
    }
    if (dt_log || alpha_log) hipLaunchKernelGGL(count_step_kernel, dim3(1), dim3(64), 0, s, C->d_ctr);
}

extern "C" {

int sedg_rk_step(sedg_ctx *C, double *u, int nsteps, double dt_fixed, double *dt_log_dev, double *alpha_log_dev,
                 void *stream)
{
    if (!C || !u || nsteps < 0) return SEDG_EINVAL;
    if (C->params.mode == SEDG_EXTERNAL) return SEDG_EINVAL;
    if (nsteps == 0) return SEDG_OK;
    const bool rk54 = C->params.integrator == SEDG_SSPRK54;
    if (rk54 && !C->d_u3 && hipMalloc(&C->d_u3, sizeof(double) * (size_t)C->nv * C->dof) != hipSuccess) {
        C->d_u3 = nullptr;
        return SEDG_ENOMEM;
    }
    auto step = [&](hipStream_t ss) {
        if (rk54) enqueue_step_rk54(C, u, dt_fixed, dt_log_dev, alpha_log_dev, ss);
        else enqueue_step(C, u, dt_fixed, dt_log_dev, alpha_log_dev, ss);
    };
    hipStream_t s = (hipStream_t)stream;
    // step counter / fixed step
    hipLaunchKernelGGL(set_scalars_kernel, dim3(1), dim3(64), 0, s, C->d_dt, dt_fixed > 0.0 ? dt_fixed : 0.0, C->d_ctr);
    if (C->prof) {
        C->prev = nullptr;
        for (int st = 0; st < nsteps; ++st) step(s);
        C->last = s;
        return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
    }
    auto key = std::make_tuple(u, dt_log_dev, alpha_log_dev, dt_fixed > 0.0 ? 1 : 0);
    hipGraphExec_t exec = nullptr;
    auto it = C->graphs.find(key);
    if (it != C->graphs.end()) {
        exec = it->second;
    } else {
        // bounded cache: a caller cycling through many state buffers re-captures
        if (C->graphs.size() >= 16) {
            if (hipStreamSynchronize(s) != hipSuccess) return SEDG_EHIP;
            for (auto &kv : C->graphs) (void)hipGraphExecDestroy(kv.second);
            C->graphs.clear();
        }
        hipStream_t cs;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return SEDG_EHIP;
        hipGraph_t graph;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) { (void)hipStreamDestroy(cs); return SEDG_EHIP; }
        step(cs);
        if (hipStreamEndCapture(cs, &graph) != hipSuccess) { (void)hipStreamDestroy(cs); return SEDG_EHIP; }
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) return SEDG_EHIP;
        C->graphs[key] = exec;
    }
    for (int st = 0; st < nsteps; ++st)
        if (hipGraphLaunch(exec, s) != hipSuccess) return SEDG_EHIP;
    C->last = s;
    return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
}

int sedg_profile(sedg_ctx *C, int on)
{
    if (!C) return SEDG_EINVAL;
    C->prof = on != 0;
    C->prev = nullptr;
    return SEDG_OK;
}

int sedg_profile_read(sedg_ctx *C, double *ms, long *count)
{
    if (!C || !ms || !count) return SEDG_EINVAL;
    if (hipStreamSynchronize(C->last) != hipSuccess) return SEDG_EHIP;
    for (int k = 0; k < 4; ++k) { ms[k] = 0.0; count[k] = 0; }
    for (auto &m : C->marks) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, m.second.first, m.second.second) != hipSuccess) return SEDG_EHIP;
        ms[m.first] += t;
        count[m.first] += 1;
    }
    C->marks.clear();
    C->pool_used = 0;
    C->prev = nullptr;
    return SEDG_OK;
}

int sedg_check(sedg_ctx *C, long *bad_elem)
{
    if (!C || !bad_elem) return SEDG_EINVAL;
    if (hipStreamSynchronize(C->last) != hipSuccess) return SEDG_EHIP;
    int h = INT_MAX;
    if (hipMemcpy(&h, C->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SEDG_EHIP;
    if (h == INT_MAX) { *bad_elem = -1; return SEDG_OK; }
    *bad_elem = h;
    int big = INT_MAX;
    if (hipMemcpy(C->d_err, &big, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return SEDG_EHIP;
    return SEDG_ESTATE;
}

int sedg_init_state(sedg_ctx *C, double *u_dev, const double *u_host, long *bad_elem)
{
    if (!C || !u_dev || !u_host) return SEDG_EINVAL;
    if (bad_elem) *bad_elem = -1;
    const size_t n = sizeof(double) * (size_t)C->nv * C->dof;
    if (hipDeviceSynchronize() != hipSuccess) return SEDG_EHIP;
    if (hipMemcpy(u_dev, u_host, n, hipMemcpyHostToDevice) != hipSuccess) return SEDG_EHIP;
    int big = INT_MAX, h = INT_MAX;
    if (hipMemcpy(C->d_err, &big, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return SEDG_EHIP;
    const unsigned nb = (unsigned)((C->dof + 255) / 256);
    if (C->mesh.dim == 2)
        hipLaunchKernelGGL(check_state_kernel<2>, dim3(nb), dim3(256), 0, 0, (const double *)u_dev, C->dof, C->G[0],
                           C->G[1], C->mesh.K, C->mesh.nelem[0], C->mesh.nelem[1], C->d_err, C->mesh.gamma);
    else
        hipLaunchKernelGGL(check_state_kernel<3>, dim3(nb), dim3(256), 0, 0, (const double *)u_dev, C->dof, C->G[0],
                           C->G[1], C->mesh.K, C->mesh.nelem[0], C->mesh.nelem[1], C->d_err, C->mesh.gamma);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return SEDG_EHIP;
    if (hipMemcpy(&h, C->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SEDG_EHIP;
    if (h == INT_MAX) return SEDG_OK;
    if (bad_elem) *bad_elem = h;
    if (hipMemcpy(C->d_err, &big, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return SEDG_EHIP;
    return SEDG_ESTATE;
}

int sedg_diagnose(sedg_ctx *C, const double *u, double *dudt, double *alpha_bar, sedg_diag *out, void *stream)
{
    if (!C || !u || !dudt || !out || u == dudt) return SEDG_EINVAL;
    if (C->params.mode == SEDG_EXTERNAL) return SEDG_EINVAL;
    const int R = 2 * C->nv + 6;
    if (!C->d_diag && hipMalloc(&C->d_diag, sizeof(double) * (size_t)R * C->nel) != hipSuccess) {
        C->d_diag = nullptr;
        return SEDG_ENOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    KArgs P = base_args(C);
    P.u = u;
    P.out = dudt;
    P.stage = 0;
    P.fbc = C->d_fbc;
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, s, C->d_fbc, 0);
    launch_analyse_any(C, P, s);
    advance_draw(C, s);
    launch_residual_any(C, P, s);
    DiagGeo D;
    std::memset(&D, 0, sizeof(D));
    D.dim = C->mesh.dim;
    D.K = C->mesh.K;
    D.nv = C->nv;
    D.nlev = C->nlev;
    D.A = C->A;
    for (int li = 0; li < MAXLEV; ++li) { D.lev_n[li] = C->lev_n[li]; D.lev_off[li] = C->lev_off[li]; }
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        D.ne[a] = C->mesh.nelem[a];
        D.G[a] = C->G[a];
        if (a < C->mesh.dim) vol *= C->dx[a] / C->mesh.K;
    }
    D.dof = C->dof;
    D.nel = C->nel;
    D.vol = vol;
    D.beta_L = C->params.beta_L;
    hipLaunchKernelGGL(diag_kernel, dim3((C->nel + 127) / 128), dim3(128), 0, s, D, (const double *)dudt,
                       (const double *)C->d_alpha, (const double *)C->d_beta, alpha_bar, C->d_diag);
    C->last = s;
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return SEDG_EHIP;
    std::vector<double> rec((size_t)R * C->nel);
    int fb = 0;
    if (hipMemcpy(rec.data(), C->d_diag, sizeof(double) * rec.size(), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(&fb, C->d_fbc, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return SEDG_EHIP;
    std::memset(out, 0, sizeof(*out));
    out->alpha_bar_min = 1e300;
    out->alpha_bar_max = -1e300;
    double asum = 0.0;
    for (int e = 0; e < C->nel; ++e) {
        const double *r = &rec[(size_t)e * R];
        for (int v = 0; v < C->nv; ++v) { out->bulk_change[v] += r[v]; out->bulk_abs[v] += r[C->nv + v]; }
        out->alpha_bar_min = r[2 * C->nv] < out->alpha_bar_min ? r[2 * C->nv] : out->alpha_bar_min;
        asum += r[2 * C->nv + 1];
        out->alpha_bar_max = r[2 * C->nv + 2] > out->alpha_bar_max ? r[2 * C->nv + 2] : out->alpha_bar_max;
        const int low = (int)r[2 * C->nv + 3];
        out->elems_by_lowest_order[low == 1 ? 0 : low == 2 ? 1 : low == 4 ? 2 : 3] += 1;
        out->squeezed += (long)r[2 * C->nv + 4];
        out->beta_rejected += (long)r[2 * C->nv + 5];
    }
    out->alpha_bar_mean = asum / (double)C->dof;
    out->fallbacks = fb;
    return SEDG_OK;
}

int sedg_rk_step_frozen(sedg_ctx *C, double *u, int nsteps, const double *dt_dev, const double *factors, void *stream)
{
    if (C && C->params.integrator != SEDG_SSPRK3) return SEDG_EUNSUPPORTED;
    if (!C || !u || nsteps < 0 || (nsteps > 0 && (!dt_dev || !factors))) return SEDG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const long long na = (long long)C->A * C->nel;
    double *stage_in[3] = {u, C->d_u1, C->d_u2};
    double *stage_out[3] = {C->d_u1, C->d_u2, u};
    for (int j = 0; j < nsteps; ++j) {
        const double *f = factors + (long long)j * 6 * na;
        KArgs P = base_args(C);
        P.dt = dt_dev + j;
        for (int k = 0; k < 3; ++k) {
            P.u = stage_in[k];
            P.u0 = u;
            P.out = stage_out[k];
            P.alpha = const_cast<double *>(f + k * na);
            P.beta = const_cast<double *>(f + (3 + k) * na);
            P.stage = k + 1;
            launch_prep_any(C, P, s);
            launch_residual_any(C, P, s);
        }
    }
    C->last = s;
    return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// frozen map and adjoint
// ---------------------------------------------------------------------------

extern "C" {

int sedg_rhs_frozen(sedg_ctx *C, const double *u, const double *alpha, const double *beta, double *dudt, void *stream)
{
    if (!C || !u || !alpha || !beta || !dudt || u == dudt) return SEDG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    KArgs P = base_args(C);
    P.u = u;
    P.out = dudt;
    P.alpha = const_cast<double *>(alpha);
    P.beta = const_cast<double *>(beta);
    P.stage = 0;
    launch_prep_any(C, P, s);
    launch_residual_any(C, P, s);
    C->last = s;
    return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
}

int sedg_adjoint_rhs(sedg_ctx *C, const double *u, const double *alpha, const double *beta, const double *lam,
                     double *lam_out, void *stream)
{
    if (!C || !u || !alpha || !beta || !lam || !lam_out || lam == lam_out || u == lam_out) return SEDG_EINVAL;
    if (!adjoint_supported(C)) return SEDG_EUNSUPPORTED;
    int rc = ensure_adjoint_buffers(C);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    KArgs P = base_args(C);
    P.u = u;
    P.lam = lam;
    P.out = lam_out;
    P.alpha = const_cast<double *>(alpha);
    P.beta = const_cast<double *>(beta);
    P.gfb = C->d_gfb;
    P.gsb = C->d_gsb;
    P.gdb = C->d_gdb;
    P.stage = 0;
    launch_prep_any(C, P, s);
    launch_eface_adjoint_any(C, P, s);
    launch_adjoint_any(C, P, s);
    C->last = s;
    return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
}

long sedg_tape_len(const sedg_ctx *C)
{
    if (!C) return SEDG_EINVAL;
    long kf = 1;
    for (int a = 1; a < C->mesh.dim; ++a) kf *= C->mesh.K;
    const long nfb = (long)C->nel * C->mesh.dim * 2 * C->nv * kf;
    return 3L * C->nv * C->dof + 6L * C->A * C->nel + 3L * (nfb + (long)C->nel * C->nv * C->A + 2L * C->nel);
}

}  // extern "C"

namespace {

// one step's tape: [u^n | u^(1) | u^(2) | alpha x 3 | beta x 3 | face states x 3 |
// sub-element means x 3 | element scales x 3] (the last three as the analyse kernel
// writes them, so that a transposed stage needs no second analysis)
struct Tape {
    double *u[3], *alpha[3], *beta[3], *fbuf[3], *mean[3], *scale[3];
};

Tape tape_view(const sedg_ctx *C, double *tape)
{
    Tape T;
    const long ns = (long)C->nv * C->dof, na = (long)C->A * C->nel;
    long kf = 1;
    for (int a = 1; a < C->mesh.dim; ++a) kf *= C->mesh.K;
    const long nfb = (long)C->nel * C->mesh.dim * 2 * C->nv * kf, nmn = (long)C->nel * C->nv * C->A,
               nsc = 2L * C->nel;
    double *q = tape + 3 * ns + 6 * na;
    for (int k = 0; k < 3; ++k) {
        T.u[k] = tape + k * ns;
        T.alpha[k] = tape + 3 * ns + k * na;
        T.beta[k] = tape + 3 * ns + (3 + k) * na;
        T.fbuf[k] = q + k * nfb;
        T.mean[k] = q + 3 * nfb + k * nmn;
        T.scale[k] = q + 3 * nfb + 3 * nmn + k * nsc;
    }
    return T;
}

}  // namespace

extern "C" {

int sedg_rk_step_tape(sedg_ctx *C, double *u, int nsteps, const double *dt_dev, double *tapes, void *stream)
{
    if (C && C->params.integrator != SEDG_SSPRK3) return SEDG_EUNSUPPORTED;
    if (!C || !u || nsteps < 0 || (nsteps > 0 && (!dt_dev || !tapes))) return SEDG_EINVAL;
    if (C->params.mode == SEDG_EXTERNAL) return SEDG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const long tl = sedg_tape_len(C);
    for (int j = 0; j < nsteps; ++j) {
        Tape T = tape_view(C, tapes + (size_t)j * tl);
        if (hipMemcpyAsync(T.u[0], u, sizeof(double) * (size_t)C->nv * C->dof, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return SEDG_EHIP;
        KArgs P = base_args(C);
        P.dt = dt_dev + j;
        // the three stages of one step, as in sedg_rk_step, with the stage states and the
        // blending factors and squeezing parameters of every stage kept on the tape
        P.u = u;
        P.out = T.u[1];
        P.alpha = T.alpha[0];
        P.beta = T.beta[0];
        P.fbuf = T.fbuf[0];
        P.mean = T.mean[0];
        P.scale = T.scale[0];
        P.stage = 1;
        launch_analyse_any(C, P, s);
        advance_draw(C, s);
        launch_residual_any(C, P, s);
        P.u = T.u[1];
        P.u0 = u;
        P.out = T.u[2];
        P.alpha = T.alpha[1];
        P.beta = T.beta[1];
        P.fbuf = T.fbuf[1];
        P.mean = T.mean[1];
        P.scale = T.scale[1];
        P.stage = 2;
        launch_analyse_any(C, P, s);
        advance_draw(C, s);
        launch_residual_any(C, P, s);
        P.u = T.u[2];
        P.u0 = u;
        P.out = u;
        P.alpha = T.alpha[2];
        P.beta = T.beta[2];
        P.fbuf = T.fbuf[2];
        P.mean = T.mean[2];
        P.scale = T.scale[2];
        P.stage = 3;
        launch_analyse_any(C, P, s);
        advance_draw(C, s);
        launch_residual_any(C, P, s);
    }
    C->last = s;
    return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
}

int sedg_adjoint_rk_step(sedg_ctx *C, const double *tapes, int nsteps, const double *dt_dev, double *lam, void *stream)
{
    if (C && C->params.integrator != SEDG_SSPRK3) return SEDG_EUNSUPPORTED;
    if (!C || !lam || nsteps < 0 || (nsteps > 0 && (!tapes || !dt_dev))) return SEDG_EINVAL;
    if (!adjoint_supported(C)) return SEDG_EUNSUPPORTED;
    int rc = ensure_adjoint_buffers(C);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const long tl = sedg_tape_len(C);
    for (int j = nsteps - 1; j >= 0; --j) {
        Tape T = tape_view(C, const_cast<double *>(tapes) + (size_t)j * tl);
        KArgs P = base_args(C);
        P.dt = dt_dev + j;
        P.gfb = C->d_gfb;
        P.gsb = C->d_gsb;
        P.gdb = C->d_gdb;
        P.acc = C->d_acc;
        const double *lin[3] = {C->d_l1, C->d_l2, lam};   // adjoint entering reverse stage 1, 2, 3
        double *lout[3] = {lam, C->d_l1, C->d_l2};
        for (int st = 2; st >= 0; --st) {
            P.u = T.u[st];
            P.alpha = T.alpha[st];
            P.beta = T.beta[st];
            P.fbuf = T.fbuf[st];
            P.mean = T.mean[st];
            P.scale = T.scale[st];
            P.lam = lin[st];
            P.out = lout[st];
            P.stage = 11 + st;
            launch_face_adjoint_any(C, P, s);
            launch_eface_adjoint_any(C, P, s);
            launch_adjoint_any(C, P, s);
        }
    }
    C->last = s;
    return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched ensembles: host side
// ---------------------------------------------------------------------------

struct sedg_batch {
    int nprob;
    sedg_params params;
    double gamma;
    int family;
    int ncu;
    std::vector<sedg_mesh> meshes;
    std::vector<ProbDesc> probs;
    long long state_len, alpha_len, fbuf_len, nel;
    sedg_batch_tuning tun;
    int ntiles, ntiles4, grid, chunk, nftiles;   // ntiles4: the K = 4 tiles, numbered first
    sedg_level_tab *d_tabs;
    ProbDesc *d_probs;
    int *d_tile_prob, *d_ftile_prob;
    double *d_alpha, *d_beta, *d_mean, *d_scale, *d_fbuf, *d_ef, *d_u1, *d_u2, *d_dt, *d_lam;
    double *d_u3;            // SSP-RK(5,4): the fourth stage state (allocated on first use)
    int *d_err, *d_ctr;
    hipStream_t last;
    std::map<std::tuple<double *, double *, int>, hipGraphExec_t> graphs;
};

namespace {

void batch_drop_graphs(sedg_batch *B)
{
    for (auto &kv : B->graphs) (void)hipGraphExecDestroy(kv.second);
    B->graphs.clear();
}

// tiles of every problem for the current elements-per-workgroup choice, and the grid
int batch_layout(sedg_batch *B)
{
    // the tiles of the K = 4 problems first, then those of the K = 8 problems, so that
    // one launch per K can cover each (their analyse kernels then get register
    // allocations of their own)
    std::vector<int> tp;
    int t = 0;
    for (int pass = 0; pass < 2; ++pass) {
        const int Kp = pass == 0 ? 4 : 8;
        for (int p = 0; p < B->nprob; ++p) {
            ProbDesc &D = B->probs[p];
            if (D.K != Kp) continue;
            const int epb = D.K == 4 ? B->tun.epb4 : B->tun.epb8;
            D.tile_off = t;
            D.ntiles = (D.nel + epb - 1) / epb;
            t += D.ntiles;
            for (int i = 0; i < D.ntiles; ++i) tp.push_back(p);
        }
        if (pass == 0) B->ntiles4 = t;
    }
    B->ntiles = t;
    // element-face tiles: 64 / K tasks (element, axis) each
    std::vector<int> ftp;
    int ft = 0;
    for (int p = 0; p < B->nprob; ++p) {
        ProbDesc &D = B->probs[p];
        const int ns = 64 / D.K;
        D.ftile_off = ft;
        const int n = (2 * D.nel + ns - 1) / ns;
        ft += n;
        for (int i = 0; i < n; ++i) ftp.push_back(p);
    }
    B->nftiles = ft;
    if (B->tun.blocks_per_cu > 0) {
        long long g = (long long)B->ncu * B->tun.blocks_per_cu;
        B->grid = (int)(g < t ? g : t);
    } else {
        B->grid = t;
    }
    B->chunk = (t + B->grid - 1) / B->grid;
    if (B->d_tile_prob) (void)hipFree(B->d_tile_prob);
    B->d_tile_prob = nullptr;
    if (hipMalloc(&B->d_tile_prob, sizeof(int) * (size_t)t) != hipSuccess) return SEDG_ENOMEM;
    if (hipMemcpy(B->d_tile_prob, tp.data(), sizeof(int) * (size_t)t, hipMemcpyHostToDevice) != hipSuccess) return SEDG_EHIP;
    if (B->d_ftile_prob) (void)hipFree(B->d_ftile_prob);
    B->d_ftile_prob = nullptr;
    if (hipMalloc(&B->d_ftile_prob, sizeof(int) * (size_t)ft) != hipSuccess) return SEDG_ENOMEM;
    if (hipMemcpy(B->d_ftile_prob, ftp.data(), sizeof(int) * (size_t)ft, hipMemcpyHostToDevice) != hipSuccess)
        return SEDG_EHIP;
    if (hipMemcpy(B->d_probs, B->probs.data(), sizeof(ProbDesc) * (size_t)B->nprob, hipMemcpyHostToDevice) != hipSuccess)
        return SEDG_EHIP;
    batch_drop_graphs(B);
    return SEDG_OK;
}

KArgs batch_args(const sedg_batch *B)
{
    KArgs P;
    std::memset(&P, 0, sizeof(P));
    P.alpha = B->d_alpha;
    P.beta = B->d_beta;
    P.mean = B->d_mean;
    P.scale = B->d_scale;
    P.fbuf = B->d_fbuf;
    P.ef = B->d_ef;
    P.tabs = (CTab *)B->d_tabs;
    P.err = B->d_err;
    P.dt = B->d_dt;
    P.probs = B->d_probs;
    P.tile_prob = B->d_tile_prob;
    P.ftile_prob = B->d_ftile_prob;
    P.ntiles = B->ntiles;
    P.chunk = B->chunk;
    P.xcd_map = B->tun.xcd_map;
    P.mode = B->params.mode;
    P.level_mask = B->params.level_mask;
    P.gamma = B->gamma;
    P.gm1 = B->gamma - 1.0;
    P.tau_A = B->params.tau_A;
    P.tau_S = B->params.tau_S;
    P.alpha_H = B->params.alpha_H;
    P.alpha_L = B->params.alpha_L;
    P.beta_L = B->params.beta_L;
    P.sigma_floor = B->params.sigma_floor > 0.0 ? B->params.sigma_floor : 1.0;
    P.ind_quick = ind_quick(B->params);
    return P;
}

template <int EPB4, int EPB8, bool PERSIST>
void batch_launch_t(int which, const sedg_batch *B, const KArgs &P, hipStream_t s)
{
    const dim3 grid(B->grid), block(64 * EPB8);
    const bool w4 = B->tun.waves_analyse == 4;
    if (which == 0 && !PERSIST) {
        // one analyse launch per K over its own tiles
        const int n4 = B->ntiles4, n8 = B->ntiles - B->ntiles4;
        KArgs Q = P;
        if (n4 > 0) {
            Q.tile_base = 0;
            if (w4) hipLaunchKernelGGL((analyse_batch_one_kernel<4, EPB4, 4>), dim3(n4), block, 0, s, Q);
            else hipLaunchKernelGGL((analyse_batch_one_kernel<4, EPB4, 3>), dim3(n4), block, 0, s, Q);
        }
        if (n8 > 0) {
            Q.tile_base = n4;
            if (w4) hipLaunchKernelGGL((analyse_batch_one_kernel<8, EPB8, 4>), dim3(n8), block, 0, s, Q);
            else hipLaunchKernelGGL((analyse_batch_one_kernel<8, EPB8, 3>), dim3(n8), block, 0, s, Q);
        }
    } else if (which == 0) {
        // persistent grid: one launch for both K
        if constexpr (PERSIST) {
            if (w4) hipLaunchKernelGGL((analyse_batch_kernel<EPB4, EPB8, PERSIST, 4>), grid, block, 0, s, P);
            else hipLaunchKernelGGL((analyse_batch_kernel<EPB4, EPB8, PERSIST, 3>), grid, block, 0, s, P);
        }
    } else {
        // the residual reads the element-face fluxes of the face kernel launched before it
        hipLaunchKernelGGL(eface_batch_kernel, dim3(B->nftiles), dim3(64), 0, s, P);
        hipLaunchKernelGGL((residual_batch_kernel<EPB4, EPB8, PERSIST>), grid, block, 0, s, P);
    }
}

void batch_launch(int which, const sedg_batch *B, const KArgs &P, hipStream_t s)
{
    const bool persist = B->tun.blocks_per_cu > 0;
    if (B->tun.epb8 == 2) {
        if (persist) batch_launch_t<8, 2, true>(which, B, P, s);
        else batch_launch_t<8, 2, false>(which, B, P, s);
    } else {
        if (persist) batch_launch_t<4, 1, true>(which, B, P, s);
        else batch_launch_t<4, 1, false>(which, B, P, s);
    }
}

void enqueue_batch_step(sedg_batch *B, double *u, bool fixed, double *dt_log, hipStream_t s)
{
    KArgs P = batch_args(B);
    P.u = u;
    P.out = B->d_u1;
    P.stage = 1;
    P.lam_part = fixed ? nullptr : B->d_lam;
    batch_launch(0, B, P, s);
    if (!fixed)
        hipLaunchKernelGGL(finalize_batch_kernel, dim3(B->nprob), dim3(BATCH_SLOTS), 0, s, B->d_lam,
                           (const ProbDesc *)B->d_probs, B->nprob, B->d_dt, dt_log, (const int *)B->d_ctr);
    batch_launch(1, B, P, s);
    P.lam_part = nullptr;
    P.u = B->d_u1;
    P.u0 = u;
    P.out = B->d_u2;
    P.stage = 2;
    batch_launch(0, B, P, s);
    batch_launch(1, B, P, s);
    P.u = B->d_u2;
    P.u0 = u;
    P.out = u;
    P.stage = 3;
    batch_launch(0, B, P, s);
    batch_launch(1, B, P, s);
    if (dt_log && !fixed) hipLaunchKernelGGL(count_step_kernel, dim3(1), dim3(64), 0, s, B->d_ctr);
}

// SSP-RK(5,4) of the ensemble: the stages and buffers of the single-problem form
// (enqueue_step_rk54), one analyse / element-face / residual launch each for the whole
// ensemble
void enqueue_batch_step_rk54(sedg_batch *B, double *u, bool fixed, double *dt_log, hipStream_t s)
{
    KArgs P = batch_args(B);
    auto set = [&](const double *r) { for (int k = 0; k < 7; ++k) P.rk[k] = r[k]; };
    P.stage = 5;
    P.u = u;
    P.u0 = P.x1 = P.y0 = nullptr;
    P.yout = nullptr;
    P.out = B->d_u1;
    const double r1[7] = {0.0, 1.0, RK54_C10, 0.0, 0.0, 0.0, 0.0};
    set(r1);
    P.lam_part = fixed ? nullptr : B->d_lam;
    batch_launch(0, B, P, s);
    if (!fixed)
        hipLaunchKernelGGL(finalize_batch_kernel, dim3(B->nprob), dim3(BATCH_SLOTS), 0, s, B->d_lam,
                           (const ProbDesc *)B->d_probs, B->nprob, B->d_dt, dt_log, (const int *)B->d_ctr);
    batch_launch(1, B, P, s);
    P.lam_part = nullptr;
    struct { double *in, *out; const double *u0, *x1, *y0; double *yout; double r[7]; } st[4] = {
        {B->d_u1, B->d_u2, u, nullptr, nullptr, nullptr, {RK54_A20, RK54_A21, RK54_C21, 0, 0, 0, 0}},
        {B->d_u2, B->d_u1, u, nullptr, nullptr, nullptr, {RK54_A30, RK54_A32, RK54_C32, 0, 0, 0, 0}},
        {B->d_u1, B->d_u3, u, nullptr, B->d_u2, B->d_u2, {RK54_A40, RK54_A43, RK54_C43, 0, RK54_A52, RK54_A53, RK54_C53}},
        {B->d_u3, u, nullptr, B->d_u2, nullptr, nullptr, {0, RK54_A54, RK54_C54, 1.0, 0, 0, 0}},
    };
    for (int k = 0; k < 4; ++k) {
        P.u = st[k].in;
        P.out = st[k].out;
        P.u0 = st[k].u0;
        P.x1 = st[k].x1;
        P.y0 = st[k].y0;
        P.yout = st[k].yout;
        set(st[k].r);
        batch_launch(0, B, P, s);
        batch_launch(1, B, P, s);
    }
    if (dt_log && !fixed) hipLaunchKernelGGL(count_step_kernel, dim3(1), dim3(64), 0, s, B->d_ctr);
}

}  // namespace

extern "C" {

int sedg_batch_destroy(sedg_batch *B)
{
    if (!B) return SEDG_OK;
    (void)hipDeviceSynchronize();
    batch_drop_graphs(B);
    void *ptrs[] = {B->d_tabs, B->d_probs, B->d_tile_prob, B->d_ftile_prob, B->d_alpha, B->d_beta, B->d_mean,
                    B->d_scale, B->d_fbuf, B->d_ef, B->d_u1, B->d_u2, B->d_u3, B->d_dt, B->d_lam, B->d_err, B->d_ctr};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete B;
    return SEDG_OK;
}

int sedg_batch_create(const sedg_mesh *meshes, int count, const sedg_params *params, sedg_batch **out)
{
    if (!meshes || count < 1 || !params || !out) return SEDG_EINVAL;
    *out = nullptr;
    if (params->top_level != 0 || params->mode == SEDG_EXTERNAL || params->mode < 0 || params->mode > 3 ||
        (params->integrator != SEDG_SSPRK3 && params->integrator != SEDG_SSPRK54))
        return SEDG_EINVAL;
    for (int p = 0; p < count; ++p) {
        const sedg_mesh &m = meshes[p];
        if (m.dim != 2) return SEDG_EUNSUPPORTED;
        if (m.K != 4 && m.K != 8) return SEDG_EUNSUPPORTED;
        if (m.gamma != meshes[0].gamma || m.family != meshes[0].family) return SEDG_EINVAL;
        if (!(m.gamma > 1.0) || (m.family != SEDG_GAUSS && m.family != SEDG_LGL)) return SEDG_EINVAL;
        for (int a = 0; a < 2; ++a) {
            if (m.nelem[a] < 1 || !(m.hi[a] > m.lo[a])) return SEDG_EINVAL;
            if (m.bc[a] != SEDG_PERIODIC && m.bc[a] != SEDG_OUTFLOW) return SEDG_EINVAL;
        }
        if (!mesh_extent_ok(2, m.K, m.nelem)) return SEDG_EINVAL;
    }
    sedg_batch *B = new sedg_batch();
    B->nprob = count;
    B->params = *params;
    B->gamma = meshes[0].gamma;
    B->family = meshes[0].family;
    B->meshes.assign(meshes, meshes + count);
    B->tun.epb4 = 4;
    B->tun.epb8 = 1;
    B->tun.blocks_per_cu = 0;
    B->tun.xcd_map = 1;
    B->tun.waves_analyse = 3;
    B->tun.waves_residual = 3;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) { delete B; return SEDG_EHIP; }
    B->ncu = prop.multiProcessorCount;
    long long so = 0, ao = 0, fo = 0, eo = 0;
    for (int p = 0; p < count; ++p) {
        const sedg_mesh &m = meshes[p];
        ProbDesc D;
        std::memset(&D, 0, sizeof(D));
        D.K = m.K;
        D.nel = m.nelem[0] * m.nelem[1];
        D.dof = (long long)D.nel * m.K * m.K;
        D.state_off = so;
        D.alpha_off = ao;
        D.fbuf_off = fo;
        D.elem_off = eo;
        const int A = m.K == 8 ? 21 : 5;
        for (int a = 0; a < 2; ++a) {
            D.ne[a] = m.nelem[a];
            D.G[a] = m.nelem[a] * m.K;
            D.bc[a] = m.bc[a];
            D.dx[a] = (m.hi[a] - m.lo[a]) / m.nelem[a];
        }
        const double dxm = D.dx[0] < D.dx[1] ? D.dx[0] : D.dx[1];
        D.cfl_num = params->cfl * dxm / (2.0 * (2.0 * m.K - 1.0));
        so += 4 * D.dof;
        ao += (long long)D.nel * A;
        fo += (long long)D.nel * 2 * 2 * 4 * m.K;
        eo += D.nel;
        B->probs.push_back(D);
    }
    if (eo > INT_MAX) { delete B; return SEDG_EINVAL; }
    B->state_len = so;
    B->alpha_len = ao;
    B->fbuf_len = fo;
    B->nel = eo;
    bool ok = true;
    ok = ok && hipMalloc(&B->d_tabs, sizeof(sedg_level_tab) * MAXLEV) == hipSuccess;
    ok = ok && hipMalloc(&B->d_probs, sizeof(ProbDesc) * (size_t)count) == hipSuccess;
    ok = ok && hipMalloc(&B->d_alpha, sizeof(double) * (size_t)ao) == hipSuccess;
    ok = ok && hipMalloc(&B->d_beta, sizeof(double) * (size_t)ao) == hipSuccess;
    ok = ok && hipMalloc(&B->d_mean, sizeof(double) * 4 * (size_t)ao) == hipSuccess;
    ok = ok && hipMalloc(&B->d_scale, sizeof(double) * 2 * (size_t)eo) == hipSuccess;
    ok = ok && hipMalloc(&B->d_fbuf, sizeof(double) * (size_t)fo) == hipSuccess;
    ok = ok && hipMalloc(&B->d_ef, sizeof(double) * (size_t)fo) == hipSuccess;
    ok = ok && hipMalloc(&B->d_u1, sizeof(double) * (size_t)so) == hipSuccess;
    ok = ok && hipMalloc(&B->d_u2, sizeof(double) * (size_t)so) == hipSuccess;
    ok = ok && hipMalloc(&B->d_dt, sizeof(double) * (size_t)count) == hipSuccess;
    ok = ok && hipMalloc(&B->d_lam, sizeof(double) * BATCH_SLOTS * (size_t)count) == hipSuccess;
    ok = ok && hipMalloc(&B->d_err, sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc(&B->d_ctr, sizeof(int)) == hipSuccess;
    if (!ok) { sedg_batch_destroy(B); return SEDG_ENOMEM; }
    sedg_level_tab h[MAXLEV];
    std::memset(h, 0, sizeof(h));
    for (int li = 0; li < 3; ++li)
        if (sedg_build_level(8 >> li, B->family, &h[li])) { sedg_batch_destroy(B); return SEDG_EINVAL; }
    int big = INT_MAX;
    ok = hipMemcpy(B->d_tabs, h, sizeof(h), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(B->d_err, &big, sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemset(B->d_lam, 0, sizeof(double) * BATCH_SLOTS * (size_t)count) == hipSuccess;
    if (!ok) { sedg_batch_destroy(B); return SEDG_EHIP; }
    int rc = batch_layout(B);
    if (rc) { sedg_batch_destroy(B); return rc; }
    B->last = nullptr;
    *out = B;
    return SEDG_OK;
}

long sedg_batch_state_len(const sedg_batch *B) { return B ? (long)B->state_len : SEDG_EINVAL; }

long sedg_batch_state_offset(const sedg_batch *B, int p)
{
    if (!B || p < 0 || p >= B->nprob) return SEDG_EINVAL;
    return (long)B->probs[p].state_off;
}

int sedg_batch_set_tuning(sedg_batch *B, const sedg_batch_tuning *t)
{
    if (!B || !t) return SEDG_EINVAL;
    const bool shape_ok = (t->epb4 == 4 && t->epb8 == 1) || (t->epb4 == 8 && t->epb8 == 2);
    auto waves_ok = [](int w) { return w == 0 || w == 3 || w == 4; };
    if (!shape_ok || t->blocks_per_cu < 0 || t->blocks_per_cu > 64 || (t->xcd_map != 0 && t->xcd_map != 1) ||
        !waves_ok(t->waves_analyse) || !waves_ok(t->waves_residual))
        return SEDG_EINVAL;
    // the residual's 4-wave register budget is not built (it spills, measured 37 % slower)
    if (t->waves_residual == 4) return SEDG_EUNSUPPORTED;
    if (hipDeviceSynchronize() != hipSuccess) return SEDG_EHIP;
    B->tun = *t;
    if (B->tun.waves_analyse == 0) B->tun.waves_analyse = 3;
    if (B->tun.waves_residual == 0) B->tun.waves_residual = 3;
    return batch_layout(B);
}

int sedg_batch_get_tuning(const sedg_batch *B, sedg_batch_tuning *t)
{
    if (!B || !t) return SEDG_EINVAL;
    *t = B->tun;
    return SEDG_OK;
}

int sedg_batch_rk_step(sedg_batch *B, double *u, int nsteps, double dt_fixed, double *dt_log_dev, void *stream)
{
    if (!B || !u || nsteps < 0) return SEDG_EINVAL;
    if (nsteps == 0) return SEDG_OK;
    const bool rk54 = B->params.integrator == SEDG_SSPRK54;
    if (rk54 && !B->d_u3 && hipMalloc(&B->d_u3, sizeof(double) * (size_t)B->state_len) != hipSuccess) {
        B->d_u3 = nullptr;
        return SEDG_ENOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    const bool fixed = dt_fixed > 0.0;
    hipLaunchKernelGGL(set_scalars_kernel, dim3(1), dim3(64), 0, s, (double *)nullptr, 0.0, B->d_ctr);
    if (fixed)
        hipLaunchKernelGGL(fill_kernel, dim3((B->nprob + 255) / 256), dim3(256), 0, s, B->d_dt, B->nprob, dt_fixed);
    auto key = std::make_tuple(u, dt_log_dev, fixed ? 1 : 0);
    hipGraphExec_t exec = nullptr;
    auto it = B->graphs.find(key);
    if (it != B->graphs.end()) {
        exec = it->second;
    } else {
        if (B->graphs.size() >= 16) {
            if (hipStreamSynchronize(s) != hipSuccess) return SEDG_EHIP;
            batch_drop_graphs(B);
        }
        hipStream_t cs;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return SEDG_EHIP;
        hipGraph_t graph;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) { (void)hipStreamDestroy(cs); return SEDG_EHIP; }
        if (rk54) enqueue_batch_step_rk54(B, u, fixed, dt_log_dev, cs);
        else enqueue_batch_step(B, u, fixed, dt_log_dev, cs);
        if (hipStreamEndCapture(cs, &graph) != hipSuccess) { (void)hipStreamDestroy(cs); return SEDG_EHIP; }
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) return SEDG_EHIP;
        B->graphs[key] = exec;
    }
    for (int st = 0; st < nsteps; ++st)
        if (hipGraphLaunch(exec, s) != hipSuccess) return SEDG_EHIP;
    B->last = s;
    return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
}

int sedg_batch_check(sedg_batch *B, int *bad_problem, long *bad_elem)
{
    if (!B || !bad_problem || !bad_elem) return SEDG_EINVAL;
    if (hipStreamSynchronize(B->last) != hipSuccess) return SEDG_EHIP;
    int h = INT_MAX;
    if (hipMemcpy(&h, B->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SEDG_EHIP;
    *bad_problem = -1;
    *bad_elem = -1;
    if (h == INT_MAX) return SEDG_OK;
    for (int p = 0; p < B->nprob; ++p)
        if (h >= B->probs[p].elem_off && h < B->probs[p].elem_off + B->probs[p].nel) {
            *bad_problem = p;
            *bad_elem = (long)(h - B->probs[p].elem_off);
        }
    int big = INT_MAX;
    if (hipMemcpy(B->d_err, &big, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return SEDG_EHIP;
    return SEDG_ESTATE;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// right-hand side without device allocation
// ---------------------------------------------------------------------------
// Every buffer beyond the caller's input and output lives in one file-scope device
// array: the operator tables of both node families (levels 8, 4, 2 each), the error
// flag and the per-element work arrays of one right-hand side (factors, squeezing
// parameters, sub-element means, face states, element-face fluxes, data scales).
// Each device the library runs on holds its own copy for the lifetime of the process.

#define SEDG_SCRATCH_BYTES (64ull << 20)
#define SEDG_MAX_DEVICES 64

static __device__ __align__(256) unsigned char scratch[SEDG_SCRATCH_BYTES];

namespace {

// byte offsets inside the scratch array
constexpr size_t NA_TABS = 0;                                            // 2 families x levels 8, 4, 2
constexpr size_t NA_ERR = ((2 * 3 * sizeof(sedg_level_tab) + 255) / 256) * 256;
constexpr size_t NA_WORK = NA_ERR + 256;

std::mutex na_mu;
unsigned char *na_ptr[SEDG_MAX_DEVICES];   // device address of each device's scratch

// set-up on the current device, once: the device address of its scratch array and the
// operator tables copied into it (a synchronous copy; the first call on a device must
// therefore not be made under stream capture)
int na_setup(int dev, unsigned char **out)
{
    std::lock_guard<std::mutex> lk(na_mu);
    if (na_ptr[dev]) { *out = na_ptr[dev]; return SEDG_OK; }
    unsigned char *ptr = nullptr;
    if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SEDG_EHIP;
    sedg_level_tab h[6];
    std::memset(h, 0, sizeof(h));
    for (int fam = 0; fam < 2; ++fam)
        for (int li = 0; li < 3; ++li)
            if (sedg_build_level(8 >> li, fam, &h[3 * fam + li])) return SEDG_EINVAL;
    if (hipMemcpy(ptr + NA_TABS, h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return SEDG_EHIP;
    na_ptr[dev] = ptr;
    *out = ptr;
    return SEDG_OK;
}

__global__ void na_set_int_kernel(int *x, int v)
{
    if (threadIdx.x == 0) x[0] = v;
}

__global__ void na_copy_int_kernel(const int *src, int *dst)
{
    if (threadIdx.x == 0) dst[0] = src[0];
}

}  // namespace

extern "C" {

int sedg_rhs_noalloc(const sedg_mesh *mesh, const sedg_params *params, const double *u, double *dudt, int *bad_dev,
                     void *stream)
{
    if (!mesh || !params || !u || !dudt || u == dudt) return SEDG_EINVAL;
    if (!supported(mesh->dim, mesh->K)) return SEDG_EUNSUPPORTED;
    if (!(mesh->gamma > 1.0) || (mesh->family != SEDG_GAUSS && mesh->family != SEDG_LGL)) return SEDG_EINVAL;
    if (params->mode != SEDG_ADAPTIVE && params->mode != SEDG_FORCE_DG && params->mode != SEDG_FORCE_FV)
        return SEDG_EINVAL;
    const int d = mesh->dim, K = mesh->K, nv = d + 2;
    const int top = params->top_level > 0 ? params->top_level : K;
    if (top < 2 || top > K || (top & (top - 1))) return SEDG_EINVAL;
    if (!mesh_extent_ok(d, K, mesh->nelem)) return SEDG_EINVAL;
    // geometry, as sedg_create validates it
    KArgs P;
    std::memset(&P, 0, sizeof(P));
    long long nel = 1, dof = 1;
    for (int a = 0; a < 3; ++a) {
        if (a < d) {
            if (mesh->nelem[a] < 1 || !(mesh->hi[a] > mesh->lo[a])) return SEDG_EINVAL;
            if (mesh->bc[a] != SEDG_PERIODIC && mesh->bc[a] != SEDG_OUTFLOW) return SEDG_EINVAL;
            P.ne[a] = mesh->nelem[a];
            P.G[a] = mesh->nelem[a] * K;
            P.bc[a] = mesh->bc[a];
            P.dx[a] = (mesh->hi[a] - mesh->lo[a]) / mesh->nelem[a];
        } else {
            P.ne[a] = 1;
            P.G[a] = 1;
            P.bc[a] = SEDG_PERIODIC;
            P.dx[a] = 1.0;
        }
        nel *= P.ne[a];
        dof *= P.G[a];
    }
    // level hierarchy and per-element work sizes
    int off = 0;
    for (int n = top; n >= 2; n /= 2) {
        int li = P.nlev++;
        P.lev_n[li] = n;
        P.lev_off[li] = off;
        int per = 1;
        for (int a = 0; a < d; ++a) per *= K / n;
        off += per;
    }
    for (int li = P.nlev; li < MAXLEV; ++li) { P.lev_n[li] = 2; P.lev_off[li] = 0; }
    P.A = off;
    long long kf = 1;
    for (int a = 1; a < d; ++a) kf *= K;
    const long long nfb = (long long)d * 2 * nv * kf;
    const long long per_el = 2LL * P.A + (long long)nv * P.A + 2 * nfb + 2;
    if (nel > INT_MAX / 8 || per_el * nel * (long long)sizeof(double) > (long long)(SEDG_SCRATCH_BYTES - NA_WORK))
        return SEDG_ESCRATCH;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SEDG_EHIP;
    if (dev < 0 || dev >= SEDG_MAX_DEVICES) return SEDG_EUNSUPPORTED;
    unsigned char *base = nullptr;
    int rc = na_setup(dev, &base);
    if (rc) return rc;

    double *w = (double *)(base + NA_WORK);
    P.alpha = w;
    P.beta = P.alpha + nel * P.A;
    P.mean = P.beta + nel * P.A;
    P.fbuf = P.mean + nel * nv * P.A;
    P.ef = P.fbuf + nel * nfb;
    P.scale = P.ef + nel * nfb;
    int li_top = top == 8 ? 0 : top == 4 ? 1 : 2;
    P.tabs = (CTab *)((sedg_level_tab *)(base + NA_TABS) + 3 * mesh->family + li_top);
    P.err = (int *)(base + NA_ERR);
    P.lam_mask = LAM_SLOTS - 1;
    P.dof = dof;
    P.nel = (int)nel;
    P.mode = params->mode;
    P.level_mask = params->level_mask;
    P.gamma = mesh->gamma;
    P.gm1 = mesh->gamma - 1.0;
    P.tau_A = params->tau_A;
    P.tau_S = params->tau_S;
    P.alpha_H = params->alpha_H;
    P.alpha_L = params->alpha_L;
    P.beta_L = params->beta_L;
    P.sigma_floor = params->sigma_floor > 0.0 ? params->sigma_floor : 1.0;
    P.ind_quick = ind_quick(*params);
    P.u = u;
    P.out = dudt;
    P.stage = 0;

    hipStream_t s = (hipStream_t)stream;
    const int epb = epb_for(d, K);
    const int nblocks = (int)((nel + epb - 1) / epb);
    hipLaunchKernelGGL(na_set_int_kernel, dim3(1), dim3(64), 0, s, P.err, INT_MAX);
    launch_shape(0, d, K, top, nblocks, P, s);
    launch_shape(6, d, K, top, nblocks, P, s);
    launch_shape(1, d, K, top, nblocks, P, s);
    if (bad_dev) hipLaunchKernelGGL(na_copy_int_kernel, dim3(1), dim3(64), 0, s, P.err, bad_dev);
    return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// refinement / coarsening entry points
// ---------------------------------------------------------------------------
namespace {

int ensure_nc(sedg_ctx *C)
{
    if (C->d_nc) return SEDG_OK;
    sedg_nc_tab hn[MAXLEV];
    std::memset(hn, 0, sizeof(hn));
    for (int li = 0; li < C->nlev; ++li)
        if (sedg_build_nc(C->lev_n[li], C->mesh.family, &hn[li])) return SEDG_EINVAL;
    if (hipMalloc(&C->d_nc, sizeof(hn)) != hipSuccess) { C->d_nc = nullptr; return SEDG_ENOMEM; }
    if (hipMemcpy(C->d_nc, hn, sizeof(hn), hipMemcpyHostToDevice) != hipSuccess) return SEDG_EHIP;
    return SEDG_OK;
}

template <int DIM, int K, int TOP>
void rc_launch(bool refine, const RcArgs &A, int nel, hipStream_t s)
{
    if (refine) hipLaunchKernelGGL((refine_kernel<DIM, K, TOP>), dim3(nel), dim3(Geo<DIM, K>::KD), 0, s, A);
    else hipLaunchKernelGGL((coarsen_kernel<DIM, K, TOP>), dim3(nel), dim3(Geo<DIM, K>::KD), 0, s, A);
}

template <int DIM, int K>
void rc_launch_top(bool refine, int top, const RcArgs &A, int nel, hipStream_t s)
{
    if (top == 2) rc_launch<DIM, K, 2>(refine, A, nel, s);
    else if (top == 4) rc_launch<DIM, K, 4>(refine, A, nel, s);
    else rc_launch<DIM, K, (K >= 8 ? 8 : 4)>(refine, A, nel, s);
}

int refine_or_coarsen(sedg_ctx *C, bool refine, const double *in, const double *alpha, double *out, void *stream)
{
    if (!C || !in || !alpha || !out || in == out) return SEDG_EINVAL;
    int rc = ensure_nc(C);
    if (rc) return rc;
    RcArgs A;
    std::memset(&A, 0, sizeof(A));
    A.in = in;
    A.alpha = alpha;
    A.out = out;
    A.tabs = (CTab *)C->d_tabs;
    A.nc = (CNc *)C->d_nc;
    A.dof_c = C->dof;
    A.dof_f = C->dof;
    for (int a = 0; a < 3; ++a) {
        A.ne[a] = C->mesh.nelem[a];
        A.Gc[a] = C->G[a];
        A.Gf[a] = a < C->mesh.dim ? 2 * C->G[a] : 1;
        if (a < C->mesh.dim) A.dof_f *= 2;
    }
    hipStream_t s = (hipStream_t)stream;
    const int d = C->mesh.dim, K = C->mesh.K, top = C->lev_n[0];
    if (d == 2 && K == 4) rc_launch_top<2, 4>(refine, top, A, C->nel, s);
    else if (d == 2 && K == 8) rc_launch_top<2, 8>(refine, top, A, C->nel, s);
    else if (d == 3 && K == 4) rc_launch_top<3, 4>(refine, top, A, C->nel, s);
    else rc_launch_top<3, 8>(refine, top, A, C->nel, s);
    C->last = s;
    return hipGetLastError() == hipSuccess ? SEDG_OK : SEDG_EHIP;
}

}  // namespace

extern "C" {

int sedg_refine(sedg_ctx *C, const double *u, const double *alpha, double *u_fine, void *stream)
{
    return refine_or_coarsen(C, true, u, alpha, u_fine, stream);
}

int sedg_coarsen(sedg_ctx *C, const double *u_fine, const double *alpha_fine, double *u, void *stream)
{
    return refine_or_coarsen(C, false, u_fine, alpha_fine, u, stream);
}

}  // extern "C"
