// HIP kernels (gfx950, wave64) for the thermal LBM with PML and open boundaries, compiled once
// per velocity stencil: LBM_Q = 37 (default; this file) or 17 (lbm_kernels_d2q17.hip), each
// instance in its own namespace (k37, k17) with its stencil's constants in scope.
//
// Every kernel takes an array of run descriptors, so one launch advances one run or a batch of
// uneven runs.  Per step:
//   k_target       (runs with the appendix's PML moments or a CBC (A) side) float64
//                  characteristic targets of the ring
//   k_phase_a      ring blocks: float64 characteristic fill of the 3-deep ring of
//                  characteristic-boundary nodes into G (eqs. PNR / thermal_LODI_macro_evo);
//                  then for the PML Q-region nodes: pull (ring: G) + moments,
//                  Q^{n+1} = Q^n + (fhat^n + fhat^{n+1})/2                      (eq. PMLQ)
//   k_frame        frame nodes (boundary layers, PML, moment strips): pull (ring nodes: G) +
//                  ZG copy, moments, U^{n+1} strip write, BGK + Omega^PML
//                                                             (eqs. PMLCOLL, zg-bc)
//   k_bulk         interior nodes: branch-free pull + moments + BGK             (eq. lbe)
//   k_advance      end of a batch of steps: advance the step counters and buffer parities
//                  (the step kernels of sub-step k of a batch use parity par + k)
// The ring blocks come first in their launches (their float64 chains are the longest) and are
// block-uniform, so they never share a wave with frame nodes.  (A separate ring launch lowers
// phase A's registers but measured slower: the ring's latency then adds instead of overlapping.)
// The collision is a per-node projection streaming 2 x q values
// through HBM: no MFMA.  Pulls are coalesced row segments shifted by e_i (each source value is
// read exactly once); descriptors are read through the constant address space (scalar
// loads) and populations through global pointers with one 32-bit byte offset per lane.
//
// Arithmetic is in deviation form: the stored populations are d_i = f_i - fbar_i with
// fbar = feq(rho0, u0, T0), and the equilibrium deviation feq(U) - fbar is evaluated from
// differences of its Hermite coefficients, so float32 storage and arithmetic keep their
// relative precision on the (small) deviations.  With theta = T - 1, a = u.xi, s = |xi|^2,
// b = |u|^2, the fourth-order equilibrium of D2Q37 (eq. feq-4 with the (c^2 - 6) reading) is
//   feq_i = w_i rho H(a, s),
//   H = E0(s) + E2(s) a^2 + a^4/24 + a (O1(s) + a^2/6),
//   E0 = k0 + k2s s + theta^2 s^2/8,  E2 = k2a + theta s/4,  O1 = k1 + theta s/2,
//   k0 = 1 - b/2 - theta + b^2/8 + theta b + theta^2,  k1 = 1 - b/2 - 2 theta,
//   k2a = 1/2 - b/4 - 3 theta/2,  k2s = theta/2 - theta b/4 - theta^2,
// and the third-order equilibrium of D2Q17 (eq. feq-3) drops the fourth-order Hermite term:
//   H = E0(s) + a^2/2 + a (O1(s) + a^2/6),  E0 = k0 + theta s/2,  k0 = 1 - b/2 - theta,
// with O1 and k1 as above; feq(U) - fbar = w (drho H0 + rho dH) with dH = H(U) - H(U0)
// expanded in products of deviations.
#include <type_traits>
#include <utility>

#include <hip/hip_ext.h>

#include "lbm_internal.h"

#define GLOBAL __attribute__((address_space(1)))
#define CONSTANT __attribute__((address_space(4)))

#ifndef LBM_Q
#define LBM_Q 37
#endif
#if LBM_Q == 37
#define LBM_LATTICE d2q37
#define LBM_KSET k37
#elif LBM_Q == 17
#define LBM_LATTICE d2q17
#define LBM_KSET k17
#elif LBM_Q == 9
#define LBM_LATTICE d2q9
#define LBM_KSET k9
#else
#error "LBM_Q must be 37, 17 or 9"
#endif

namespace lbm {
namespace LBM_KSET {

using namespace ::lbm::LBM_LATTICE;
using CRun = const CONSTANT RunDev;

// Index guard of the bounds-checked debug build (compiled with LBM_BOUNDS): an element index i
// outside [0, n) marks the run's descriptor (a vector atomic) and is replaced by 0, so the access
// stays inside its buffer and lbm_check reports the run.  The normal build uses i unchanged.
#ifdef LBM_BOUNDS
__device__ __forceinline__ long long guard(CRun &R, long long i, long long n) {
    if ((unsigned long long)i < (unsigned long long)n) return i;
    GLOBAL unsigned *flag = (GLOBAL unsigned *)(uintptr_t)&R.oob;   // the descriptor, written as global memory
    __hip_atomic_fetch_or(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0;
}
#define LBM_GUARD(R, i, n) guard((R), (i), (n))
// element `off` bytes past base, inside buffer buf of n elements
#define LBM_AT(R, base, off, buf, n) \
    ((buf) + guard((R), ((base) - (buf)) + (long long)((off) / sizeof(*(buf))), (n)))
#else
#define LBM_GUARD(R, i, n) (i)
#define LBM_AT(R, base, off, buf, n) at((base), (off))
#endif

// ------------------------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------------------------
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

template <class S> struct Traits;
template <> struct Traits<double> { using C = double; };
template <> struct Traits<float> { using C = float; };
template <> struct Traits<_Float16> { using C = float; };

// element at byte offset `off` from a uniform base
template <class T>
__device__ __forceinline__ const GLOBAL T *at(const GLOBAL T *base, unsigned off) {
    return (const GLOBAL T *)((const GLOBAL char *)base + off);
}
template <class T>
__device__ __forceinline__ GLOBAL T *at(GLOBAL T *base, unsigned off) {
    return (GLOBAL T *)((GLOBAL char *)base + off);
}

__device__ __forceinline__ double cvt_in(double v, double) { return v; }
__device__ __forceinline__ float cvt_in(float v, float) { return v; }
__device__ __forceinline__ float cvt_in(_Float16 v, float inv) { return (float)v * inv; }
__device__ __forceinline__ double cvt_out(double v, double, double *) { return v; }
__device__ __forceinline__ float cvt_out(float v, float, float *) { return v; }
__device__ __forceinline__ _Float16 cvt_out(float v, float sc, _Float16 *) { return (_Float16)(v * sc); }

// Run constants in the compute type.
template <class C> struct K {
    C omega, rho0, u0x, u0y, th0, b0, r0x, r0y, c2Tb0, scale, inv_scale;
};

template <class C> __device__ __forceinline__ K<C> load_k(CRun &R) {
    K<C> k;
    if constexpr (std::is_same<C, double>::value) {
        k.omega = R.omega; k.rho0 = R.rho0; k.u0x = R.u0x; k.u0y = R.u0y; k.th0 = R.th0;
        k.b0 = R.b0; k.r0x = R.r0x; k.r0y = R.r0y; k.c2Tb0 = 2.0 * R.T0 + R.b0;
        k.scale = R.scale; k.inv_scale = R.inv_scale;
    } else {
        k.omega = R.omega_f; k.rho0 = R.rho0_f; k.u0x = R.u0x_f; k.u0y = R.u0y_f; k.th0 = R.th0_f;
        k.b0 = R.b0_f; k.r0x = R.r0x_f; k.r0y = R.r0y_f; k.c2Tb0 = 2.0f * R.T0_f + R.b0_f;
        k.scale = R.scale_f; k.inv_scale = R.inv_scale_f;
    }
    return k;
}

template <class C> __device__ __forceinline__ C cH0e(CRun &R, int p) {
    if constexpr (std::is_same<C, double>::value) return R.H0e[p]; else return R.H0e_f[p];
}
template <class C> __device__ __forceinline__ C cH0o(CRun &R, int p) {
    if constexpr (std::is_same<C, double>::value) return R.H0o[p]; else return R.H0o_f[p];
}
template <class C> __device__ __forceinline__ C cE2_0(CRun &R, int s) {
    if constexpr (std::is_same<C, double>::value) return R.E2_0[s]; else return R.E2_0_f[s];
}
template <class C> __device__ __forceinline__ C cO1_0(CRun &R, int s) {
    if constexpr (std::is_same<C, double>::value) return R.O1_0[s]; else return R.O1_0_f[s];
}
template <class C> __device__ __forceinline__ C cH0rest(CRun &R) {
    if constexpr (std::is_same<C, double>::value) return R.H0rest; else return R.H0rest_f;
}

// Blocks of one launch are dealt round-robin to the 8 XCDs; remap so that consecutive tiles
// (neighbours sharing cache lines at their edges) run on the same XCD and its L2.
__device__ __forceinline__ int xcd_swizzle(int b, int n) {
    int per = n >> 3, rem = n & 7, xcd = b & 7, loc = b >> 3;
    return xcd < rem ? xcd * (per + 1) + loc : rem * (per + 1) + (xcd - rem) * per + loc;
}

__device__ __forceinline__ int find_run(const int *prefix, int nruns, int b) {
    const CONSTANT int *p = (const CONSTANT int *)prefix;
    int lo = 0, hi = nruns;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (p[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ CRun &run_of(RunDev *const *runs, int j) {
    return *(CRun *)(((RunDev *const CONSTANT *)runs)[j]);
}

// Steps are launched in batches: sub-step k of a batch sees the run k steps past its descriptor's
// step counter, whose buffer parity is then par + k, and works only while that stays below the
// run's limit.  k_advance moves the counters at the end of the batch.  Returns the parity, or -1
// for a run that is no longer active at sub-step k.
__device__ __forceinline__ int sub_par(CRun &R, int k) {
    return R.step + k < R.limit ? ((R.par + k) & 1) : -1;
}

// Strip numbering of a frame of depths (dxm, dxp, dym, dyp): bottom strip, top strip, left
// strip, right strip.
__device__ __forceinline__ void strip_xy(int Nx, int Ny, int dxm, int dxp, int dym, int dyp, int t,
                                         int &x, int &y) {
    int Fb = dym * Nx, Ft = dyp * Nx, H = Ny - dym - dyp, Fl = H * dxm;
    if (t < Fb) { y = t / Nx; x = t - y * Nx; }
    else if (t < Fb + Ft) { t -= Fb; int r = t / Nx; y = Ny - dyp + r; x = t - r * Nx; }
    else if (t < Fb + Ft + Fl) { t -= Fb + Ft; int r = t / dxm; y = dym + r; x = t - r * dxm; }
    else { t -= Fb + Ft + Fl; int r = t / dxp; y = dym + r; x = Nx - dxp + (t - r * dxp); }
}

__device__ __forceinline__ void ring_xy(CRun &R, int t, int &x, int &y) {
    strip_xy(R.Nx, R.Ny, R.rxm, R.rxp, R.rym, R.ryp, t, x, y);
    x = (int)LBM_GUARD(R, x, R.Nx);
    y = (int)LBM_GUARD(R, y, R.Ny);
}
// Node a of the frame off the ring (annulus numbering, 0 <= a < ann_n); its frame index is
// ann0 + a.
__device__ __forceinline__ void ann_xy(CRun &R, int a, int &x, int &y) {
    strip_xy(R.Nx - R.rxm - R.rxp, R.Ny - R.rym - R.ryp, R.axm, R.axp, R.aym, R.ayp, a, x, y);
    x = (int)LBM_GUARD(R, x + R.rxm, R.Nx);
    y = (int)LBM_GUARD(R, y + R.rym, R.Ny);
}
// Node of frame index t (ring nodes first, then the annulus from ann0; t not in the gap).
__device__ __forceinline__ void frame_xy(CRun &R, int t, int &x, int &y) {
    if (t < R.ring_n) ring_xy(R, t, x, y);
    else ann_xy(R, t - R.ann0, x, y);
}

// Inverse of strip_xy: strip index of (x, y), or -1 outside the strips.
__device__ __forceinline__ int strip_idx(int Nx, int Ny, int dxm, int dxp, int dym, int dyp, int x, int y) {
    if (y < dym) return y * Nx + x;
    if (y >= Ny - dyp) return (dym + y - (Ny - dyp)) * Nx + x;
    int H = Ny - dym - dyp, base = (dym + dyp) * Nx, yy = y - dym;
    if (x < dxm) return base + yy * dxm + x;
    if (x >= Nx - dxp) return base + H * dxm + yy * dxp + (x - (Nx - dxp));
    return -1;
}

__device__ __forceinline__ int ridx(CRun &R, int x, int y) {
    return strip_idx(R.Nx, R.Ny, R.rxm, R.rxp, R.rym, R.ryp, x, y);
}
// Frame index of (x, y) on the grid, or -1 for a node of the fast rectangle.
__device__ __forceinline__ int fidx(CRun &R, int x, int y) {
    if (R.ring_n > 0) {   // (uniform) without a ring the annulus is the whole frame
        const int r = ridx(R, x, y);
        if (r >= 0) return r;
    }
    const int a = strip_idx(R.Nx - R.rxm - R.rxp, R.Ny - R.rym - R.ryp, R.axm, R.axp, R.aym, R.ayp,
                            x - R.rxm, y - R.rym);
    return a < 0 ? -1 : R.ann0 + a;
}

__device__ __forceinline__ bool in_q(CRun &R, int x, int y) {
    return (R.Wxm > 0 && x < R.qd) || (R.Wxp > 0 && x >= R.Nx - R.qd) ||
           (R.Wym > 0 && y < R.qd) || (R.Wyp > 0 && y >= R.Ny - R.qd);
}

// Characteristic-boundary node: within the outer 3 layers of an NRBC side.
__device__ __forceinline__ bool in_ring(CRun &R, int x, int y) {
    return (R.rxm > 0 && x < 3) || (R.rxp > 0 && x >= R.Nx - 3) ||
           (R.rym > 0 && y < 3) || (R.ryp > 0 && y >= R.Ny - 3);
}

// eq. PML_ramp on the Chebyshev ring level.
__device__ __forceinline__ double sigma_at(CRun &R, int x, int y) {
    int lx = x < R.Wxm ? R.Wxm - x : (x >= R.Nx - R.Wxp ? x - (R.Nx - R.Wxp) + 1 : 0);
    int ly = y < R.Wym ? R.Wym - y : (y >= R.Ny - R.Wyp ? y - (R.Ny - R.Wyp) + 1 : 0);
    int l = lx > ly ? lx : ly;
    return l > 0 ? R.sigma_max * (double)(l * l) * R.inv_W2 : 0.0;
}

// ------------------------------------------------------------------------------------------
// moments (eq. macro) in deviation form
// ------------------------------------------------------------------------------------------
template <class C> struct Mom { C drho, dux, duy, dT, rho; };

// Moment sums of populations taken pair by pair (pairs in order): s = sum g, j = sum e g,
// e2 = sum |e|^2 g, then the primitive deviations from them.
template <class C> struct MomAcc { C s, jx, jy, e2; };

template <class C>
__device__ __forceinline__ MomAcc<C> mom_begin(C g0) { return MomAcc<C>{g0, C(0), C(0), C(0)}; }

template <int p, class C>
__device__ __forceinline__ void mom_pair(MomAcc<C> &m, C a, C b) {
    C sp = a + b, dp = a - b;
    m.s += sp;
    if constexpr (PEX[p] == 1) m.jx += dp;
    else if constexpr (PEX[p] == -1) m.jx -= dp;
    else if constexpr (PEX[p] != 0) m.jx += C(PEX[p]) * dp;
    if constexpr (PEY[p] == 1) m.jy += dp;
    else if constexpr (PEY[p] == -1) m.jy -= dp;
    else if constexpr (PEY[p] != 0) m.jy += C(PEY[p]) * dp;
    if constexpr (SHELL_E2[PSH[p]] == 1) m.e2 += sp;
    else m.e2 += C(SHELL_E2[PSH[p]]) * sp;
}

template <class C>
__device__ __forceinline__ Mom<C> mom_end(const MomAcc<C> &a, const K<C> &k) {
    const C s = a.s;
    Mom<C> m;
    m.drho = s;
    m.rho = k.rho0 + s;
    C inv = C(1) / m.rho;
    C Jx = C(LAT_R) * a.jx, Jy = C(LAT_R) * a.jy, E = C(LAT_R2) * a.e2;
    m.dux = (Jx - s * k.u0x) * inv;
    m.duy = (Jy - s * k.u0y) * inv;
    C t = E - s * k.c2Tb0 - C(2) * m.rho * (k.u0x * m.dux + k.u0y * m.duy) -
          m.rho * (m.dux * m.dux + m.duy * m.duy);
    m.dT = C(0.5) * t * inv;
    return m;
}

template <class C>
__device__ __forceinline__ Mom<C> moments(const C (&g)[NQ], const K<C> &k) {
    MomAcc<C> a = mom_begin<C>(g[0]);
    static_for<0, NPAIR>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        mom_pair<p>(a, g[1 + 2 * p], g[2 + 2 * p]);
    });
    return mom_end<C>(a, k);
}

// Moments of populations read by get(i) in groups of PC pairs, each group's reads issued
// together and the groups kept apart, so only one group is held in registers; the same sums
// in the same order as moments().
template <int PC, class C, class Get>
__device__ __forceinline__ Mom<C> moments_streamed(Get &&get, const K<C> &k) {
    MomAcc<C> a = mom_begin<C>(get(std::integral_constant<int, 0>{}));
    static_for<0, (NPAIR + PC - 1) / PC>([&](auto cc) {
        constexpr int P0 = decltype(cc)::value * PC;
        constexpr int P1 = P0 + PC < NPAIR ? P0 + PC : NPAIR;
        C v[2 * (P1 - P0)];
        static_for<0, 2 * (P1 - P0)>([&](auto lc) {
            constexpr int l = decltype(lc)::value;
            v[l] = get(std::integral_constant<int, 1 + 2 * P0 + l>{});
        });
        static_for<P0, P1>([&](auto pc) {
            constexpr int p = decltype(pc)::value;
            mom_pair<p>(a, v[2 * (p - P0)], v[2 * (p - P0) + 1]);
        });
        __builtin_amdgcn_sched_barrier(0);
    });
    return mom_end<C>(a, k);
}

// ------------------------------------------------------------------------------------------
// equilibrium deviation feq(U) - fbar
// ------------------------------------------------------------------------------------------
template <class C> struct Eq {
    C drho, rho, Rdux, Rduy, dT, dk0, dk1, dk2a, dk2s, dth2;
    C dE0, dE2, dO1;   // current shell
};

template <class C>
__device__ __forceinline__ Eq<C> eq_coef(C drho, C dux, C duy, C dT, const K<C> &k) {
    Eq<C> q;
    q.drho = drho;
    q.rho = k.rho0 + drho;
    q.Rdux = C(LAT_R) * dux;
    q.Rduy = C(LAT_R) * duy;
    q.dT = dT;
    C db = dux * (C(2) * k.u0x + dux) + duy * (C(2) * k.u0y + duy);
    if constexpr (ORDER == 4) {
        C ux = k.u0x + dux, uy = k.u0y + duy, th = k.th0 + dT;
        C b = ux * ux + uy * uy;
        C dth2 = dT * (th + k.th0);
        C dthb = dT * b + k.th0 * db;
        C db2 = db * (b + k.b0);
        q.dk0 = -C(0.5) * db - dT + C(0.125) * db2 + dthb + dth2;
        q.dk2a = -C(0.25) * db - C(1.5) * dT;
        q.dk2s = C(0.5) * dT - C(0.25) * dthb - dth2;
        q.dth2 = dth2;
    } else {   // third and second order: k0 = 1 - b/2 - theta, k2a = 1/2, k2s = theta/2
        q.dk0 = -C(0.5) * db - dT;
        q.dk2a = C(0);
        q.dk2s = C(0.5) * dT;
        q.dth2 = C(0);
    }
    // odd part: O1 = k1 + theta c^2/2 with k1 = 1 - b/2 - 2 theta (fourth and third order);
    // the second-order equilibrium's odd part is a alone (O1 = 1)
    if constexpr (ORDER >= 3) q.dk1 = -C(0.5) * db - C(2) * dT;
    else q.dk1 = C(0);
    q.dE0 = q.dE2 = q.dO1 = C(0);
    return q;
}

template <class C>
__device__ __forceinline__ C feq_rest(const Eq<C> &q, CRun &R) {
    return C(SHELL_W[0]) * (q.drho * cH0rest<C>(R) + q.rho * q.dk0);
}

// Shell coefficient deviations (computed once per shell).
template <class C, int sh>
__device__ __forceinline__ void eq_shell(Eq<C> &q) {
    constexpr double sv = LAT_R2 * SHELL_E2[sh];
    if constexpr (ORDER == 4) {
        q.dE0 = q.dk0 + q.dk2s * C(sv) + q.dth2 * C(0.125 * sv * sv);
        q.dE2 = q.dk2a + q.dT * C(0.25 * sv);
    } else {
        q.dE0 = q.dk0 + q.dk2s * C(sv);
        q.dE2 = C(0);
    }
    if constexpr (ORDER >= 3) q.dO1 = q.dk1 + q.dT * C(0.5 * sv);
    else q.dO1 = C(0);
}

// feq - fbar of the pair p: (+e_p, -e_p).
template <class C, int p>
__device__ __forceinline__ void eq_pair(const Eq<C> &q, CRun &R, const K<C> &k, C &fp, C &fm) {
    constexpr int sh = PSH[p];
    constexpr int ex = PEX[p], ey = PEY[p];
    C a0, da;
    if constexpr (ey == 0) { a0 = C(ex) * k.r0x; da = C(ex) * q.Rdux; }
    else if constexpr (ex == 0) { a0 = C(ey) * k.r0y; da = C(ey) * q.Rduy; }
    else { a0 = C(ex) * k.r0x + C(ey) * k.r0y; da = C(ex) * q.Rdux + C(ey) * q.Rduy; }
    const C O1_0 = cO1_0<C>(R, sh);
    C a = a0 + da;
    C A2 = a * a, A02 = a0 * a0;
    C dA2 = da * (a + a0);
    C dEv;
    if constexpr (ORDER == 4)
        dEv = q.dE0 + q.dE2 * A2 + cE2_0<C>(R, sh) * dA2 + dA2 * (A2 + A02) * C(1.0 / 24.0);
    else   // E2 = 1/2 for every shell and state
        dEv = q.dE0 + C(0.5) * dA2;
    C dOd;
    if constexpr (ORDER >= 3)
        dOd = q.dO1 * a + O1_0 * da + da * (A2 + a * a0 + A02) * C(1.0 / 6.0);
    else   // eq. feq-2: the odd part is a itself
        dOd = da;
    C Tev = q.drho * cH0e<C>(R, p) + q.rho * dEv;
    C Tod = q.drho * cH0o<C>(R, p) + q.rho * dOd;
    constexpr double w = SHELL_W[sh];
    fp = C(w) * (Tev + Tod);
    fm = C(w) * (Tev - Tod);
}

// Calls emit(i, feq_i - fbar_i) for i = 0..NQ-1 with compile-time i.
template <class C, class F>
__device__ __forceinline__ void for_each_feq(Eq<C> q, CRun &R, const K<C> &k, F &&emit) {
    emit(std::integral_constant<int, 0>{}, feq_rest<C>(q, R));
    static_for<0, NPAIR>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        if constexpr (p == 0 || PSH[p - 1] != PSH[p]) eq_shell<C, PSH[p]>(q);
        C fp, fm;
        eq_pair<C, p>(q, R, k, fp, fm);
        emit(std::integral_constant<int, 1 + 2 * p>{}, fp);
        emit(std::integral_constant<int, 2 + 2 * p>{}, fm);
    });
}

// Two equilibria in one pass: emit(i, feq_a_i - fbar_i, feq_b_i - fbar_i).
template <class C, class F>
__device__ __forceinline__ void for_each_feq2(Eq<C> qa, Eq<C> qb, CRun &R, const K<C> &k, F &&emit) {
    emit(std::integral_constant<int, 0>{}, feq_rest<C>(qa, R), feq_rest<C>(qb, R));
    static_for<0, NPAIR>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        if constexpr (p == 0 || PSH[p - 1] != PSH[p]) {
            eq_shell<C, PSH[p]>(qa);
            eq_shell<C, PSH[p]>(qb);
        }
        C ap, am, bp, bm;
        eq_pair<C, p>(qa, R, k, ap, am);
        eq_pair<C, p>(qb, R, k, bp, bm);
        emit(std::integral_constant<int, 1 + 2 * p>{}, ap, bp);
        emit(std::integral_constant<int, 2 + 2 * p>{}, am, bm);
    });
}

// Pairs [P0, P1) of two equilibria: emit(i, feq_a_i - fbar_i, feq_b_i - fbar_i); the shell
// coefficients carry over in qa and qb from the pairs before P0 (pairs in order), so a sweep in
// groups gives the values of for_each_feq2.
template <int P0, int P1, class C, class F>
__device__ __forceinline__ void feq2_pairs(Eq<C> &qa, Eq<C> &qb, CRun &R, const K<C> &k, F &&emit) {
    static_for<P0, P1>([&](auto pc) {
        constexpr int p = decltype(pc)::value;
        if constexpr (p == 0 || PSH[p - 1] != PSH[p]) {
            eq_shell<C, PSH[p]>(qa);
            eq_shell<C, PSH[p]>(qb);
        }
        C ap, am, bp, bm;
        eq_pair<C, p>(qa, R, k, ap, am);
        eq_pair<C, p>(qb, R, k, bp, bm);
        emit(std::integral_constant<int, 1 + 2 * p>{}, ap, bp);
        emit(std::integral_constant<int, 2 + 2 * p>{}, am, bm);
    });
}

// ------------------------------------------------------------------------------------------
// characteristic boundary (float64 always)
// ------------------------------------------------------------------------------------------
// LODI along the outward normal of `side` for boundary node (x, y): primitive variables
// V = (rho, u_n, u_t, T), A = S^{-1} Lambda S, Lambda = diag(u_n - c, u_n, u_n, u_n + c),
// c = sqrt(2T) (p = rho T, gamma = 2).  Incoming amplitudes are zero (eq. PNR); an outgoing
// amplitude takes the upwind difference over the interval its characteristic crosses in one
// step (nu = lambda/r cells, foot point limited to two cells).  Adds the one-step increment
// dV = -S^{-1} Lbar (eq. thermal_LODI_macro_evo) to Ut in the global frame.
__device__ void lodi_add(CRun &R, const GLOBAL double *Uc, int side, int x, int y, int t,
                         double Ut[4]) {
    const unsigned qp = (unsigned)R.qplane;
    int nx = side == XMIN ? -1 : (side == XMAX ? 1 : 0);
    int ny = side == YMIN ? -1 : (side == YMAX ? 1 : 0);
    double V[3][4];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        int jj = j == 0 ? t : fidx(R, x - j * nx, y - j * ny);
        if (jj < 0) jj = t;
        jj = (int)LBM_GUARD(R, jj, R.qplane);
        double rho = Uc[jj], ux = Uc[qp + jj], uy = Uc[2 * qp + jj], T = Uc[3 * qp + jj];
        V[j][0] = rho;
        V[j][1] = nx ? nx * ux : ny * uy;
        V[j][2] = nx ? uy : ux;
        V[j][3] = T;
    }
    double rho = V[0][0], un = V[0][1], T = V[0][3];
    double c = sqrt(2.0 * T);
    double lam[4] = {un - c, un, un, un + c};
    double L[4][4] = {{T, -rho * c, 0.0, rho}, {T, 0.0, 0.0, -rho}, {0.0, 0.0, 1.0, 0.0},
                      {T, rho * c, 0.0, rho}};
    double D[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double w[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            w[j] = L[k][0] * V[j][0] + L[k][1] * V[j][1] + L[k][2] * V[j][2] + L[k][3] * V[j][3];
        if (lam[k] > 0.0) {
            double nu = fmin(lam[k] * (1.0 / LAT_R), 2.0);
            int j0 = nu >= 1.0 ? 1 : 0;
            double phi = nu - j0;
            double wa = j0 ? w[1] : w[0], wb = j0 ? w[2] : w[1];
            double wfoot = (1.0 - phi) * wa + phi * wb;
            D[k] = w[0] - wfoot;
        } else {
            D[k] = 0.0;
        }
    }
    // closed-form S^{-1}: columns (1/4T, -1/2rc, 0, 1/4r), (1/2T, 0, 0, -1/2r), e3,
    // (1/4T, 1/2rc, 0, 1/4r)
    double dR = -((D[0] + D[3]) / (4.0 * T) + D[1] / (2.0 * T));
    double dUn = -(D[3] - D[0]) / (2.0 * rho * c);
    double dUt = -D[2];
    double dTT = -((D[0] + D[3]) / (4.0 * rho) - D[1] / (2.0 * rho));
    Ut[0] += dR;
    Ut[3] += dTT;
    if (nx) { Ut[1] += nx * dUn; Ut[2] += dUt; }
    else    { Ut[2] += ny * dUn; Ut[1] += dUt; }
}

// Characteristic variables of the Euler flux along one direction for primitive variables
// v = (rho, u_along, u_across, T) (p = rho T, gamma = 2, c = sqrt(2T)), rows for the eigenvalues
// u - c, u (entropy), u (shear), u + c, and the inverse map.
__device__ __forceinline__ void char_fwd(double rho, double T, double c, const double (&v)[4], double (&w)[4]) {
    w[0] = T * v[0] - rho * c * v[1] + rho * v[3];
    w[1] = T * v[0] - rho * v[3];
    w[2] = v[2];
    w[3] = T * v[0] + rho * c * v[1] + rho * v[3];
}
__device__ __forceinline__ void char_inv(double rho, double T, double c, const double (&b)[4], double (&v)[4]) {
    v[0] = (b[0] + b[3]) / (4.0 * T) + b[1] / (2.0 * T);
    v[1] = (b[3] - b[0]) / (2.0 * rho * c);
    v[2] = b[2];
    v[3] = (b[0] + b[3]) / (4.0 * rho) - b[1] / (2.0 * rho);
}

// One-step increment, at edge position j (compile-time, 2..4 of 0..6), of the Euler flux along
// the edge: each characteristic variable of the edge direction, eigenvectors frozen at Vn[j],
// moves over the interval its characteristic crosses in one step (foot point at most 2 cells
// away, linear interpolation), written in differences so a state constant along the edge gives
// exactly zero.  Vn and dV in the normal frame (rho, u_n, u_t, T).
template <int J>
__device__ __forceinline__ void edge_advect(const double (&Vn)[7][4], double (&dV)[4]) {
    const double rho = Vn[J][0], ut = Vn[J][2], T = Vn[J][3], c = sqrt(2.0 * T);
    double w[5][4];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        const double vt[4] = {Vn[J - 2 + m][0], Vn[J - 2 + m][2], Vn[J - 2 + m][1], Vn[J - 2 + m][3]};
        char_fwd(rho, T, c, vt, w[m]);
    }
    const double lam[4] = {ut - c, ut, ut, ut + c};
    double dW[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double nu = lam[k] * (1.0 / LAT_R);
        if (!(nu == nu)) nu = 0.0;
        nu = fmin(fmax(nu, -2.0), 2.0);
        const double a = fabs(nu);
        const bool far = a >= 1.0, fwd = nu > 0.0;      // foot beyond one cell; foot at -nu
        const double phi = far ? a - 1.0 : a;
        const double w1 = fwd ? w[1][k] : w[3][k], w2 = fwd ? w[0][k] : w[4][k];
        const double wa = far ? w1 : w[2][k], wb = far ? w2 : w1;
        dW[k] = -((1.0 - phi) * (w[2][k] - wa) + phi * (w[2][k] - wb));
    }
    double dt[4];
    char_inv(rho, T, c, dW, dt);
    dV[0] = dt[0]; dV[1] = dt[2]; dV[2] = dt[1]; dV[3] = dt[3];
}

// CBC (A) (Sec. 4 eq. thermal_CBC_macro_evo with eq. CBC-Relax of Sec. 5.2) at node (x, y) of
// `side`, a node on no other open side: U_tgt += one step of dU/dt = -S^{-1} (Lbar + T + V) in
// the normal frame, where
//   - outgoing waves keep their LODI amplitude (upwind over the crossed interval, as lodi_add)
//     plus the transverse and viscous parts;
//   - T: the Euler flux along the edge, advected in the edge's characteristics (edge_advect) on
//     the node's own layer;
//   - V: tangential second derivatives only (normal viscous fluxes of an outflow vanish),
//     nu = (tau - 1/2)/r^2 on both velocity components and 2 nu on T (Pr = 1, c_p/c_v = 2),
//     taken of the transverse-advected states at the node and its edge neighbours (advection,
//     then diffusion: the unsplit sum of the two explicit parts is unstable);
//   - eq. CBC-Relax with T and V as right-hand-side terms: an incoming amplitude is
//     (1 - Ma) T_inc + V_inc of them, leaving it Ma T_inc (Ma = |u0| with c_s = 1).
// Edge neighbours beyond an open edge's ends repeat the end node.  Float64 throughout.
__device__ void cbc_a_add(CRun &R, const GLOBAL double *Uc, int side, int x, int y, int t, double Ut[4]) {
    const unsigned qp = (unsigned)R.qplane;
    const int nx = side == XMIN ? -1 : (side == XMAX ? 1 : 0);
    const int ny = side == YMIN ? -1 : (side == YMAX ? 1 : 0);
    const int nt = nx ? R.Ny : R.Nx, ct = nx ? y : x;
    const bool topen = nx ? R.open_y : R.open_x;
    double Vn[7][4];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        int cc = ct + j - 3;
        if (topen) cc = min(max(cc, 0), nt - 1);
        else cc = cc < 0 ? cc + nt : (cc >= nt ? cc - nt : cc);
        int jj = nx ? fidx(R, x, cc) : fidx(R, cc, y);
        if (jj < 0) jj = t;
        jj = (int)LBM_GUARD(R, jj, R.qplane);
        const double ux = Uc[qp + jj], uy = Uc[2 * qp + jj];
        Vn[j][0] = Uc[jj];
        Vn[j][1] = nx ? nx * ux : ny * uy;
        Vn[j][2] = nx ? uy : ux;
        Vn[j][3] = Uc[3 * qp + jj];
    }
    const double rho = Vn[3][0], un = Vn[3][1], T = Vn[3][3], c = sqrt(2.0 * T);
    const double lam[4] = {un - c, un, un, un + c};
    // LODI amplitudes of the outgoing normal characteristics, from x_b, x_b - n, x_b - 2n
    double wn[3][4];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int jj = k == 0 ? t : fidx(R, x - k * nx, y - k * ny);
        if (jj < 0) jj = t;
        jj = (int)LBM_GUARD(R, jj, R.qplane);
        const double ux = Uc[qp + jj], uy = Uc[2 * qp + jj];
        const double v[4] = {Uc[jj], nx ? nx * ux : ny * uy, nx ? uy : ux, Uc[3 * qp + jj]};
        char_fwd(rho, T, c, v, wn[k]);
    }
    // transverse part at the node and its edge neighbours; viscous part of the advected states
    double dVT[4], dm[4], dp[4];
    edge_advect<2>(Vn, dm);
    edge_advect<3>(Vn, dVT);
    edge_advect<4>(Vn, dp);
    double dVV[4] = {0.0, 0.0, 0.0, 0.0};
    if (!(topen && (ct == 0 || ct == nt - 1))) {
        const double nuv = (1.0 / R.omega - 0.5) * (1.0 / LAT_R2);
#pragma unroll
        for (int m = 1; m < 4; ++m) {
            const double a0 = Vn[2][m] + dm[m], a1 = Vn[3][m] + dVT[m], a2 = Vn[4][m] + dp[m];
            dVV[m] = (m == 3 ? 2.0 * nuv : nuv) * (a2 - 2.0 * a1 + a0);
        }
    }
    double aT[4], aV[4];
    char_fwd(rho, T, c, dVT, aT);
    char_fwd(rho, T, c, dVV, aV);
    const double ma = sqrt(R.b0);
    double dw[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (lam[k] > 0.0) {
            const double nu = fmin(lam[k] * (1.0 / LAT_R), 2.0);
            const bool far = nu >= 1.0;
            const double phi = far ? nu - 1.0 : nu;
            const double wa = far ? wn[1][k] : wn[0][k], wb = far ? wn[2][k] : wn[1][k];
            const double D = (1.0 - phi) * (wn[0][k] - wa) + phi * (wn[0][k] - wb);
            dw[k] = -D + aT[k] + aV[k];
        } else {
            dw[k] = ma * aT[k];
        }
    }
    double d[4];
    char_inv(rho, T, c, dw, d);
    Ut[0] += d[0];
    Ut[3] += d[3];
    if (nx) { Ut[1] += nx * d[1]; Ut[2] += d[2]; }
    else    { Ut[2] += ny * d[1]; Ut[1] += d[2]; }
}

// Pull of x_f = clamp(x, 3, N-4) on open axes (eq. zg-bc copies all q populations of x_f to a
// boundary node; interior frame nodes are their own x_f), with a single periodic wrap on
// periodic axes (N >= 3): identical shifts across populations fold to 7 source-row and
// 7 source-column offsets per node, so each population costs one add.
template <class S, class C, int I>
__device__ __forceinline__ C pull_one(CRun &R, const GLOBAL S *src, int xs, int ys, C inv_scale) {
    const int Nx = R.Nx, Ny = R.Ny;
    int sy = ys - ey_of(I), sx = xs - ex_of(I);
    if constexpr (ey_of(I) > 0) sy += sy < 0 ? Ny : 0;
    if constexpr (ey_of(I) < 0) sy -= sy >= Ny ? Ny : 0;
    if constexpr (ex_of(I) > 0) sx += sx < 0 ? Nx : 0;
    if constexpr (ex_of(I) < 0) sx -= sx >= Nx ? Nx : 0;
    return cvt_in(src[LBM_GUARD(R, (long long)I * R.plane + (long long)sy * R.pitch + sx, R.fsize)], inv_scale);
}

__device__ __forceinline__ int clamp_x(CRun &R, int x) { return R.open_x ? min(max(x, 3), R.Nx - 4) : x; }
__device__ __forceinline__ int clamp_y(CRun &R, int y) { return R.open_y ? min(max(y, 3), R.Ny - 4) : y; }

template <class S, class C>
__device__ __forceinline__ void gather_clamped(CRun &R, const GLOBAL S *src, int x, int y,
                                               C inv_scale, C (&g)[NQ]) {
    const int xs = clamp_x(R, x), ys = clamp_y(R, y);
    static_for<0, NQ>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        g[i] = pull_one<S, C, i>(R, src, xs, ys, inv_scale);
    });
}

// Non-equilibrium extrapolation into G (ring index tt): G <- feq(U_tgt) + g(x_f) - feq(U(x_f)),
// in float64, g the pulled populations of x_f (deviation form).  Two sweeps keep it in few
// registers: the moments of the pull first, then the fill a few pairs at a time from a second
// pull of the same values (cache hits).
template <class S, class C>
__device__ __forceinline__ void nrbc_fill(CRun &R, const GLOBAL S *src, int x, int y, C inv_scale,
                                          const double (&Ut)[4], int tt) {
    K<double> kd = load_k<double>(R);
    Mom<double> mf;
    {
        const int xs = clamp_x(R, x), ys = clamp_y(R, y);
        mf = moments_streamed<6, double>(
            [&](auto ic) { return (double)pull_one<S, C, decltype(ic)::value>(R, src, xs, ys, inv_scale); }, kd);
    }
    __builtin_amdgcn_sched_barrier(0);
    Eq<double> ef = eq_coef<double>(mf.drho, mf.dux, mf.duy, mf.dT, kd);
    Eq<double> et = eq_coef<double>(Ut[0] - R.rho0, Ut[1] - R.u0x, Ut[2] - R.u0y, Ut[3] - R.T0, kd);
    int xs = clamp_x(R, x), ys = clamp_y(R, y);
    // recompute the addresses of the second pull instead of keeping those of the first live
    asm volatile("" : "+v"(xs), "+v"(ys));
    GLOBAL C *G = (GLOBAL C *)R.G;
    const unsigned rp = (unsigned)R.rplane;
    {
        const C g0 = pull_one<S, C, 0>(R, src, xs, ys, inv_scale);
        G[tt] = (C)((double)g0 + (feq_rest<double>(et, R) - feq_rest<double>(ef, R)));
    }
    constexpr int PC = 3;   // pairs per sweep group
    static_for<0, (NPAIR + PC - 1) / PC>([&](auto cc) {
        constexpr int P0 = decltype(cc)::value * PC;
        constexpr int P1 = P0 + PC < NPAIR ? P0 + PC : NPAIR;
        C gv[2 * (P1 - P0)];
        static_for<0, 2 * (P1 - P0)>([&](auto lc) {
            constexpr int l = decltype(lc)::value;
            gv[l] = pull_one<S, C, 1 + 2 * P0 + l>(R, src, xs, ys, inv_scale);
        });
        feq2_pairs<P0, P1>(et, ef, R, kd, [&](auto ic, double ft, double ff) {
            constexpr int i = decltype(ic)::value;
            G[i * rp + tt] = (C)((double)gv[i - 1 - 2 * P0] + (ft - ff));
        });
        __builtin_amdgcn_sched_barrier(0);
    });
}

// grad Q stencil of a frame node (frame index t): d/dalpha Q = cs*Q(x) + c0*Q(j0) + c1*Q(j1),
// central (0, 1/2, -1/2 at x+1, x-1), one-sided at the outermost layer of an open axis (outward
// normal s: s*(3/2, -2, 1/2) at x, x-s, x-2s) (eqs. FD-dx-center, FD-dx-bw).  Offsets are byte
// offsets into one Q plane; a neighbour outside the frame falls back to the node itself (such
// nodes lie off the layer, where sigma = 0).
template <class C> struct QStencil {
    unsigned ot, ox0, ox1, oy0, oy1;
    C cxs, cx0, cx1, cys, cy0, cy1;
};

template <class C>
__device__ __forceinline__ QStencil<C> q_stencil(CRun &R, int x, int y, int t) {
    QStencil<C> q;
    int jx0, jx1, jy0, jy1;
    if (R.open_x && x == 0) {
        jx0 = fidx(R, 1, y); jx1 = fidx(R, 2, y);
        q.cxs = C(-1.5); q.cx0 = C(2); q.cx1 = C(-0.5);
    } else if (R.open_x && x == R.Nx - 1) {
        jx0 = fidx(R, x - 1, y); jx1 = fidx(R, x - 2, y);
        q.cxs = C(1.5); q.cx0 = C(-2); q.cx1 = C(0.5);
    } else {
        int xp = x + 1, xm = x - 1;
        if (xp >= R.Nx) xp -= R.Nx;
        if (xm < 0) xm += R.Nx;
        jx0 = fidx(R, xp, y); jx1 = fidx(R, xm, y);
        q.cxs = C(0); q.cx0 = C(0.5); q.cx1 = C(-0.5);
    }
    if (R.open_y && y == 0) {
        jy0 = fidx(R, x, 1); jy1 = fidx(R, x, 2);
        q.cys = C(-1.5); q.cy0 = C(2); q.cy1 = C(-0.5);
    } else if (R.open_y && y == R.Ny - 1) {
        jy0 = fidx(R, x, y - 1); jy1 = fidx(R, x, y - 2);
        q.cys = C(1.5); q.cy0 = C(-2); q.cy1 = C(0.5);
    } else {
        int yp = y + 1, ym = y - 1;
        if (yp >= R.Ny) yp -= R.Ny;
        if (ym < 0) ym += R.Ny;
        jy0 = fidx(R, x, yp); jy1 = fidx(R, x, ym);
        q.cys = C(0); q.cy0 = C(0.5); q.cy1 = C(-0.5);
    }
    q.ox0 = (unsigned)LBM_GUARD(R, jx0 < 0 ? t : jx0, R.qplane) * (unsigned)sizeof(C);
    q.ox1 = (unsigned)LBM_GUARD(R, jx1 < 0 ? t : jx1, R.qplane) * (unsigned)sizeof(C);
    q.oy0 = (unsigned)LBM_GUARD(R, jy0 < 0 ? t : jy0, R.qplane) * (unsigned)sizeof(C);
    q.oy1 = (unsigned)LBM_GUARD(R, jy1 < 0 ? t : jy1, R.qplane) * (unsigned)sizeof(C);
    q.ot = (unsigned)LBM_GUARD(R, t, R.qplane) * (unsigned)sizeof(C);
    return q;
}

// Appendix (eq. NSF-CHAR-PML): with a PML the macroscopic equations carry source terms built
// from the auxiliary moments; with phi = (1, xi_x, xi_y, |xi|^2/2) the selected parts
// I = sum phi_i e_i . grad Q_i (bit 0), II = 2 sum phi_i fhat_i (bit 1) and
// III = sigma sum phi_i Q_i (bit 2) move the characteristic target over one step by
// s = +sigma (I + II + III) (the appendix's signs) in conserved variables (rho, rho u,
// rho (|u|^2/2 + T)), converted to (rho, u, T) at U^n by the chain rule.  The quadrature carries
// the conserved moments of feq exactly, so II = 2 (U^n - Ubar) in conserved form.  Q and U of
// level n; float64 arithmetic; the population loop is left rolled (few nodes, low pressure).
template <class C>
__device__ __forceinline__ void pml_moments(CRun &R, int x, int y, int t, const GLOBAL double *Uc,
                                            double (&dU)[4]) {
    dU[0] = dU[1] = dU[2] = dU[3] = 0.0;
    const double sg = sigma_at(R, x, y);
    if (!(sg > 0.0)) return;
    const unsigned qp = (unsigned)R.qplane, flags = (unsigned)R.pml_terms;
    const double rho = Uc[t], ux = Uc[qp + t], uy = Uc[2 * qp + t], T = Uc[3 * qp + t];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (flags & 5u) {
        const QStencil<C> qs = q_stencil<C>(R, x, y, t);
        const GLOBAL C *Q = (const GLOBAL C *)R.Q;
#pragma unroll 1
        for (int i = 0; i < NQ; ++i) {
            const int ex = ex_of(i), ey = ey_of(i);
            const GLOBAL C *Qi = Q + (long long)i * qp;
            const double Qt = (double)*at(Qi, qs.ot);
            double a = 0.0;
            if (flags & 1u) {
                if (ex != 0)
                    a += ex * ((double)qs.cxs * Qt + (double)qs.cx0 * (double)*at(Qi, qs.ox0) +
                               (double)qs.cx1 * (double)*at(Qi, qs.ox1));
                if (ey != 0)
                    a += ey * ((double)qs.cys * Qt + (double)qs.cy0 * (double)*at(Qi, qs.oy0) +
                               (double)qs.cy1 * (double)*at(Qi, qs.oy1));
            }
            if (flags & 4u) a += sg * Qt;
            const double xx = LAT_R * ex, yy = LAT_R * ey;
            s0 += a;
            s1 += xx * a;
            s2 += yy * a;
            s3 += (0.5 * (xx * xx + yy * yy)) * a;
        }
    }
    if (flags & 2u) {
        const double b0 = R.rho0, bx = R.u0x, by = R.u0y, bT = R.T0;
        s0 += 2.0 * (rho - b0);
        s1 += 2.0 * (rho * ux - b0 * bx);
        s2 += 2.0 * (rho * uy - b0 * by);
        s3 += 2.0 * (rho * (0.5 * (ux * ux + uy * uy) + T) - b0 * (0.5 * (bx * bx + by * by) + bT));
    }
    s0 *= sg; s1 *= sg; s2 *= sg; s3 *= sg;
    dU[0] = s0;
    dU[1] = (s1 - ux * s0) / rho;
    dU[2] = (s2 - uy * s0) / rho;
    dU[3] = (s3 - ux * s1 - uy * s2 + (0.5 * (ux * ux + uy * uy) - T) * s0) / rho;
}

// Blocks of a run's boundary launches: the characteristic ring first (ring numbering, RING_BLOCK
// nodes per block), then the frame off the ring (annulus numbering, FRAME_BLOCK nodes per block),
// both counts padded to multiples of 8.  frame_start maps a frame block to its first annulus
// index, XCD by XCD.
__device__ __forceinline__ int ring_blocks(CRun &R) { return ring_block_count(R.ring_n); }
__device__ __forceinline__ int frame_start(CRun &R, int fblock) {
    return xcd_swizzle(fblock, frame_block_count(R.ann_n)) * FRAME_BLOCK;
}

// Characteristic targets of the ring, formed ahead of phase A for runs that select the appendix's
// PML moments or have a CBC (A) side: U_tgt = U^n(x_b) plus, for each characteristic side the
// node lies on, the CBC (A) increment (a node on that side only) or the LODI increment (corners
// add both normals), plus the PML moments; stored to P (4 planes of the ring numbering,
// float64).
template <class S>
__global__ __launch_bounds__(256) void k_target(RunDev *const *__restrict__ runs,
                                                const int *__restrict__ prefix, int nruns, int ks) {
    using C = typename Traits<S>::C;
    const int b = blockIdx.x;
    const int j = find_run(prefix, nruns, b);
    CRun &R = run_of(runs, j);
    const int par = sub_par(R, ks);
    if (par < 0 || !R.tgt_pre) return;
    if ((int)threadIdx.x >= RING_BLOCK) return;
    const int tt = (b - ((const CONSTANT int *)prefix)[j]) * RING_BLOCK + (int)threadIdx.x;
    if (tt >= R.ring_n) return;
    int x, y;
    ring_xy(R, tt, x, y);
    const int t = (int)LBM_GUARD(R, tt, R.rplane);   // a ring node's frame index is its ring index
    const GLOBAL double *Uc = (const GLOBAL double *)R.U[par];
    const unsigned qp = (unsigned)R.qplane;
    double Ut[4] = {Uc[t], Uc[qp + t], Uc[2 * qp + t], Uc[3 * qp + t]};
    // open sides whose boundary layers hold the node: CBC (A) applies on one side only, corners
    // take the LODI target of each characteristic normal
    bool on[4];
    int n_open = 0;
    for (int s = 0; s < 4; ++s) {
        on[s] = s == XMIN ? x < 3 : s == XMAX ? x >= R.Nx - 3 : s == YMIN ? y < 3 : y >= R.Ny - 3;
        on[s] = on[s] && R.bc[s] != BC_PERIODIC;
        n_open += on[s];
    }
    for (int s = 0; s < 4; ++s) {
        if (!on[s]) continue;
        if (R.bc[s] == BC_NRBC_A && n_open == 1) cbc_a_add(R, Uc, s, x, y, t, Ut);
        else if (is_char_bc(R.bc[s])) lodi_add(R, Uc, s, x, y, t, Ut);
    }
    if (R.pml_terms) {
        double dU[4];
        pml_moments<C>(R, x, y, t, Uc, dU);
        for (int k = 0; k < 4; ++k) Ut[k] += dU[k];
    }
    GLOBAL double *P = (GLOBAL double *)R.P;
    const unsigned rp = (unsigned)R.rplane;
#pragma unroll
    for (int k = 0; k < 4; ++k) P[k * rp + tt] = Ut[k];
}

// Ring node of characteristic sides: U_tgt = U(x_b) of the last completed level plus the LODI
// increment of each NRBC side the node lies on (corners add both normals) or, for runs that form
// their targets ahead, the target of k_target; then the clamped pull of x_f and the
// non-equilibrium extrapolation into G (ring index tt), where the Q update, the frame kernel and
// the moment export read it.
template <class S, class C>
__device__ __forceinline__ void nrbc_node(CRun &R, int par, int tt, int x, int y, int t, C inv_scale) {
    const GLOBAL double *Uc = (const GLOBAL double *)R.U[par];
    const unsigned qp = (unsigned)R.qplane;
    const bool pre = R.tgt_pre != 0;
    const GLOBAL double *Ub = pre ? (const GLOBAL double *)R.P : Uc;
    const unsigned ib = pre ? (unsigned)tt : (unsigned)t, sb = pre ? (unsigned)R.rplane : qp;
    double Ut[4] = {Ub[ib], Ub[sb + ib], Ub[2 * sb + ib], Ub[3 * sb + ib]};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        bool on = s == XMIN ? x < 3 : s == XMAX ? x >= R.Nx - 3 : s == YMIN ? y < 3 : y >= R.Ny - 3;
        // (runs with a CBC (A) side always form their targets ahead: pre is set)
        if (on && !pre && R.bc[s] == BC_NRBC) lodi_add(R, Uc, s, x, y, t, Ut);
    }
    nrbc_fill<S, C>(R, (const GLOBAL S *)R.f[par], x, y, inv_scale, Ut, tt);
}

// ------------------------------------------------------------------------------------------
// step kernels
// ------------------------------------------------------------------------------------------
// Bulk tile b (logical, after the XCD remap) of a launch set.
template <class S, int TX>
__device__ __forceinline__ void bulk_tile(RunDev *const *__restrict__ runs,
                                          const int *__restrict__ prefix, int nruns, int ks, int b) {
    using C = typename Traits<S>::C;
    constexpr int TY = 256 / TX;
    constexpr int TI = TX == 64 ? 0 : (TX == 128 ? 1 : 2);
    const int j = find_run(prefix, nruns, b);
    CRun &R = run_of(runs, j);
    const int par = sub_par(R, ks);
    if (par < 0) return;
    const int tb = b - ((const CONSTANT int *)prefix)[j];
    const int ty = tb / R.tiles_x[TI], tx = tb - ty * R.tiles_x[TI];
    const int x = (R.fx0 / TX) * TX + tx * TX + (int)(threadIdx.x % TX);
    const int y = R.fy0 + ty * TY + (int)(threadIdx.x / TX);
    if (x < R.fx0 || x >= R.fx1 || y >= R.fy1) return;
    const K<C> k = load_k<C>(R);
    const GLOBAL S *src = (const GLOBAL S *)R.f[par];
    GLOBAL S *dst = (GLOBAL S *)R.f[par ^ 1];
    const long long plane = R.plane;
    const int pitch = R.pitch;
    // uniform base at the tile's first row; per-lane 32-bit byte offset inside the tile
    const int y0 = R.fy0 + ty * TY;
    const GLOBAL S *src0 = src + (long long)y0 * pitch;
    GLOBAL S *dst0 = dst + (long long)y0 * pitch;
    const unsigned off = (unsigned)((y - y0) * pitch + x) * (unsigned)sizeof(S);
    C g[NQ];
    static_for<0, NQ>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const GLOBAL S *base = src0 + ((long long)i * plane - (ey_of(i) * pitch + ex_of(i)));
        g[i] = cvt_in(*LBM_AT(R, base, off, src, R.fsize), k.inv_scale);
    });
    Mom<C> m = moments<C>(g, k);
    Eq<C> q = eq_coef<C>(m.drho, m.dux, m.duy, m.dT, k);
    for_each_feq<C>(q, R, k, [&](auto ic, C fe) {
        constexpr int i = decltype(ic)::value;
        C out = g[i] + k.omega * (fe - g[i]);
        // FP64/FP32: streaming store (the next reads of these lines are a step away); FP16 rows
        // of a wave are single cache lines and measure faster as ordinary stores
        if constexpr (sizeof(S) >= 4)
            __builtin_nontemporal_store(cvt_out(out, k.scale, (S *)nullptr),
                                        LBM_AT(R, dst0 + (long long)i * plane, off, dst, R.fsize));
        else
            *LBM_AT(R, dst0 + (long long)i * plane, off, dst, R.fsize) = cvt_out(out, k.scale, (S *)nullptr);
    });
}

template <class S, int TX>
__global__ __launch_bounds__(256) void k_bulk(RunDev *const *__restrict__ runs,
                                              const int *__restrict__ prefix, int nruns, int ks) {
    bulk_tile<S, TX>(runs, prefix, nruns, ks, xcd_swizzle(blockIdx.x, gridDim.x));
}

// Collision of a frame node (frame index t) from its post-stream, post-boundary populations g:
// BGK plus, on PML nodes, -sigma (e.grad Q + 2 fhat + sigma Q) (eq. PMLCOLL) with grad Q central
// and one-sided at the outermost layer of an open axis (eqs. FD-dx-*); the moments go to U.
// The BGK part and -2 sigma fhat are formed first, in place of g; Q at the node and its
// neighbours is then read a few populations at a time, every read of a group issued before its
// first use (the pointers are restrict-qualified so later groups may be read ahead of earlier
// stores): a handful of memory round trips per node instead of one per population.
template <class S, class C>
__device__ __forceinline__ void frame_collide(CRun &R, const K<C> &k, const C (&g)[NQ], int x, int y,
                                              int t, const GLOBAL C *__restrict__ Q,
                                              GLOBAL S *__restrict__ dnode,
                                              GLOBAL double *__restrict__ Un) {
    const long long plane = R.plane;
    const unsigned qp = (unsigned)R.qplane;
    Mom<C> m = moments<C>(g, k);
    Eq<C> q = eq_coef<C>(m.drho, m.dux, m.duy, m.dT, k);
    if (R.has_q) {
        const QStencil<C> qs = q_stencil<C>(R, x, y, t);
        const unsigned ot = qs.ot, ox0 = qs.ox0, ox1 = qs.ox1, oy0 = qs.oy0, oy1 = qs.oy1;
        const C cxs = qs.cxs, cx0 = qs.cx0, cx1 = qs.cx1, cys = qs.cys, cy0 = qs.cy0, cy1 = qs.cy1;
        // sigma = 0 off the layer: the PML terms are then -0 * (finite) and leave BGK's bits
        const C s = (C)(R.W > 0 ? sigma_at(R, x, y) : 0.0);
        C h[NQ];
        for_each_feq<C>(q, R, k, [&](auto ic, C fe) {
            constexpr int i = decltype(ic)::value;
            C out = g[i] + k.omega * (fe - g[i]);
            h[i] = out - s * (C(2) * fe);
        });
        constexpr int CH = sizeof(C) == 8 ? 4 : 12;   // populations per group of Q reads
        static_for<0, (NQ + CH - 1) / CH>([&](auto cc) {
            constexpr int c0 = decltype(cc)::value * CH;
            constexpr int c1 = c0 + CH < NQ ? c0 + CH : NQ;
            C v[c1 - c0][5];
            static_for<c0, c1>([&](auto ic) {
                constexpr int i = decltype(ic)::value, l = i - c0;
                const GLOBAL C *Qi = Q + (long long)i * qp;
                v[l][0] = *at(Qi, ot);
                if constexpr (ex_of(i) != 0) { v[l][1] = *at(Qi, ox0); v[l][2] = *at(Qi, ox1); }
                if constexpr (ey_of(i) != 0) { v[l][3] = *at(Qi, oy0); v[l][4] = *at(Qi, oy1); }
            });
            static_for<c0, c1>([&](auto ic) {
                constexpr int i = decltype(ic)::value, l = i - c0;
                C gq = C(0);
                if constexpr (ex_of(i) != 0)
                    gq += C(ex_of(i)) * (cxs * v[l][0] + cx0 * v[l][1] + cx1 * v[l][2]);
                if constexpr (ey_of(i) != 0)
                    gq += C(ey_of(i)) * (cys * v[l][0] + cy0 * v[l][3] + cy1 * v[l][4]);
                C out = h[i] - s * (gq + s * v[l][0]);
                __builtin_nontemporal_store(cvt_out(out, k.scale, (S *)nullptr), dnode + (long long)i * plane);
            });
        });
    } else {
        for_each_feq<C>(q, R, k, [&](auto ic, C fe) {
            constexpr int i = decltype(ic)::value;
            C out = g[i] + k.omega * (fe - g[i]);
            __builtin_nontemporal_store(cvt_out(out, k.scale, (S *)nullptr), dnode + (long long)i * plane);
        });
    }
    Un[t] = R.rho0 + (double)m.drho;
    Un[qp + t] = R.u0x + (double)m.dux;
    Un[2 * qp + t] = R.u0y + (double)m.duy;
    Un[3 * qp + t] = R.T0 + (double)m.dT;
}

// Phase B of a step on the frame: ring blocks take the post-boundary populations phase A stored
// in G; the frame blocks, which cover the frame off the ring, pull (periodic wrap, or eq.
// zg-bc's copy of x_f = clamp(x, 3, N-4) on open axes).
template <class S>
__global__ __launch_bounds__(256) void k_frame(RunDev *const *__restrict__ runs,
                                               const int *__restrict__ prefix, int nruns, int ks) {
    using C = typename Traits<S>::C;
    const int b = blockIdx.x;
    const int j = find_run(prefix, nruns, b);
    CRun &R = run_of(runs, j);
    const int par = sub_par(R, ks);
    if (par < 0) return;
    const int tb = b - ((const CONSTANT int *)prefix)[j];
    const int rb = ring_blocks(R);
    const K<C> k = load_k<C>(R);
    int x, y, t;
    C g[NQ];
    if (tb < rb) {
        if ((int)threadIdx.x >= RING_BLOCK) return;
        const int tt = tb * RING_BLOCK + (int)threadIdx.x;
        if (tt >= R.ring_n) return;
        ring_xy(R, tt, x, y);
        t = (int)LBM_GUARD(R, tt, R.rplane);
        const GLOBAL C *G = (const GLOBAL C *)R.G;
        const unsigned rp = (unsigned)R.rplane;
#pragma unroll
        for (int i = 0; i < NQ; ++i) g[i] = G[i * rp + t];
    } else {
        const int ta = frame_start(R, tb - rb) + (int)threadIdx.x;
        if (ta >= R.ann_n) return;
        ann_xy(R, ta, x, y);
        t = (int)LBM_GUARD(R, R.ann0 + ta, R.qplane);
        gather_clamped<S, C>(R, (const GLOBAL S *)R.f[par], x, y, k.inv_scale, g);
    }
    frame_collide<S, C>(R, k, g, x, y, t, (const GLOBAL C *)R.Q,
                        (GLOBAL S *)R.f[par ^ 1] + (long long)y * R.pitch + x,
                        (GLOBAL double *)R.U[par ^ 1]);
}

// PML auxiliary update Q += (fhat^n + fhat^{n+1}) / 2 at frame node t (eq. PMLQ, trapezoid rule),
// fhat^n from the moment strip of the last level, fhat^{n+1} from m, the moments of g^{n+1}.  Q is
// read a few pairs at a time (each group's reads issued together, the groups kept apart), so the
// update runs in few registers.
template <class C>
__device__ __forceinline__ void q_update(CRun &R, int par, const K<C> &k0, const Mom<C> &m, int t) {
    // the uniform pair terms (e_p . u0 and its square) are formed afresh here: shared with the
    // ring fill's, they would stay live across it
    K<C> k = k0;
    asm volatile("" : "+s"(k.r0x), "+s"(k.r0y));
    const GLOBAL double *Uc = (const GLOBAL double *)R.U[par];
    const unsigned qp = (unsigned)R.qplane;
    GLOBAL C *Q = (GLOBAL C *)R.Q;
    const double r0 = Uc[t], ux0 = Uc[qp + t], uy0 = Uc[2 * qp + t], T0 = Uc[3 * qp + t];
    const unsigned ot = (unsigned)LBM_GUARD(R, t, R.qplane) * (unsigned)sizeof(C);
    Eq<C> q1 = eq_coef<C>(m.drho, m.dux, m.duy, m.dT, k);
    Eq<C> q0 = eq_coef<C>((C)(r0 - R.rho0), (C)(ux0 - R.u0x), (C)(uy0 - R.u0y), (C)(T0 - R.T0), k);
    {
        const C q = *at(Q, ot);
        *at(Q, ot) = q + C(0.5) * (feq_rest<C>(q0, R) + feq_rest<C>(q1, R));
    }
    constexpr int PC = 4;   // pairs per group of Q reads
    static_for<0, (NPAIR + PC - 1) / PC>([&](auto cc) {
        constexpr int P0 = decltype(cc)::value * PC;
        constexpr int P1 = P0 + PC < NPAIR ? P0 + PC : NPAIR;
        C Qv[2 * (P1 - P0)];
        static_for<0, 2 * (P1 - P0)>([&](auto lc) {
            constexpr int l = decltype(lc)::value;
            Qv[l] = *at(Q + (long long)(1 + 2 * P0 + l) * qp, ot);
        });
        feq2_pairs<P0, P1>(q1, q0, R, k, [&](auto ic, C fe1, C fe0) {
            constexpr int i = decltype(ic)::value;
            *at(Q + (long long)i * qp, ot) = Qv[i - 1 - 2 * P0] + C(0.5) * (fe0 + fe1);
        });
        __builtin_amdgcn_sched_barrier(0);
    });
}

// Block b of the phase-A class: ring blocks form the characteristic fill of the ring (into G)
// and, on PML nodes, update Q from it; frame blocks update Q of the PML nodes off the ring from
// their pull.
template <class S>
__device__ __forceinline__ void phase_a_block(RunDev *const *__restrict__ runs,
                                              const int *__restrict__ prefix, int nruns, int ks, int b) {
    using C = typename Traits<S>::C;
    const int j = find_run(prefix, nruns, b);
    CRun &R = run_of(runs, j);
    const int par = sub_par(R, ks);
    if (par < 0) return;
    const int tb = b - ((const CONSTANT int *)prefix)[j];
    const int rb = ring_blocks(R);
    const K<C> k = load_k<C>(R);
    int x, y, t;
    Mom<C> m;
    if (tb < rb) {
        if ((int)threadIdx.x >= RING_BLOCK) return;
        const int tt = tb * RING_BLOCK + (int)threadIdx.x;
        if (tt >= R.ring_n) return;
        ring_xy(R, tt, x, y);
        t = (int)LBM_GUARD(R, tt, R.rplane);
        nrbc_node<S, C>(R, par, t, x, y, t, k.inv_scale);
        if (!R.has_q || !in_q(R, x, y)) return;
        // the moments of the filled populations, read back from G (this thread's own stores);
        // the opaque index makes the reads form their addresses afresh rather than keep those
        // of the stores live
        int tr = t;
        asm volatile("" : "+v"(tr) : : "memory");
        const GLOBAL C *G = (const GLOBAL C *)R.G;
        const unsigned rp = (unsigned)R.rplane;
        m = moments_streamed<6, C>([&](auto ic) { return G[decltype(ic)::value * rp + tr]; }, k);
    } else {
        const int ta = frame_start(R, tb - rb) + (int)threadIdx.x;
        if (!R.has_q || ta >= R.ann_n) return;
        ann_xy(R, ta, x, y);
        if (!in_q(R, x, y)) return;
        t = (int)LBM_GUARD(R, R.ann0 + ta, R.qplane);
        C g[NQ];
        gather_clamped<S, C>(R, (const GLOBAL S *)R.f[par], x, y, k.inv_scale, g);
        m = moments<C>(g, k);
    }
    __builtin_amdgcn_sched_barrier(0);
    q_update<C>(R, par, k, m, t);
}

// Phase A of a step (eq. PMLQ on the Q region; the characteristic fill of the ring).
template <class S>
__global__ __launch_bounds__(256) void k_phase_a(RunDev *const *__restrict__ runs,
                                                 const int *__restrict__ prefix, int nruns, int ks) {
    phase_a_block<S>(runs, prefix, nruns, ks, blockIdx.x);
}

// Phase A and the bulk tiles of a step in one launch: h bulk tiles, the nA phase-A blocks, then
// the other nB - h bulk tiles.  The latency-bound phase-A waves run beside streaming tiles; the
// tiles after them keep them off the grid's tail, the tiles before them evict less of what the
// frame kernel then reads.  nA and h are multiples of 8, so every block keeps its XCD map.  Both
// paths share one register budget, held at 4 waves per SIMD (128 VGPRs) by the low-register
// boundary code, the branch-light block dispatch and the occupancy target.
template <class S, int TX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_phase_a_bulk(RunDev *const *__restrict__ runs,
                                                      const int *__restrict__ preA, int nA,
                                                      const int *__restrict__ preB, int nB, int h,
                                                      int nruns, int ks) {
    const int b = blockIdx.x;
    const int pa = b - h;   // blocks [h, h + nA) are phase A; the tiles before and after them
    if ((unsigned)pa < (unsigned)nA) phase_a_block<S>(runs, preA, nruns, ks, pa);
    else bulk_tile<S, TX>(runs, preB, nruns, ks, xcd_swizzle(pa < 0 ? b : b - nA, nB));
}

// End of a batch of n steps: each run advances by the sub-steps it was active for, min(n,
// limit - step), and its buffer parity by the same count.
__global__ void k_advance(RunDev *const *runs, int nruns, int n) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nruns) return;
    RunDev *R = runs[j];
    long long a = R->limit - R->step;
    a = a < 0 ? 0 : (a > n ? n : a);
    R->step += a;
    R->par ^= (int)(a & 1);
}

// Debug canary: before the step kernels of sub-step ks, every buffer that a step writes in full
// -- the destination populations, the new moment strips, and the ring's characteristic fill G
// and targets P -- is filled with NaN in its own type.  A node or component that the step leaves
// unwritten and a later kernel reads then carries NaN into the result.
template <class S>
__global__ __launch_bounds__(256) void k_poison(RunDev *const *runs, int ks) {
    using C = typename Traits<S>::C;
    CRun &R = run_of(runs, blockIdx.y);
    const int par = sub_par(R, ks);
    if (par < 0) return;
    const long long t0 = (long long)blockIdx.x * 256 + threadIdx.x, st = (long long)gridDim.x * 256;
    GLOBAL S *f = (GLOBAL S *)R.f[par ^ 1];
    const S ns = (S)__builtin_nanf("");
    for (long long i = t0; i < R.fsize; i += st) f[i] = ns;
    GLOBAL double *U = (GLOBAL double *)R.U[par ^ 1];
    for (long long i = t0; i < 4 * R.qplane; i += st) U[i] = __builtin_nan("");
    if (R.ring_n > 0 && R.G) {
        GLOBAL C *G = (GLOBAL C *)R.G;
        for (long long i = t0; i < (long long)NQ * R.rplane; i += st) G[i] = (C)__builtin_nanf("");
    }
    if (R.ring_n > 0 && R.P) {
        GLOBAL double *P = (GLOBAL double *)R.P;
        for (long long i = t0; i < 4 * R.rplane; i += st) P[i] = __builtin_nan("");
    }
}

__global__ void k_set_limit(RunDev *run, long long limit) {
    if (threadIdx.x == 0) run->limit = limit;
}

__global__ void k_set_limits(RunDev *const *runs, const long long *limits, int n) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) runs[j]->limit = limits[j];
}

// ------------------------------------------------------------------------------------------
// init, export, checks, reductions
// ------------------------------------------------------------------------------------------
template <class S>
__global__ __launch_bounds__(256) void k_init(RunDev *Rw, const double *rho, const double *ux,
                                              const double *uy, const double *T, float *absmax) {
    using C = typename Traits<S>::C;
    CRun &R = *(CRun *)Rw;
    __shared__ float red[256];
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int nn = R.Nx * R.Ny;
    float mx = 0.0f;
    if (n < nn) {
        const int y = n / R.Nx, x = n - y * R.Nx;
        const K<C> k = load_k<C>(R);
        Eq<C> q = eq_coef<C>((C)(rho[n] - R.rho0), (C)(ux[n] - R.u0x), (C)(uy[n] - R.u0y),
                             (C)(T[n] - R.T0), k);
        GLOBAL S *dst = (GLOBAL S *)R.f[0];
        const long long idx = (long long)y * R.pitch + x, plane = R.plane;
        for_each_feq<C>(q, R, k, [&](auto ic, C fe) {
            constexpr int i = decltype(ic)::value;
            if (absmax) mx = fmaxf(mx, fabsf((float)fe));
            else dst[(long long)i * plane + idx] = cvt_out(fe, k.scale, (S *)nullptr);
        });
        if (!absmax) {
            int t = fidx(R, x, y);
            if (t >= 0) {
                const long long qp = R.qplane;
                for (int c = 0; c < 2; ++c) {
                    GLOBAL double *U = (GLOBAL double *)R.U[c];
                    U[t] = rho[n];
                    U[qp + t] = ux[n];
                    U[2 * qp + t] = uy[n];
                    U[3 * qp + t] = T[n];
                }
            }
        }
    }
    if (absmax) {
        red[threadIdx.x] = mx;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) absmax[blockIdx.x] = red[0];
    }
}

// Moments of node (x, y) at the current step (post-stream, post-boundary): re-pull from the
// previous buffer with the previous moment strips; after 0 steps, moments of f*(0).
template <class S, class C>
__device__ __forceinline__ Mom<C> state_moments(CRun &R, int x, int y, const K<C> &k) {
    C g[NQ];
    if (R.step == 0) {
        const GLOBAL S *src = (const GLOBAL S *)R.f[R.par];
        const long long idx = (long long)y * R.pitch + x;
#pragma unroll
        for (int i = 0; i < NQ; ++i) g[i] = cvt_in(src[(long long)i * R.plane + idx], k.inv_scale);
    } else {
        const GLOBAL S *src = (const GLOBAL S *)R.f[R.par ^ 1];
        if (in_ring(R, x, y)) {   // ring: G, refreshed by the caller for this level
            const GLOBAL C *G = (const GLOBAL C *)R.G;
            const unsigned rp = (unsigned)R.rplane, r = (unsigned)ridx(R, x, y);
#pragma unroll
            for (int i = 0; i < NQ; ++i) g[i] = G[i * rp + r];
        } else {
            gather_clamped<S, C>(R, src, x, y, k.inv_scale, g);
        }
    }
    return moments<C>(g, k);
}

template <class S>
__global__ __launch_bounds__(256) void k_moments(RunDev *Rw, double *rho, double *ux, double *uy,
                                                 double *T) {
    using C = typename Traits<S>::C;
    CRun &R = *(CRun *)Rw;
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= R.Nx * R.Ny) return;
    const int y = n / R.Nx, x = n - y * R.Nx;
    const K<C> k = load_k<C>(R);
    Mom<C> m = state_moments<S, C>(R, x, y, k);
    if (rho) rho[n] = R.rho0 + (double)m.drho;
    if (ux) ux[n] = R.u0x + (double)m.dux;
    if (uy) uy[n] = R.u0y + (double)m.duy;
    if (T) T[n] = R.T0 + (double)m.dT;
}

template <class S>
__global__ __launch_bounds__(256) void k_export_f(RunDev *Rw, const double *fbar, double *out) {
    using C = typename Traits<S>::C;
    CRun &R = *(CRun *)Rw;
    const int n = blockIdx.x * 256 + threadIdx.x;
    const int nn = R.Nx * R.Ny;
    if (n >= nn) return;
    const int y = n / R.Nx, x = n - y * R.Nx;
    const K<C> k = load_k<C>(R);
    const GLOBAL S *src = (const GLOBAL S *)R.f[R.par];
    const long long idx = (long long)y * R.pitch + x;
    for (int i = 0; i < NQ; ++i)
        out[(long long)i * nn + n] = fbar[i] + (double)cvt_in(src[(long long)i * R.plane + idx], k.inv_scale);
}

template <class S>
__global__ __launch_bounds__(256) void k_export_q(RunDev *Rw, double *out) {
    using C = typename Traits<S>::C;
    CRun &R = *(CRun *)Rw;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= R.ann0 + R.ann_n || (t >= R.ring_n && t < R.ann0)) return;   // past the end; the gap
    int x, y;
    frame_xy(R, t, x, y);
    const long long nn = (long long)R.Nx * R.Ny;
    const GLOBAL C *Q = (const GLOBAL C *)R.Q;
    for (int i = 0; i < NQ; ++i) out[i * nn + (long long)y * R.Nx + x] = (double)Q[i * R.qplane + t];
}

template <class S>
__global__ __launch_bounds__(256) void k_check(RunDev *Rw, int *flag) {
    using C = typename Traits<S>::C;
    CRun &R = *(CRun *)Rw;
    const int n = blockIdx.x * 256 + threadIdx.x;
#ifdef LBM_BOUNDS
    if (n == 0 && R.oob) atomicOr(flag, 2);   // an index out of range since the run was set up
#endif
    if (n >= R.Nx * R.Ny) return;
    const int y = n / R.Nx, x = n - y * R.Nx;
    const K<C> k = load_k<C>(R);
    const GLOBAL S *src = (const GLOBAL S *)R.f[R.par];
    const long long idx = (long long)y * R.pitch + x;
    C g[NQ];
    bool bad = false;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        g[i] = cvt_in(src[(long long)i * R.plane + idx], k.inv_scale);
        bad |= !isfinite((double)g[i]);
    }
    Mom<C> m = moments<C>(g, k);
    double rho = R.rho0 + (double)m.drho, T = R.T0 + (double)m.dT;
    bad |= !(rho > 0.0) || !(T > 0.0) || !isfinite(rho) || !isfinite(T);
    if (bad) atomicOr(flag, 1);
}

// Reflection-error sums of one bulk row per block, fixed order (strided per thread, then a
// tree in LDS): partials[3*row + z].
__global__ __launch_bounds__(256) void k_err_rows(const double *rho, const double *ux,
                                                  const double *T, int Nx, int x0, int y0, int lx,
                                                  const double *rr, const double *ru,
                                                  const double *rt, double *partials) {
    __shared__ double red[3][256];
    const int row = blockIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    for (int xb = threadIdx.x; xb < lx; xb += 256) {
        long long n = (long long)(row + y0) * Nx + (xb + x0), m = (long long)row * lx + xb;
        double a = (rho[n] - rr[m]) / rr[m], b = (ux[n] - ru[m]) / ru[m], c = (T[n] - rt[m]) / rt[m];
        s[0] += a * a; s[1] += b * b; s[2] += c * c;
    }
    for (int z = 0; z < 3; ++z) red[z][threadIdx.x] = s[z];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int z = 0; z < 3; ++z) red[z][threadIdx.x] += red[z][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) partials[3 * row + threadIdx.x] = red[threadIdx.x][0];
}

// The reflection-error sums of k_err_rows taken straight from the run's state (the moments of
// state_moments, formed as k_moments writes them): the same values, the same order, so the same
// bits as k_moments followed by k_err_rows.  One bulk row per block; refs are bulk-sized.
template <class S>
__global__ __launch_bounds__(256) void k_err_rows_state(RunDev *Rw, int x0, int y0, int lx,
                                                        const double *rr, const double *ru,
                                                        const double *rt, double *partials) {
    using C = typename Traits<S>::C;
    CRun &R = *(CRun *)Rw;
    __shared__ double red[3][256];
    const int row = blockIdx.x;
    const K<C> k = load_k<C>(R);
    double s[3] = {0.0, 0.0, 0.0};
    for (int xb = threadIdx.x; xb < lx; xb += 256) {
        const Mom<C> m = state_moments<S, C>(R, xb + x0, row + y0, k);
        const double rho = R.rho0 + (double)m.drho, ux = R.u0x + (double)m.dux, T = R.T0 + (double)m.dT;
        const long long q = (long long)row * lx + xb;
        double a = (rho - rr[q]) / rr[q], b = (ux - ru[q]) / ru[q], c = (T - rt[q]) / rt[q];
        s[0] += a * a; s[1] += b * b; s[2] += c * c;
    }
    for (int z = 0; z < 3; ++z) red[z][threadIdx.x] = s[z];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int z = 0; z < 3; ++z) red[z][threadIdx.x] += red[z][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) partials[3 * row + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_err_final(const double *partials, int nrows, double *out) {
    __shared__ double red[3][256];
    double s[3] = {0.0, 0.0, 0.0};
    for (int r = threadIdx.x; r < nrows; r += 256)
        for (int z = 0; z < 3; ++z) s[z] += partials[3 * r + z];
    for (int z = 0; z < 3; ++z) red[z][threadIdx.x] = s[z];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int z = 0; z < 3; ++z) red[z][threadIdx.x] += red[z][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = sqrt(red[threadIdx.x][0]);
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
#define LBM_DISPATCH(storage, ...)                                                          \
    switch (storage) {                                                                      \
    case ST_F64: { using S = double; __VA_ARGS__; break; }                                  \
    case ST_F32: { using S = float; __VA_ARGS__; break; }                                   \
    default: { using S = _Float16; __VA_ARGS__; break; }                                    \
    }

static inline int blocks_for(long long n) { return (int)((n + 255) / 256); }

static hipError_t launch_phase_a(const LaunchSet &L, int storage, int ks, hipStream_t s) {
    if (L.blocks[CLS_A] > 0)
        LBM_DISPATCH(storage, hipLaunchKernelGGL((k_phase_a<S>), dim3(L.blocks[CLS_A]), dim3(256), 0, s,
                                                 L.runs, L.prefix[CLS_A], L.nruns, ks));
    return hipGetLastError();
}

static hipError_t launch_target(const LaunchSet &L, int storage, int ks, hipStream_t s) {
    if (L.blocks[CLS_TGT] > 0)
        LBM_DISPATCH(storage, hipLaunchKernelGGL((k_target<S>), dim3(L.blocks[CLS_TGT]), dim3(256), 0, s,
                                                 L.runs, L.prefix[CLS_TGT], L.nruns, ks));
    return hipGetLastError();
}

static hipError_t launch_frame(const LaunchSet &L, int storage, int ks, hipStream_t s, hipEvent_t a,
                               hipEvent_t b) {
    const int nb = L.blocks[CLS_FRAME];
    if (nb <= 0) return hipSuccess;
    const int *pre = L.prefix[CLS_FRAME];
    LBM_DISPATCH(storage, if (a) hipExtLaunchKernelGGL((k_frame<S>), dim3(nb), dim3(256), 0, s, a, b, 0,
                                                       L.runs, pre, L.nruns, ks);
                          else hipLaunchKernelGGL((k_frame<S>), dim3(nb), dim3(256), 0, s, L.runs, pre,
                                                  L.nruns, ks));
    return hipGetLastError();
}

static hipError_t launch_bulk(const LaunchSet &L, int storage, int tx, int ks, hipStream_t s,
                              hipEvent_t a, hipEvent_t b) {
    const int nb = L.blocks[CLS_BULK];
    if (nb <= 0) return hipSuccess;
    const int *pre = L.prefix[CLS_BULK];
    // events attached to the dispatch itself (no separate event packets around the kernel)
#define LBM_BULK(TXV)                                                                              \
    LBM_DISPATCH(storage, if (a) hipExtLaunchKernelGGL((k_bulk<S, TXV>), dim3(nb), dim3(256), 0, s, \
                                                       a, b, 0, L.runs, pre, L.nruns, ks);        \
                          else hipLaunchKernelGGL((k_bulk<S, TXV>), dim3(nb), dim3(256), 0, s,     \
                                                  L.runs, pre, L.nruns, ks))
    switch (tx) {
    case 64: LBM_BULK(64); break;
    case 128: LBM_BULK(128); break;
    default: LBM_BULK(256); break;
    }
#undef LBM_BULK
    return hipGetLastError();
}

static hipError_t launch_phase_a_bulk(const LaunchSet &L, int storage, int tx, int ks, hipStream_t s,
                                      hipEvent_t a, hipEvent_t b) {
    const int nA = L.blocks[CLS_A], nB = L.blocks[CLS_BULK];
    if (nA + nB <= 0) return hipSuccess;
    // Bulk tiles ahead of the phase-A blocks (by default).  On large grids, where the tiles
    // outnumber the phase-A blocks eightfold or more, all of them: phase A's latency then hides
    // in the grid's tail, 0.1-3% faster at 4224^2 (D2Q37 NRBC FP32 1158.7 against 1171.3 us per
    // step, FP16 707.9 against 722.5; D2Q17 ZG FP16 303.6 against 313.1; D2Q9 ZG FP64 510.1
    // against 523.3).  Otherwise half of them for D2Q37 in FP64, where the half after phase A
    // still outlasts its latency (1088^2 NRBC + PML: 178.5 against 185.5 us per step), and none
    // for the rest, where the shorter tiles would leave phase A on the tail (FP32 98.8 against
    // 97.1 us, FP16 66.6 against 62.0, D2Q9 FP64 47.1 against 46.5).
    const int h = L.split >= 0 ? (nB * L.split / 8) & ~7
                  : nB >= 8 * nA ? nB & ~7
                  : (NQ == 37 && storage == ST_F64) ? (nB / 2) & ~7 : 0;
    const int *pa = L.prefix[CLS_A], *pb = L.prefix[CLS_BULK];
#define LBM_PAB(TXV)                                                                               \
    LBM_DISPATCH(storage, if (a) hipExtLaunchKernelGGL((k_phase_a_bulk<S, TXV>), dim3(nA + nB), dim3(256), \
                                                       0, s, a, b, 0, L.runs, pa, nA, pb, nB, h,   \
                                                       L.nruns, ks);                               \
                          else hipLaunchKernelGGL((k_phase_a_bulk<S, TXV>), dim3(nA + nB), dim3(256), \
                                                  0, s, L.runs, pa, nA, pb, nB, h, L.nruns, ks))
    switch (tx) {
    case 64: LBM_PAB(64); break;
    case 128: LBM_PAB(128); break;
    default: LBM_PAB(256); break;
    }
#undef LBM_PAB
    return hipGetLastError();
}

static hipError_t launch_advance(const LaunchSet &L, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3((L.nruns + 255) / 256), dim3(256), 0, s, L.runs, L.nruns, n);
    return hipGetLastError();
}

static hipError_t launch_poison(const LaunchSet &L, int storage, int ks, hipStream_t s) {
    if (L.nruns <= 0) return hipSuccess;
    LBM_DISPATCH(storage, hipLaunchKernelGGL((k_poison<S>), dim3(1024, L.nruns), dim3(256), 0, s, L.runs,
                                             ks));
    return hipGetLastError();
}

static hipError_t launch_set_limit(RunDev *run, long long limit, hipStream_t s) {
    hipLaunchKernelGGL(k_set_limit, dim3(1), dim3(64), 0, s, run, limit);
    return hipGetLastError();
}

static hipError_t launch_set_limits(RunDev *const *runs, const long long *limits, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_set_limits, dim3((n + 255) / 256), dim3(256), 0, s, runs, limits, n);
    return hipGetLastError();
}

static hipError_t launch_init(RunDev *run, int storage, int Nx, int Ny, const double *rho,
                       const double *ux, const double *uy, const double *T, float *absmax,
                       hipStream_t s) {
    int nb = blocks_for((long long)Nx * Ny);
    LBM_DISPATCH(storage, hipLaunchKernelGGL((k_init<S>), dim3(nb), dim3(256), 0, s, run, rho, ux, uy,
                                             T, absmax));
    return hipGetLastError();
}

static hipError_t launch_moments(RunDev *run, int storage, int Nx, int Ny, double *rho, double *ux,
                          double *uy, double *T, hipStream_t s) {
    int nb = blocks_for((long long)Nx * Ny);
    LBM_DISPATCH(storage, hipLaunchKernelGGL((k_moments<S>), dim3(nb), dim3(256), 0, s, run, rho, ux,
                                             uy, T));
    return hipGetLastError();
}

static hipError_t launch_export_f(RunDev *run, int storage, int Nx, int Ny, const double *fbar,
                           double *out, hipStream_t s) {
    int nb = blocks_for((long long)Nx * Ny);
    LBM_DISPATCH(storage, hipLaunchKernelGGL((k_export_f<S>), dim3(nb), dim3(256), 0, s, run, fbar,
                                             out));
    return hipGetLastError();
}

static hipError_t launch_export_q(RunDev *run, int storage, int nt, double *out, hipStream_t s) {
    if (nt <= 0) return hipSuccess;
    int nb = blocks_for(nt);
    LBM_DISPATCH(storage, hipLaunchKernelGGL((k_export_q<S>), dim3(nb), dim3(256), 0, s, run, out));
    return hipGetLastError();
}

static hipError_t launch_check(RunDev *run, int storage, int Nx, int Ny, int *flag, hipStream_t s) {
    int nb = blocks_for((long long)Nx * Ny);
    LBM_DISPATCH(storage, hipLaunchKernelGGL((k_check<S>), dim3(nb), dim3(256), 0, s, run, flag));
    return hipGetLastError();
}

static hipError_t launch_err_rows(const double *rho, const double *ux, const double *T, int Nx, int x0,
                           int y0, int lx, int ly, const double *rr, const double *ru,
                           const double *rt, double *partials, hipStream_t s) {
    if (ly <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_err_rows, dim3(ly), dim3(256), 0, s, rho, ux, T, Nx, x0, y0, lx, rr, ru, rt,
                       partials);
    return hipGetLastError();
}

static hipError_t launch_err_rows_state(RunDev *run, int storage, int x0, int y0, int lx, int ly,
                                        const double *rr, const double *ru, const double *rt,
                                        double *partials, hipStream_t s) {
    if (ly <= 0) return hipSuccess;
    LBM_DISPATCH(storage, hipLaunchKernelGGL((k_err_rows_state<S>), dim3(ly), dim3(256), 0, s, run, x0, y0,
                                             lx, rr, ru, rt, partials));
    return hipGetLastError();
}

static hipError_t launch_err_final(const double *partials, int nrows, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_err_final, dim3(1), dim3(256), 0, s, partials, nrows, out);
    return hipGetLastError();
}

// host-side table (the device pass has no host functions to point at)
#ifndef __HIP_DEVICE_COMPILE__
const KernelSet kernels = {NQ, launch_phase_a, launch_frame, launch_target, launch_phase_a_bulk, launch_bulk,
                           launch_advance, launch_set_limit, launch_set_limits, launch_init,
                           launch_moments, launch_export_f, launch_export_q, launch_check,
                           launch_err_rows, launch_err_rows_state, launch_err_final, launch_poison};
#endif

}  // namespace LBM_KSET
}  // namespace lbm
