// Lattice constants of the library (host and device): the D2Q37, D2Q17 and D2Q9 velocity
// stencils.
//
// All three are minimal Gauss-Hermite rules in 2D with integer velocities of maximum
// displacement at most 3 and positive weights (paper Sec. 2, "Velocity stencils"): D2Q37 of
// ninth order, carrying the fourth-order equilibrium (eq. feq-4), D2Q17 of seventh order with
// the third-order equilibrium (eq. feq-3), and D2Q9 of fifth order with the second-order one
// (eq. feq-2).  Weights and scales as published by Philippi et al., PRE 73 (2006) 056702 and
// Shan, PRE 81 (2010) 036702 (D2Q17 in closed form: r^2 = (125 + 5 sqrt193)/72; D2Q9: r^2 = 3,
// weights 4/9, 1/9, 1/36).
// Thermal velocities are xi_i = LAT_R e_i (sound-speed unit 1).
//
// Library population order: 0 is the rest velocity; pair p = 0..NPAIR-1 holds +e_p at index
// 1 + 2p and -e_p at index 2 + 2p, so odd/even Hermite parts are shared within a pair.  The
// kernels are compiled once per stencil with that stencil's namespace in scope; the host reads
// the same tables through LatticeInfo.
#pragma once

namespace lbm {

constexpr int NQ_MAX = 37;
constexpr int NPAIR_MAX = 18;
constexpr int NSHELL_MAX = 8;

namespace d2q37 {
constexpr int NQ = 37;
constexpr int NPAIR = 18;
constexpr int NSHELL = 8;
constexpr int ORDER = 4;   // Hermite order of the equilibrium

constexpr double LAT_R = 1.196979770393074358972388;
constexpr double LAT_R2 = LAT_R * LAT_R;

// shell k: |e|^2 and the weight of each of its velocities
inline constexpr int SHELL_E2[NSHELL] = {0, 1, 2, 4, 5, 8, 9, 10};
inline constexpr double SHELL_W[NSHELL] = {
    0.2331506691323525022865,    0.1073060915422190024125,
    0.05766785988879488203007,   0.0142082161584507502647,
    0.005353049000513775232732,  0.001011937592673575475411,
    0.0002453010277577173454659, 0.0002834142529941982174005};

// pair p: +e = (PEX[p], PEY[p]) in shell PSH[p]
inline constexpr int PEX[NPAIR] = {1, 0, 1, -1, 2, 0, 2, -2, 1, -1, 2, -2, 3, 0, 3, -3, 1, -1};
inline constexpr int PEY[NPAIR] = {0, 1, 1, 1, 0, 2, 1, 1, 2, 2, 2, 2, 0, 3, 1, 1, 3, 3};
inline constexpr int PSH[NPAIR] = {1, 1, 2, 2, 3, 3, 4, 4, 4, 4, 5, 5, 6, 6, 7, 7, 7, 7};

constexpr int ex_of(int i) { return i == 0 ? 0 : ((i - 1) & 1) ? -PEX[(i - 1) >> 1] : PEX[(i - 1) >> 1]; }
constexpr int ey_of(int i) { return i == 0 ? 0 : ((i - 1) & 1) ? -PEY[(i - 1) >> 1] : PEY[(i - 1) >> 1]; }
constexpr int shell_of(int i) { return i == 0 ? 0 : PSH[(i - 1) >> 1]; }
}  // namespace d2q37

namespace d2q17 {
constexpr int NQ = 17;
constexpr int NPAIR = 8;
constexpr int NSHELL = 5;
constexpr int ORDER = 3;

constexpr double LAT_R = 1.6434306087979541468226542;
constexpr double LAT_R2 = LAT_R * LAT_R;

// shells |e|^2 = 0, 1, 2, 8, 9: rest, axis and diagonal unit velocities, (+-2, +-2) and the
// axis velocities of length 3
inline constexpr int SHELL_E2[NSHELL] = {0, 1, 2, 8, 9};
inline constexpr double SHELL_W[NSHELL] = {
    0.40200514690911262594166439, 0.11615486649778154387403546,
    0.033006353622986913949753826, 7.9078602165918131237133241e-05,
    2.5841454978746755955748610e-04};

inline constexpr int PEX[NPAIR] = {1, 0, 1, -1, 2, -2, 3, 0};
inline constexpr int PEY[NPAIR] = {0, 1, 1, 1, 2, 2, 0, 3};
inline constexpr int PSH[NPAIR] = {1, 1, 2, 2, 3, 3, 4, 4};

constexpr int ex_of(int i) { return i == 0 ? 0 : ((i - 1) & 1) ? -PEX[(i - 1) >> 1] : PEX[(i - 1) >> 1]; }
constexpr int ey_of(int i) { return i == 0 ? 0 : ((i - 1) & 1) ? -PEY[(i - 1) >> 1] : PEY[(i - 1) >> 1]; }
constexpr int shell_of(int i) { return i == 0 ? 0 : PSH[(i - 1) >> 1]; }
}  // namespace d2q17

namespace d2q9 {
constexpr int NQ = 9;
constexpr int NPAIR = 4;
constexpr int NSHELL = 3;
constexpr int ORDER = 2;

constexpr double LAT_R = 1.7320508075688772935274463;   // sqrt(3)
constexpr double LAT_R2 = LAT_R * LAT_R;

// shells |e|^2 = 0, 1, 2: rest, axis and diagonal unit velocities
inline constexpr int SHELL_E2[NSHELL] = {0, 1, 2};
inline constexpr double SHELL_W[NSHELL] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};

inline constexpr int PEX[NPAIR] = {1, 0, 1, -1};
inline constexpr int PEY[NPAIR] = {0, 1, 1, 1};
inline constexpr int PSH[NPAIR] = {1, 1, 2, 2};

constexpr int ex_of(int i) { return i == 0 ? 0 : ((i - 1) & 1) ? -PEX[(i - 1) >> 1] : PEX[(i - 1) >> 1]; }
constexpr int ey_of(int i) { return i == 0 ? 0 : ((i - 1) & 1) ? -PEY[(i - 1) >> 1] : PEY[(i - 1) >> 1]; }
constexpr int shell_of(int i) { return i == 0 ? 0 : PSH[(i - 1) >> 1]; }
}  // namespace d2q9

// Host view of one stencil's tables.
struct LatticeInfo {
    int q, npair, nshell, order;
    double r;
    const int *shell_e2;
    const double *shell_w;
    const int *pex, *pey, *psh;
    int ex(int i) const { return i == 0 ? 0 : ((i - 1) & 1) ? -pex[(i - 1) >> 1] : pex[(i - 1) >> 1]; }
    int ey(int i) const { return i == 0 ? 0 : ((i - 1) & 1) ? -pey[(i - 1) >> 1] : pey[(i - 1) >> 1]; }
    int shell(int i) const { return i == 0 ? 0 : psh[(i - 1) >> 1]; }
};

inline constexpr LatticeInfo LATTICE_D2Q37 = {d2q37::NQ, d2q37::NPAIR, d2q37::NSHELL, d2q37::ORDER,
                                              d2q37::LAT_R, d2q37::SHELL_E2, d2q37::SHELL_W,
                                              d2q37::PEX, d2q37::PEY, d2q37::PSH};
inline constexpr LatticeInfo LATTICE_D2Q17 = {d2q17::NQ, d2q17::NPAIR, d2q17::NSHELL, d2q17::ORDER,
                                              d2q17::LAT_R, d2q17::SHELL_E2, d2q17::SHELL_W,
                                              d2q17::PEX, d2q17::PEY, d2q17::PSH};
inline constexpr LatticeInfo LATTICE_D2Q9 = {d2q9::NQ, d2q9::NPAIR, d2q9::NSHELL, d2q9::ORDER,
                                             d2q9::LAT_R, d2q9::SHELL_E2, d2q9::SHELL_W,
                                             d2q9::PEX, d2q9::PEY, d2q9::PSH};

// The stencil a lattice code (37, 17, 9; 0 = 37) names, or nullptr.
inline const LatticeInfo *lattice_info(int code) {
    return code == 0 || code == 37 ? &LATTICE_D2Q37 : code == 17 ? &LATTICE_D2Q17
                                                    : code == 9 ? &LATTICE_D2Q9 : nullptr;
}

}  // namespace lbm
