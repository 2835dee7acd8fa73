// D2Q37 lattice constants of the library (host and device).
//
// The velocity set is the minimal ninth-order Gauss-Hermite rule in 2D with integer
// velocities of maximum displacement 3 and positive weights (paper Sec. 2, "Velocity
// stencils"; weights and scale as published by Philippi et al., PRE 73 (2006) 056702 and
// Shan, PRE 81 (2010) 036702).  Thermal velocities are xi_i = LAT_R e_i (sound-speed unit 1).
//
// Library population order: 0 is the rest velocity; pair p = 0..17 holds +e_p at index
// 1 + 2p and -e_p at index 2 + 2p, so odd/even Hermite parts are shared within a pair.
#pragma once

namespace lbm {

constexpr int NQ = 37;
constexpr int NPAIR = 18;
constexpr int NSHELL = 8;

constexpr double LAT_R = 1.196979770393074358972388;
constexpr double LAT_R2 = LAT_R * LAT_R;

// shell k: |e|^2 and the weight of each of its velocities
constexpr int SHELL_E2[NSHELL] = {0, 1, 2, 4, 5, 8, 9, 10};
constexpr double SHELL_W[NSHELL] = {
    0.2331506691323525022865,    0.1073060915422190024125,
    0.05766785988879488203007,   0.0142082161584507502647,
    0.005353049000513775232732,  0.001011937592673575475411,
    0.0002453010277577173454659, 0.0002834142529941982174005};

// pair p: +e = (PEX[p], PEY[p]) in shell PSH[p]
constexpr int PEX[NPAIR] = {1, 0, 1, -1, 2, 0, 2, -2, 1, -1, 2, -2, 3, 0, 3, -3, 1, -1};
constexpr int PEY[NPAIR] = {0, 1, 1, 1, 0, 2, 1, 1, 2, 2, 2, 2, 0, 3, 1, 1, 3, 3};
constexpr int PSH[NPAIR] = {1, 1, 2, 2, 3, 3, 4, 4, 4, 4, 5, 5, 6, 6, 7, 7, 7, 7};

constexpr int ex_of(int i) { return i == 0 ? 0 : ((i - 1) & 1) ? -PEX[(i - 1) >> 1] : PEX[(i - 1) >> 1]; }
constexpr int ey_of(int i) { return i == 0 ? 0 : ((i - 1) & 1) ? -PEY[(i - 1) >> 1] : PEY[(i - 1) >> 1]; }
constexpr int shell_of(int i) { return i == 0 ? 0 : PSH[(i - 1) >> 1]; }

}  // namespace lbm
