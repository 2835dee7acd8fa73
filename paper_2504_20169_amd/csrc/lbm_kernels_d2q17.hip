// The step kernels instantiated for the D2Q17 stencil (seventh-order rule, third-order
// equilibrium eq. feq-3): namespace lbm::k17.
#define LBM_Q 17
#include "lbm_kernels.hip"
