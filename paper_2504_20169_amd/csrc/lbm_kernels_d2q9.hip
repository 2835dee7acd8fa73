// The step kernels instantiated for the D2Q9 stencil (fifth-order rule, second-order
// equilibrium eq. feq-2): namespace lbm::k9.
#define LBM_Q 9
#include "lbm_kernels.hip"
