// Translation unit of libesmp2 holding everything but the Sylvester kernels,
// whose instantiations (vv3.hip, vv3b.hip) are compiled as objects of their own.
#include "linalg.hip"
#include "rhs.hip"
#include "sigma.hip"
#include "pcg.hip"
#include "semican.hip"
#include "arrow.hip"
#include "gemv.hip"
#include "adjoint.hip"
#include "export.hip"
#include "topk.hip"
#include "batch.hip"
#include "api.hip"
