// Single translation unit of libesmp2.
#include "linalg.hip"
#include "rhs.hip"
#include "sigma.hip"
#include "vv3.hip"
#include "pcg.hip"
#include "semican.hip"
#include "arrow.hip"
#include "api.hip"
