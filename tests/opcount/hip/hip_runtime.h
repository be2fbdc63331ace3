// Host stand-in for the HIP header, used only to compile the point-wise
// numerics of the library as plain host C++ for operation counting.
#pragma once
#include <cmath>
#define __device__
#define __host__
#define __forceinline__ inline
using std::fabs;
using std::fmax;
using std::fmin;
using std::isfinite;
using std::sqrt;
