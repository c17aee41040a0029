// fast_144.hip -- the specialised FP32 passes for N = 144 (one translation unit per
// size, so that the sizes compile in parallel).
#include "ns_fast_eval.hpp"

NS_FAST_INSTANTIATE(144)
