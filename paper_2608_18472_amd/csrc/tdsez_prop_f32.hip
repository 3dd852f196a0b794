// Persistent Crank-Nicolson kernels, FP32-refined arithmetic (plain variant).  A translation
// unit of its own so that the kernel families compile in parallel.
#include "tdsez_run.hpp"

TDSEZ_DEFINE_PLAIN_LAUNCHER(float, launch_prop_f32)
