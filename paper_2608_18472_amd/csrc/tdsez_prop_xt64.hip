// Persistent Crank-Nicolson kernels, FP64 arithmetic, extended variant (absorbing
// potential, extended per-step series, a_Q).  A translation
// unit of its own so that the kernel families compile in parallel.
#include "tdsez_run.hpp"

TDSEZ_DEFINE_XT_LAUNCHER(double, launch_prop_xt64)
