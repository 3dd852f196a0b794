// Persistent Crank-Nicolson kernels, FP64 arithmetic (plain variant).  A translation
// unit of its own so that the kernel families compile in parallel.
#include "tdsez_run.hpp"

TDSEZ_DEFINE_PLAIN_LAUNCHER(double, launch_prop_f64)
