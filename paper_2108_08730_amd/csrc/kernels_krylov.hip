// placeholder for the Krylov / multigrid kernels
#include "stencil.h"
