// placeholder: filled in with the Krylov solver
#include "internal.h"
void solver_free(helm27_op* op) { (void)op; }
