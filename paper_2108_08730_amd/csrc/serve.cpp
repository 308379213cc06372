#include "internal.h"
void helm27_serve_shutdown(helm27_ctx* ctx) { (void)ctx; }
