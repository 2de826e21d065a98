// Learned GMRES warm start (per-element MLP): forward, backward and Adam kernels.
#include "internal.h"
