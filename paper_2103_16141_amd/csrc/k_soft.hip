// Soft spherical assignment kernels (filled in below).
#include "internal.h"
