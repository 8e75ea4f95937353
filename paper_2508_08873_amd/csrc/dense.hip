// dense kernels: filled in below
#include "lrpr_internal.h"
