// rr_scan.hip -- dense brute-force range scan (placeholder until the MFMA scan lands)
#include <hip/hip_runtime.h>
#include "rr_internal.h"
