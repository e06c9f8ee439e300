// rr_inst.hip -- the search kernels (beam, greedy phase, doubling) of one
// data type.  The build compiles this file once per kernel data type, with
// RR_INST set to it (rr_search.h: element type | inner-product bit), so the
// instantiations compile in parallel.

#include "rr_search.h"

#ifndef RR_INST
#error "compile with -DRR_INST=<kernel data type>"
#endif

namespace rr {
RR_DECLARE_BEAM_GREEDY(RR_INST, )
// doubling search runs in exact precision only (no bfloat16 or 8-bit pass)
#if (RR_INST & 7) <= 2
RR_DECLARE_DOUBLING(RR_INST, )
#endif
} // namespace rr
