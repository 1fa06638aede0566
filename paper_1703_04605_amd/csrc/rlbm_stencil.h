// Host-side stencil construction shared by the library's entry points.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "../../include/rlbm.h"
#include "rlbm_tables.h"

// Builds the quadrature and the class table (tab may be NULL); err receives a
// message on failure.  Returns RLBM_OK or a negative RLBM_E* code.
int rlbm_build_table(const rlbm_stencil_desc* d, rlbm_stencil_info* info, RlbmTable* tab, char* err,
                     size_t errlen);
const char* rlbm_global_error();
void rlbm_set_global_error(const char* msg);

// 64-bit FNV-1a fingerprint of the parts of a class table that the fixed-
// stencil kernels compile in (class count, dimension, precision, class
// displacements, float moment and equilibrium rows and their rounding
// remainders, float64 constants).
uint64_t rlbm_table_fingerprint(const RlbmTable* t);

// Chebyshev pieces of the inverse equation of state T(u)/u for mbar = zeta
// (layout of RlbmTable::eos).
void rlbm_build_eos_table(double zeta, double (*out)[RLBM_EOS_DEG]);
