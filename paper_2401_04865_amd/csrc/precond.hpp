// Block-Jacobi preconditioner: internal interface.
#pragma once

#include "pe_internal.hpp"

namespace pe {

// Group bodies into shape types and build (or reuse) each type's inverse.
void precond_setup(pe_context* c);
// z = P^{-1} x over the saddle vector [q; dPsi] (every body's block).
template <typename T>
void precond_apply(hipStream_t s, pe_context* c, const double* x, double* z);

}  // namespace pe
