// Block-Jacobi preconditioner: internal interface.
#pragma once

#include "pe_internal.hpp"

namespace pe {

// Inverse of the free-space body saddle block of one shape (double and float).
void build_type_inverse(pe_context* c, BodyType& t);
// z = P^{-1} x over the saddle vector [q; dPsi] (every body's block).
template <typename T>
void precond_apply(hipStream_t s, pe_context* c, const double* x, double* z);

}  // namespace pe
