// Learned initial guess: internal interface used by the API unit.
#pragma once

#include "pe_internal.hpp"

namespace pe {

void guess_destroy(pe_context* c);
void guess_on_system(pe_context* c);     // a new configuration was loaded
bool guess_ready(const pe_context* c);   // weights present
void guess_predict(pe_context* c, double* x);  // x[0:n_bead] = projected prediction, x[n_bead:] = 0

}  // namespace pe
