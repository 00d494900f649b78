// Learned initial guess (placeholder until the network kernels land).
#include "guess.hpp"

namespace pe {

struct LearnedGuess {
  int dummy = 0;
};

void guess_destroy(pe_context* c) {
  delete c->guess;
  c->guess = nullptr;
}
void guess_on_system(pe_context*) {}
bool guess_ready(const pe_context*) { return false; }
void guess_predict(pe_context*, double*) { throw Error(PE_ERR_STATE, "learned guess not available"); }

}  // namespace pe

extern "C" {
pe_status pe_guess_init(pe_context*, uint64_t) { return PE_ERR_STATE; }
pe_status pe_guess_set_types(pe_context*, const int32_t*) { return PE_ERR_STATE; }
pe_status pe_guess_record(pe_context*, const double*) { return PE_ERR_STATE; }
pe_status pe_guess_clear(pe_context*) { return PE_ERR_STATE; }
pe_status pe_guess_train(pe_context*, int32_t, int32_t, double, uint64_t, double*) { return PE_ERR_STATE; }
pe_status pe_guess_predict(pe_context*, double*) { return PE_ERR_STATE; }
pe_status pe_guess_save(const pe_context*, const char*) { return PE_ERR_STATE; }
pe_status pe_guess_load(pe_context*, const char*) { return PE_ERR_STATE; }
pe_status pe_bd_step(pe_context*, double, double, double, uint64_t, uint64_t, double*, double*, double*, double*) {
  return PE_ERR_STATE;
}
}
