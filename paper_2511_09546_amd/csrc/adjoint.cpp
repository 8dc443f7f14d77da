// Backward pass: energy gradient through K unrolled CTMRG iterations.
#include "ipeps_impl.hpp"

namespace ipeps {

double energy_grad(Context& cx, const std::vector<TermSpec>& terms,
                   double* grad_host) {
  (void)cx;
  (void)terms;
  (void)grad_host;
  throw NotImplError("gradient");
}

}  // namespace ipeps
