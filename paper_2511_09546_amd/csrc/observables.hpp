// Building blocks of the energy network shared by the forward and backward
// passes.
#pragma once

#include "ipeps_impl.hpp"

namespace ipeps {

Tensor site_view(const Context& cx, const Tensor& A, int s);
Tensor open_double_layer(Context& cx, int s);
Tensor rotate_open(Context& cx, const Tensor& ao, int c);
Tensor corner_of(Context& cx, const Env& e, int c, int s, const Tensor& ac);
Tensor site_env(Context& cx, const Env& e, int s);
Tensor term_rdm(Context& cx, const Env& e, const TermSpec& t);

}  // namespace ipeps
