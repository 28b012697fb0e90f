// Internal declarations shared by the host translation units of the library.
#pragma once

#include <cstdarg>
#include <cstdint>
#include <vector>

#include "../../include/gbs.h"
#include "bigrat.hpp"

namespace gbs {

// Records a message for gbs_last_error() on this thread and returns status.
int fail(int status, const char* fmt, ...);

int check_steps(int32_t m, const int32_t* steps);
int exact_weights(int32_t p, int32_t m, const int32_t* steps, int32_t n_free,
                  const int32_t* free_idx, const Rational* c_free, std::vector<Rational>& c);
std::vector<Rational> seq_poly(int n);
double isb_of(int k, const int32_t* steps, const std::vector<Rational>& c);
double stencil_sigma(int fd_order);

}  // namespace gbs
