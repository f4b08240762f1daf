// The genome models (paper Sec. 2 Methods: the kernel serves any fixed-length
// genome through three functions, initialize, mutate and evaluate). A model is
// a type with
//   static constexpr bool kString;   // carries the 64-bit string P0, P1
//   static void initialize(Genome&, const Block& draw);  // founders
//   static void mutate(Genome& child, const Block& r, const MutateArgs&);
//   static float evaluate(const Genome&);
// and is compiled into every generation kernel as a template argument, so
// each model gets specialised code. Adding one: its header below and one
// entry in GA_FOR_EACH_MODEL (its id is the value of ga_config.genome_model).
// Included by ga_device.hpp after Block, Genome and MutateArgs.
#pragma once

#include "fitness.hpp"
#include "strings.hpp"
#include "onemax.hpp"
#include "trap4.hpp"

// X(id, type) for every model
#define GA_FOR_EACH_MODEL(X) \
  X(0, FitnessModel)         \
  X(1, OneMaxModel)          \
  X(2, Trap4Model)

namespace ga {

#define GA_COUNT_MODEL(ID, M) +1
constexpr uint32_t kModelCount = 0 GA_FOR_EACH_MODEL(GA_COUNT_MODEL);
#undef GA_COUNT_MODEL

// Whether model `id` carries a string (host and device).
constexpr bool model_has_string(uint32_t id) {
#define GA_STRING_OF(ID, M) if (id == ID) return M::kString;
  GA_FOR_EACH_MODEL(GA_STRING_OF)
#undef GA_STRING_OF
  return false;
}

}  // namespace ga
