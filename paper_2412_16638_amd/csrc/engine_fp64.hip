// Instantiation of the LP-solve engine for storage double, compute double.
#include "engine.hpp"

namespace mprk {
Engine* make_engine_fp64() { return new EngineT<double, double>(); }
}  // namespace mprk
