// Instantiation of the LP-solve engine for storage half_t, compute float.
#include "engine.hpp"

namespace mprk {
Engine* make_engine_fp16() { return new EngineT<half_t, float>(); }
}  // namespace mprk
