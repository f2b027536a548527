// Instantiation of the LP-solve engine for storage float, compute float.
#include "engine.hpp"

namespace mprk {
Engine* make_engine_fp32() { return new EngineT<float, float>(); }
}  // namespace mprk
