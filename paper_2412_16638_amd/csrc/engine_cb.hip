// Instantiations of the LP-solve engine with FP64 arithmetic over FP16 / FP32 storage: the
// compressed-basis Krylov variants (the basis and every Krylov vector stored in the low
// precision, all arithmetic, dot products and updates in FP64).
#include "engine.hpp"

namespace mprk {
Engine* make_engine_cb16() { return new EngineT<half_t, double>(); }
Engine* make_engine_cb32() { return new EngineT<float, double>(); }
}  // namespace mprk
