// Serving entry points (continuous batching); filled in by the serving layer.
#include "internal.hpp"
