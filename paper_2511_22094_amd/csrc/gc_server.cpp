// placeholder translation unit, replaced by the serving loop
#include "gc_runtime.hpp"
