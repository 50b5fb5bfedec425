// Serving runtime (continuous batching of gate / add / mul / matvec jobs).
#include "runtime.h"
