// Storage-type dependent kernels of the fast level set evolution,
// instantiated for float images (see lse_store.h).
#include "lse_store.h"

template struct lse::Store<float>;
