// Storage-type dependent kernels of the fast level set evolution,
// instantiated for __half images (see lse_store.h).
#include "lse_store.h"

template struct lse::Store<__half>;
