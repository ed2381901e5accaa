// Storage-type dependent kernels of the fast level set evolution,
// instantiated for __hip_bfloat16 images (see lse_store.h).
#include "lse_store.h"

template struct lse::Store<__hip_bfloat16>;
