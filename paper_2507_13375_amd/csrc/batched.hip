// Batched form (filled in below the plain form).
#include "la_internal.h"
