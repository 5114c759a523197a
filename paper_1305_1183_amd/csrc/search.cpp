// search.cpp -- plan ranking (filled in with the cost models).
#include "kf_internal.h"
