// Link derivative kernel (placeholder translation unit; filled in below).
#include "common.hpp"
