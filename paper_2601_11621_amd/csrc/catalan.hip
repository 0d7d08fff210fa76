// Single translation unit of the gfx950 Catalan library (device code and
// the C ABI), so that the __constant__ tables need no relocatable device code.
#include "common.hpp"
#include "ntt.inc.hip"
#include "small.inc.hip"
#include "fused.inc.hip"
#include "sieve.inc.hip"
#include "ratio.inc.hip"
#include "decimal.inc.hip"
#include "host.inc.hip"
#include "decimal_host.inc.hip"
#include "rates.inc.hip"
