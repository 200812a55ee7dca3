// The library's single device translation unit: the batched kernel shares
// the rank tables (binomials, popcount-ordered masks) built for the layer
// sweep, so both are compiled together.
#include "perm_layers.hip"
#include "perm_layer_c128.hip"
#include "perm_layer_modp.hip"
#include "perm_batch.hip"
#include "perm_ryser.hip"
#include "perm_multi.hip"
#include "perm_probe.hip"
#include "perm_noalloc.hip"
