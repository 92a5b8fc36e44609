// Accessors of the network handle used by the batch coupling
// (hlbm_closure_step).  Internal to the library.
#pragma once

struct hlbm_cnn;

// which = 0: moments buffer, 1: increments buffer; each [4][max_batch][ny nx] floats
float *hlbm_cnn_io(hlbm_cnn *c, int which);
int hlbm_cnn_max_batch(const hlbm_cnn *c);
int hlbm_cnn_ny(const hlbm_cnn *c);
int hlbm_cnn_nx(const hlbm_cnn *c);
// changes whenever values captured into launch arguments (standardisation,
// output clamp) change, so captured graphs can be rebuilt
int hlbm_cnn_version(const hlbm_cnn *c);
