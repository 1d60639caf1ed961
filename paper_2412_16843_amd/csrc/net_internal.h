// Internal interface between the solver and the learned-guess network.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/cdi.h"

namespace cdinet {
size_t param_count();
size_t workspace_bytes(int B, int H, int W, bool train);
void forward(cdi_net* n);                       // features -> output, on the net's stream
void backward(cdi_net* n, const float* target); // after forward
void pack_weights_public(cdi_net* n);
float* features(cdi_net* n);                    // FP32 [B][3][H][W]
float* output(cdi_net* n);                      // FP32 [B][H][W]
hipStream_t stream_of(cdi_net* n);
int height(cdi_net* n);
int width(cdi_net* n);
int batch(cdi_net* n);
}  // namespace cdinet
