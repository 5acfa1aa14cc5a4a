// Access to a network context from the solver (the learned initial guess).
#pragma once
#include <hip/hip_runtime.h>

#include "sgn.h"

// Grid of the network (H rows of W points).
int sgn_cnn_grid(const sgn_cnn* net, int* H, int* W);
// Staging buffers owned by the network context: input [H][W][3], output [H][W] (FP32).
float* sgn_cnn_in3_buffer(sgn_cnn* net);
float* sgn_cnn_out_buffer(sgn_cnn* net);
// The forward pass on the caller's stream (out = output channel 0, FP32).
int sgn_cnn_forward_on(sgn_cnn* net, const float* in3, float* out, hipStream_t s);
