// Device-side description of the networks' Linear layers (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// One Linear layer prepared for the MFMA tile engine.
struct DevLayer {
  int K = 0, N = 0;              // logical fan-in / fan-out
  int nkb = 0, nnt = 0;          // fragment blocks along k, 16-column tiles along n
  const uint4* w = nullptr;      // fragment blocks in the layer's storage precision
  const float* b = nullptr;      // bias, fp32, zero-padded to nnt * 16
  const float* bs = nullptr;     // the bias times 2 log2(e), for tanh epilogues computed from 2^y
  float dq = 1.f;                // dequantisation factor of the products (1 unless FP8)
};

// A layer with a single output, evaluated as a dot product in fp32.
struct DevVec {
  int K = 0;
  const float* w = nullptr;      // [K] fp32
  float b = 0.f;
};

// Storage scales of the interaction network's edge states and node projections.
// FP8 keeps each as E4M3(value * scale) with a per-tensor power-of-two scale chosen
// on the host from a bound on the tensor (so nothing saturates); every other
// precision stores the values themselves (scales 1).
struct GnnScale {
  float e = 1.f, inv_e = 1.f;    // edge states
  float p = 1.f, inv_p = 1.f;    // per-node projections
};

// The interaction network split for the factorised edge updates.
struct DevGNN {
  int H = 0, iters = 0;
  GnnScale sc;
  DevLayer node_enc1, node_enc2;   // [3,H], [H,H]
  DevLayer edge_enc1, edge_enc2;   // [6,H], [H,H]
  DevLayer edge_c;                 // e-block of the first edge-network layer [H,H] (+ its bias)
  DevLayer edge_ab;                // [W1a | W1b]: h_src and h_dst blocks [H, 2H] (no bias)
  DevLayer edge_2;                 // second edge-network layer [H,H]
  DevLayer node_1, node_2;         // node network [2H,H], [H,H]
  DevLayer out_c;                  // e-block of the output head's first layer [H,H] (+ bias)
  DevLayer out_ab;                 // [Wo1a | Wo1b] [H, 2H]
  DevVec out_2;                    // [H] -> 1
};
