// Learned source-iteration correction (internal declarations).
#pragma once

#include <cstdint>
#include <vector>

#include "internal.hpp"

namespace snsw {

// One 3x3x3 convolution of the network; parameters at w_off (cout x cin x 27)
// and b_off (cout) of the flat parameter vector.
struct NetLayer {
    int cin = 0, cout = 0, stride = 1, act = 1, level_in = 0;
    int64_t w_off = 0, b_off = 0;
};

std::vector<NetLayer> net_layers(const int widths[3]);

// phi_swept += prolong(s * N(x)) for the residual phi_swept - phi_prev of
// problem prob (enqueued on the problem's stream).
void net_apply_correction(snsw_net* net, snsw_problem* prob, const double* phi_prev, double* phi_swept);

}  // namespace snsw
