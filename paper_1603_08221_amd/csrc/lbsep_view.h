// Library-internal view of a channel, shared by the translation units of the
// library (the forward sweep and the adjoint): the problem statement and the
// derived constants the device code needs.
#pragma once

#include <hip/hip_runtime.h>

#include "lbsep.h"
#include "lbsep_device.h"

namespace lbsep {

struct ChannelView {
  lbsep_params p;
  RelaxConsts rc;
  double rho_bc[2][2];  // [inlet, outlet][species] boundary densities of Eq. (rho2)
  hipStream_t stream;
};

// Fills *out from the channel; false if h is NULL.
bool channel_view(const lbsep_channel* h, ChannelView* out);

// Records an error message for lbsep_last_error and returns code.
int set_error(int code, const char* msg);

}  // namespace lbsep
