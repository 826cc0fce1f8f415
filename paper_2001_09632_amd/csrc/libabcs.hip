// libabcs: MI355X (gfx950) adaptive block compressive sensing.
// Single translation unit: kernels, their __constant__ tables and the host ABI.
#include "abcs.h"
#include "common.hpp"
#include "transform16.hpp"
#include "budget_kernels.hpp"
#include "sense_kernels.hpp"
#include "ida_kernels.hpp"
#include "bm3d_kernels.hpp"
#include "cnn_kernels.hpp"
#include "dncnn_kernels.hpp"
#include "generic_kernels.hpp"
#include "threshold_kernels.hpp"
#include "api.cpp.inc"
