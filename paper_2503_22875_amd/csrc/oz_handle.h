// oz_handle.h -- accessors of the library handle shared by the host sources.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/oz.h"

bool oz_handle_valid(oz_handle_t h);
int oz_handle_use_device(oz_handle_t h);  // makes the handle's device current (OZ_OK / OZ_ERR_HIP)
hipStream_t oz_handle_stream(oz_handle_t h);
int oz_handle_device(oz_handle_t h);
