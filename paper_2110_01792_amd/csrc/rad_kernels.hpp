// Radiation transport and matter-radiation coupling kernels (placeholder).
#pragma once
#include "qk_device.hpp"
