// Time-step pieces: detection, assembly, PDIP and integration.
#pragma once

#include "context.h"
