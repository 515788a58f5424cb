// Status codes (mirror of bard_status in include/bard.h) for internal sources.
#pragma once

#include "../../include/bard.h"
