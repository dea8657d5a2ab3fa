#define DLMA_PREC 3
#include "hop_inst.h"
