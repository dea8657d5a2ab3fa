#define DLMA_PREC 2
#include "hop_inst.h"
