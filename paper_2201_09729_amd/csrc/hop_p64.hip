#define DLMA_PREC 0
#include "hop_inst.h"
