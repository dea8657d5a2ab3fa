#define DLMA_PREC 1
#include "hop_inst.h"
