// Kernels with populations stored as bf16.
#define LBK_ST lbk::ST_BF16
#define LBK_GETTER kernels_bf16
#include "kernels_st.h"
