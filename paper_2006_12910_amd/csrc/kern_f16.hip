// Kernels with populations stored as f16.
#define LBK_ST lbk::ST_F16
#define LBK_GETTER kernels_f16
#include "kernels_st.h"
