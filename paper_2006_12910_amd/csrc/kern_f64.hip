// Kernels with populations stored as f64.
#define LBK_ST lbk::ST_F64
#define LBK_GETTER kernels_f64
#include "kernels_st.h"
