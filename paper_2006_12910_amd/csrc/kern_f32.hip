// Kernels with populations stored as f32.
#define LBK_ST lbk::ST_F32
#define LBK_GETTER kernels_f32
#include "kernels_st.h"
