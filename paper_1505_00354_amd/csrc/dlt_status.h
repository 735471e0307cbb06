#pragma once
// status codes shared by the C-ABI and the host plan code
#define DLT_OK 0
#define DLT_ERR_INVALID_ARG (-1)
#define DLT_ERR_UNSUPPORTED (-2)
#define DLT_ERR_HIP (-3)
#define DLT_ERR_NOMEM (-4)
#define DLT_ERR_NOT_PREPARED (-5)
