/* CPU oracle for the L_d norms -- test infrastructure only (tests, smoke check,
 * CPU-baseline leg of the benchmark).  See ld_oracle.c for the definitions. */
#ifndef LD_ORACLE_H
#define LD_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif
int64_t oracle_l1(const int32_t* M, int n, int m, int nthreads);
int64_t oracle_l1_all(const int32_t* M, int n, int m, int nthreads);
int64_t oracle_lmarg(const int32_t* M, int n, int m, int nthreads);
int64_t oracle_ld(const int32_t* M, int n, int m, int d, int nthreads);
int64_t oracle_ld_all(const int32_t* M, int n, int m, int d, int nthreads);
int64_t oracle_range(const int32_t* M, int n, int m, int d, int marg, int q,
                     uint64_t pfx_begin, uint64_t pfx_end, int nthreads);
int64_t oracle_l1_split(const int32_t* M, int n, int m, int marg, int nthreads);
int64_t oracle_ld_split(const int32_t* M, int n, int m, int d, int nthreads);
int64_t oracle_ld_classes(const int32_t* M, int n, int m, int d, int nthreads);
uint64_t oracle_rgs_count(int n, int d);
int64_t oracle_value_of(const int32_t* M, int n, int m, int d, int marg, const int8_t* a);
#ifdef __cplusplus
}
#endif
#endif
