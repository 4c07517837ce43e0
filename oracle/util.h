/* Oracle-private helpers.  Test infrastructure only (see oracle.h). */
#ifndef MG_ORACLE_UTIL_H
#define MG_ORACLE_UTIL_H
#include <stdio.h>
#include <stdlib.h>

static inline void *malloc_or_die(size_t bytes)
{
    void *p = calloc(1, bytes ? bytes : 1);
    if (!p) {
        fprintf(stderr, "oracle: out of memory (%zu bytes)\n", bytes);
        abort();
    }
    return p;
}
#endif
