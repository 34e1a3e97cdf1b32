/* Stand-in for libaddock's ownership calls, for CPU tests of the Python
 * binding's teardown.  It keeps the contract of include/addock.h: a context
 * owns its batches and pre-screens; ad_destroy detaches the ones still alive;
 * freeing a detached child only deletes the handle.  Any call with a handle
 * that was already freed (or never created) aborts the process, as a
 * use-after-free in the real library would crash it. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#define MAXH 4096
enum { FREE = 0, CTX = 1, BATCH = 2, PRESCREEN = 3 };
static int kind[MAXH];
static int owner[MAXH];   /* child -> context handle index (0: detached) */
static int next_h = 1;

static int take(int k, int own) {
  if (next_h >= MAXH) abort();
  kind[next_h] = k;
  owner[next_h] = own;
  return next_h++;
}
static int idx(void *h, int k) {
  intptr_t i = (intptr_t)h;
  if (i <= 0 || i >= MAXH || kind[i] != k) {
    fprintf(stderr, "stub: bad handle %ld (kind %d)\n", (long)i, k);
    fflush(stderr);
    abort();
  }
  return (int)i;
}

int ad_create(void **out, int device, const void *ff, void *stream) {
  (void)device; (void)ff; (void)stream;
  *out = (void *)(intptr_t)take(CTX, 0);
  return 0;
}
void ad_destroy(void *c) {
  int i = idx(c, CTX);
  for (int h = 1; h < next_h; ++h)
    if ((kind[h] == BATCH || kind[h] == PRESCREEN) && owner[h] == i) owner[h] = 0;
  kind[i] = FREE;
}
const char *ad_last_error(const void *c) { (void)c; return "stub"; }
int stub_new_batch(void *c, void **out) {
  *out = (void *)(intptr_t)take(BATCH, idx(c, CTX));
  return 0;
}
void ad_free_batch(void *b) {
  int i = idx(b, BATCH);
  if (owner[i] && kind[owner[i]] != CTX) abort();   /* attached to a dead context */
  kind[i] = FREE;
}
int ad_prescreen_n_params(void) { return 1; }
int ad_prescreen_create(void *c, const void *cfg, uint64_t seed, void **out) {
  (void)cfg; (void)seed;
  *out = (void *)(intptr_t)take(PRESCREEN, idx(c, CTX));
  return 0;
}
void ad_prescreen_destroy(void *p) {
  int i = idx(p, PRESCREEN);
  if (owner[i] && kind[owner[i]] != CTX) abort();
  kind[i] = FREE;
}
/* handles still allocated (contexts, batches, pre-screens) */
int stub_live(void) {
  int n = 0;
  for (int h = 1; h < next_h; ++h) n += kind[h] != FREE;
  return n;
}
