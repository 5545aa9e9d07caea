// Host-side reference: rocRAND's Philox4x32-10 engine (library routine used
// only as an independent check of the oracle's generator).  Reads lines of
// "ctr0 ctr1 ctr2 ctr3 key0 key1" (hex) and prints the four output words.
// The engine's (seed, subsequence, offset) map to key = seed, counter words
// 2-3 = subsequence and words 0-1 = offset/4, so ctr1 must stay below 2^30.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main(){
  unsigned c0,c1,c2,c3,k0,k1;
  while (scanf("%x %x %x %x %x %x",&c0,&c1,&c2,&c3,&k0,&k1)==6){
    unsigned long long seed = ((unsigned long long)k1<<32)|k0;
    unsigned long long sub = ((unsigned long long)c3<<32)|c2;
    unsigned long long off = 4ull*(((unsigned long long)c1<<32)|c0);
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    uint4 r = e.next4();
    printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
  }
}
