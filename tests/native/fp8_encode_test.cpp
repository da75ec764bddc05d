// Reads float32 bit patterns (hex, one per line) on stdin and prints the E4M3
// code host_f2e4m3 gives each, and the power-of-two scale of the whole list.
#include <stdio.h>
#include <string.h>
#include <vector>

#include "../../paper_2501_05520_amd/csrc/host_quant.h"

int main() {
  std::vector<float> v;
  unsigned u;
  while (scanf("%x", &u) == 1) {
    float f;
    memcpy(&f, &u, 4);
    v.push_back(f);
  }
  for (float f : v) printf("%d\n", host_f2e4m3(f));
  printf("scale %.9g\n", fp8_weight_scale(v.data(), v.size()));
  return 0;
}
