// QTT compression of the scaled Newton matrix and its approximate inverse.
#include "context.h"

namespace qtp {

void build_inverse(Ctx& c, int hot) {
  (void)hot;
  c.have_inverse = false;
  throw Error(QTP_E_STATE, "QTT inverse construction is not built yet");
}

}  // namespace qtp
